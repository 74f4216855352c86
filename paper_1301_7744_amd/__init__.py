"""Python binding of libsttsm.so: symmetric tensor times same matrix on
MI355X with tensors in Blocked Compact Symmetric Storage (BCSS).

Argument marshalling only.  Every step runs in the library's HIP kernels;
PyTorch supplies device memory and the current stream.  There is no CPU
fallback: without the built library every call raises.

Names follow the C ABI in include/sttsm.h.
"""
from __future__ import annotations

import ctypes
import functools
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsttsm.so")

F32, BF16, F64 = 0, 1, 2
PREC_FP32, PREC_BF16, PREC_BF16X3_FIRST_FP32, PREC_BF16X3_FIRST_BF16 = 0, 1, 2, 3
PREC_NAMES = {"fp32": PREC_FP32, "bf16": PREC_BF16, "bf16x3_fp32": PREC_BF16X3_FIRST_FP32,
              "bf16x3_bf16": PREC_BF16X3_FIRST_BF16}
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EAGAIN", -5: "ENOTFOUND"}


class SttsmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class Layout(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int64), ("b", ctypes.c_int32), ("dtype", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("A", Layout), ("C", Layout), ("A_bcss", ctypes.c_void_p), ("X", ctypes.c_void_p),
                ("rs_x", ctypes.c_int64), ("cs_x", ctypes.c_int64), ("prec", ctypes.c_int32),
                ("src_is_host", ctypes.c_int32)]


QUEUED, ADMITTED, RUNNING, DONE, FAILED = 0, 1, 2, 3, 4


_lib = None


def load():
    """The loaded libsttsm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsttsm.so is not built (run __graft_entry__.build() or "
                          "python paper_1301_7744_amd/build.py); there is no fallback")
    lib = ctypes.CDLL(LIB_PATH)
    L = ctypes.POINTER(Layout)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    sig = {
        "bcss_num_blocks": (i64, [i32, i64]),
        "bcss_num_elems": (i64, [L]),
        "bcss_pack": (ctypes.c_int, [L, vp, vp, vp]),
        "bcss_unpack": (ctypes.c_int, [L, vp, vp, vp]),
        "sttsm_flops": (i64, [L, L]),
        "bcss_fill_hashed": (ctypes.c_int, [L, ctypes.c_uint64, ctypes.c_double, ctypes.c_double, vp, vp]),
        "bcss_symmetrize": (ctypes.c_int, [L, vp, vp]),
        "sttsm_vectors": (ctypes.c_int, [L, vp, vp, i64, i64, vp, i64, vp, vp, sz, vp]),
        "sttsm_vectors_workspace_bytes": (sz, [L, i64]),
        "sttsm_vectors_flops": (i64, [L, i64]),
        "sttsm_workspace_bytes": (sz, [L, L, i32]),
        "sttsm": (ctypes.c_int, [L, vp, vp, i64, i64, L, vp, i32, vp, sz, vp]),
        "sttsm_noalloc": (ctypes.c_int, [L, vp, vp, i64, i64, L, vp, i32, vp]),
        "sttsm_all_but_one": (ctypes.c_int, [L, vp, vp, i64, i64, L, vp, i32, vp, sz, vp]),
        "sttsm_all_but_one_elems": (i64, [L, L, i32]),
        "sttsm_rank_update": (ctypes.c_int, [L, vp, vp, i64, i64, L, vp, i32, i32, vp, sz, vp]),
        "sttsm_rank_update_workspace_bytes": (sz, [L, L, i32, i32]),
        "sttsm_workspace_temp": (ctypes.c_int, [L, L, i32, i32, ctypes.POINTER(sz), ctypes.POINTER(i32),
                                                ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "sttsm_plan_info": (ctypes.c_int, [L, L, i32, i32, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                           ctypes.POINTER(i64), ctypes.POINTER(i32)]),
        "sttsm_profile_enable": (ctypes.c_int, [i32]),
        "sttsm_profile_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), i32,
                                              ctypes.POINTER(i64)]),
        "sttsm_profile_disable": (ctypes.c_int, []),
        "sttsm_request_footprint": (sz, [ctypes.POINTER(Request)]),
        "sttsm_server_create": (ctypes.c_int, [vp, sz, i32, ctypes.POINTER(ctypes.c_void_p)]),
        "sttsm_submit": (ctypes.c_int, [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
        "sttsm_poll": (ctypes.c_int, [vp, ctypes.c_uint64, ctypes.POINTER(i32)]),
        "sttsm_wait": (ctypes.c_int, [vp, ctypes.c_uint64, i64, ctypes.POINTER(i32)]),
        "sttsm_fetch": (ctypes.c_int, [vp, ctypes.c_uint64, vp, i32]),
        "sttsm_server_stats": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64),
                                              ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "sttsm_server_destroy": (ctypes.c_int, [vp]),
        "sttsm_last_error": (ctypes.c_char_p, []),
        "sttsm_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return ["bcss_num_blocks", "bcss_num_elems", "bcss_pack", "bcss_unpack", "bcss_fill_hashed", "bcss_symmetrize",
            "sttsm_flops", "sttsm_vectors", "sttsm_vectors_workspace_bytes", "sttsm_vectors_flops",
            "sttsm_workspace_bytes", "sttsm", "sttsm_noalloc", "sttsm_all_but_one", "sttsm_all_but_one_elems", "sttsm_rank_update",
            "sttsm_rank_update_workspace_bytes", "sttsm_workspace_temp", "sttsm_plan_info", "sttsm_profile_enable",
            "sttsm_profile_read", "sttsm_profile_disable", "sttsm_request_footprint", "sttsm_server_create",
            "sttsm_submit", "sttsm_poll", "sttsm_wait", "sttsm_fetch", "sttsm_server_stats", "sttsm_server_destroy",
            "sttsm_last_error", "sttsm_version"]


def _check(rc: int):
    if rc != 0:
        raise SttsmError(rc, load().sttsm_last_error().decode())


def layout(m: int, n: int, b: int, dtype: int = F32) -> Layout:
    return Layout(int(m), int(n), int(b), int(dtype))


def _torch_dtype_code(t) -> int:
    import torch
    return {torch.float32: F32, torch.bfloat16: BF16, torch.float64: F64}[t.dtype]


def _torch_dtype(code: int):
    import torch
    return {F32: torch.float32, BF16: torch.bfloat16, F64: torch.float64}[code]


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def _ptr(t) -> int:
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


# ------------------------------------------------------------------ queries
def bcss_num_blocks(m: int, nbar: int) -> int:
    return load().bcss_num_blocks(m, nbar)


def bcss_num_elems(m: int, n: int, b: int, dtype: int = F32) -> int:
    return load().bcss_num_elems(ctypes.byref(layout(m, n, b, dtype)))


def sttsm_flops(m: int, n: int, p: int, bA: int, bC: int) -> int:
    return load().sttsm_flops(ctypes.byref(layout(m, n, bA)), ctypes.byref(layout(m, p, bC)))


def sttsm_workspace_bytes(m: int, n: int, p: int, bA: int, bC: int, prec: int = PREC_FP32,
                          dtype: int = F32) -> int:
    return load().sttsm_workspace_bytes(ctypes.byref(layout(m, n, bA, dtype)), ctypes.byref(layout(m, p, bC)), prec)


@functools.lru_cache(maxsize=256)
def _workspace_temp(m, n, p, bA, bC, prec, k, dtype, generic_env):
    # generic_env: the STTSM_GENERIC_KERNELS setting, which changes the plan
    off, dt = ctypes.c_size_t(), ctypes.c_int32()
    nj, npf, blk = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().sttsm_workspace_temp(ctypes.byref(layout(m, n, bA, dtype)), ctypes.byref(layout(m, p, bC)), prec,
                                       k, ctypes.byref(off), ctypes.byref(dt), ctypes.byref(nj),
                                       ctypes.byref(npf), ctypes.byref(blk)))
    return (off.value, dt.value, nj.value, npf.value, blk.value)


def sttsm_workspace_temp(m: int, n: int, p: int, bA: int, bC: int, prec: int, k: int, dtype: int = F32) -> dict:
    """Where T^(k) sits in sttsm's workspace (cached per shape)."""
    off, dt, nj, npf, blk = _workspace_temp(int(m), int(n), int(p), int(bA), int(bC), int(prec), int(k), int(dtype),
                                            os.environ.get("STTSM_GENERIC_KERNELS", ""))
    return dict(byte_offset=off, dtype=dt, num_jtuples=nj, num_prefixes=npf, block_elems=blk)


def sttsm_plan_info(m: int, n: int, p: int, bA: int, bC: int, prec: int, level: int, dtype: int = F32) -> dict:
    g, t, f = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    tile = (ctypes.c_int32 * 5)()
    _check(load().sttsm_plan_info(ctypes.byref(layout(m, n, bA, dtype)), ctypes.byref(layout(m, p, bC)), prec,
                                  level, ctypes.byref(g), ctypes.byref(t), ctypes.byref(f), tile))
    kernel = ("generic", "fp32_block_copy", "bf16_block_copy", "bf16_xres", "bf16_b64")[tile[0]]
    return dict(groups=g.value, tasks=t.value, flops=f.value, kernel=kernel, tile=tuple(tile[1:]))


# ------------------------------------------------------------------ operations
def bcss_pack(dense, m: int, n: int, b: int, out=None, stream=None):
    """Dense device tensor (n^m entries, dimensional order) -> BCSS tensor."""
    import torch
    dt = _torch_dtype_code(dense)
    if dense.numel() != n ** m:
        raise ValueError("dense tensor must hold n^m entries")
    ne = bcss_num_elems(m, n, b, dt)
    if out is None:
        out = torch.empty(ne, dtype=dense.dtype, device=dense.device)
    elif out.numel() < ne or out.dtype != dense.dtype:
        raise ValueError("output too small or of the wrong dtype")
    _check(load().bcss_pack(ctypes.byref(layout(m, n, b, dt)), _ptr(dense), _ptr(out), _stream(stream)))
    return out


def bcss_fill_hashed(m: int, n: int, b: int, seed: int, dtype=None, lo: float = -1.0, hi: float = 1.0, out=None,
                     stream=None, device="cuda"):
    """BCSS tensor of a symmetric pseudo-random tensor (hashed sorted index)."""
    import torch
    tdt = dtype or torch.float32
    dt = {torch.float32: F32, torch.bfloat16: BF16, torch.float64: F64}[tdt]
    ne = bcss_num_elems(m, n, b, dt)
    if out is None:
        out = torch.empty(ne, dtype=tdt, device=device)
    _check(load().bcss_fill_hashed(ctypes.byref(layout(m, n, b, dt)), int(seed) & (2 ** 64 - 1), lo, hi, _ptr(out),
                                   _stream(stream)))
    return out


def bcss_unpack(bcss, m: int, n: int, b: int, out=None, stream=None):
    """BCSS device tensor -> dense (n^m entries, dimensional order)."""
    import torch
    dt = _torch_dtype_code(bcss)
    if bcss.numel() < bcss_num_elems(m, n, b, dt):
        raise ValueError("BCSS tensor too small")
    if out is None:
        out = torch.empty(n ** m, dtype=bcss.dtype, device=bcss.device)
    elif out.numel() < n ** m or out.dtype != bcss.dtype:
        raise ValueError("output too small or of the wrong dtype")
    _check(load().bcss_unpack(ctypes.byref(layout(m, n, b, dt)), _ptr(bcss), _ptr(out), _stream(stream)))
    return out


def sttsm_vectors_flops(m: int, n: int, b: int, V: int) -> int:
    return load().sttsm_vectors_flops(ctypes.byref(layout(m, n, b)), int(V))


def sttsm_vectors(A_bcss, x, m: int, n: int, b: int, y=None, s=None, ws=None, stream=None):
    """y_v = A x_v^(m-1) and s_v = A x_v^m for the rows x_v of x (V x n, A's
    dtype).  Returns (y (V x n fp32), s (V fp32), ws)."""
    import torch
    dt = _torch_dtype_code(A_bcss)
    if x.dtype != A_bcss.dtype or x.dim() != 2 or x.shape[1] != n or x.stride(1) != 1:
        raise ValueError("x must be a (V, n) row-major tensor of A's dtype")
    V = x.shape[0]
    LA = layout(m, n, b, dt)
    if y is None:
        y = torch.empty(V, n, dtype=torch.float32, device=A_bcss.device)
    if s is None:
        s = torch.empty(V, dtype=torch.float32, device=A_bcss.device)
    wsb = load().sttsm_vectors_workspace_bytes(ctypes.byref(LA), V)
    if wsb == 0:
        raise SttsmError(-1, "bad vector-product arguments")
    if ws is None or ws.numel() < wsb:
        ws = torch.empty(wsb, dtype=torch.uint8, device=A_bcss.device)
    _check(load().sttsm_vectors(ctypes.byref(LA), _ptr(A_bcss), x.data_ptr(), V, x.stride(0), y.data_ptr(),
                                y.stride(0), s.data_ptr(), _ptr(ws), ws.numel(), _stream(stream)))
    return y, s, ws


def bcss_symmetrize(bcss, m: int, n: int, b: int, stream=None):
    """Average every entry of each block with repeated block indices over
    the block's stabiliser, in place; returns the tensor."""
    dt = _torch_dtype_code(bcss)
    if bcss.numel() < bcss_num_elems(m, n, b, dt):
        raise ValueError("BCSS tensor too small")
    _check(load().bcss_symmetrize(ctypes.byref(layout(m, n, b, dt)), _ptr(bcss), _stream(stream)))
    return bcss


def sttsm(A_bcss, X, m: int, n: int, p: int, bA: int, bC: int, prec: int = PREC_FP32, C=None, ws=None,
          stream=None):
    """C := [A; X, ..., X] with A and C in BCSS (X is p x n on the device).

    Returns (C, ws); pass both back to reuse their memory."""
    import torch
    dt = _torch_dtype_code(A_bcss)
    if X.dtype != A_bcss.dtype or X.dim() != 2 or tuple(X.shape) != (p, n):
        raise ValueError("X must be a (p, n) tensor of A's dtype")
    LA, LC = layout(m, n, bA, dt), layout(m, p, bC, F32)
    if A_bcss.numel() < bcss_num_elems(m, n, bA, dt):
        raise ValueError("A too small for its layout")
    nc = bcss_num_elems(m, p, bC, F32)
    if C is None:
        C = torch.empty(nc, dtype=torch.float32, device=A_bcss.device)
    elif C.numel() < nc or C.dtype != torch.float32:
        raise ValueError("C too small or not float32")
    wsb = load().sttsm_workspace_bytes(ctypes.byref(LA), ctypes.byref(LC), prec)
    if wsb == 0:
        raise SttsmError(-1, load().sttsm_last_error().decode())
    if ws is None or ws.numel() < wsb:
        ws = torch.empty(wsb, dtype=torch.uint8, device=A_bcss.device)
    _check(load().sttsm(ctypes.byref(LA), _ptr(A_bcss), X.data_ptr(), X.stride(0), X.stride(1),
                        ctypes.byref(LC), _ptr(C), prec, _ptr(ws), ws.numel(), _stream(stream)))
    return C, ws


NOALLOC_SCRATCH_BYTES = 96 << 20


def sttsm_noalloc(A_bcss, X, m: int, n: int, p: int, bA: int, bC: int, C, prec: int = PREC_FP32, stream=None):
    """C := [A; X, ..., X] into the caller's C (float32, BCSS) with no
    workspace: the library's static device scratch array holds the
    temporaries and tables.  Returns C."""
    dt = _torch_dtype_code(A_bcss)
    if X.dtype != A_bcss.dtype or X.dim() != 2 or tuple(X.shape) != (p, n):
        raise ValueError("X must be a (p, n) tensor of A's dtype")
    LA, LC = layout(m, n, bA, dt), layout(m, p, bC, F32)
    if A_bcss.numel() < bcss_num_elems(m, n, bA, dt):
        raise ValueError("A too small for its layout")
    import torch
    if C.numel() < bcss_num_elems(m, p, bC, F32) or C.dtype != torch.float32:
        raise ValueError("C too small or not float32")
    _check(load().sttsm_noalloc(ctypes.byref(LA), _ptr(A_bcss), X.data_ptr(), X.stride(0), X.stride(1),
                                ctypes.byref(LC), _ptr(C), prec, _stream(stream)))
    return C


def sttsm_all_but_one(A_bcss, X, m: int, n: int, p: int, bA: int, bC: int, prec: int = PREC_FP32, T=None,
                      ws=None, stream=None):
    """T := A x_1 X ... x_{m-1} X (every mode but mode 0), laid out as the
    temporary T^(1): a tensor (num_jtuples, nbar, bA * bC^(m-1)) of the
    temporaries' dtype.  Returns (T, ws)."""
    import torch
    dt = _torch_dtype_code(A_bcss)
    if X.dtype != A_bcss.dtype or X.dim() != 2 or tuple(X.shape) != (p, n):
        raise ValueError("X must be a (p, n) tensor of A's dtype")
    LA, LC = layout(m, n, bA, dt), layout(m, p, bC, F32)
    if A_bcss.numel() < bcss_num_elems(m, n, bA, dt):
        raise ValueError("A too small for its layout")
    info = sttsm_workspace_temp(m, n, p, bA, bC, prec, 1, dt)
    ne = load().sttsm_all_but_one_elems(ctypes.byref(LA), ctypes.byref(LC), prec)
    if ne < 0:
        raise SttsmError(-1, load().sttsm_last_error().decode())
    tdt = _torch_dtype(info["dtype"])
    if T is None:
        T = torch.empty(ne, dtype=tdt, device=A_bcss.device)
    elif T.numel() < ne or T.dtype != tdt:
        raise ValueError("T too small or of the wrong dtype")
    wsb = load().sttsm_workspace_bytes(ctypes.byref(LA), ctypes.byref(LC), prec)
    if wsb == 0:
        raise SttsmError(-1, load().sttsm_last_error().decode())
    if ws is None or ws.numel() < wsb:
        ws = torch.empty(wsb, dtype=torch.uint8, device=A_bcss.device)
    _check(load().sttsm_all_but_one(ctypes.byref(LA), _ptr(A_bcss), X.data_ptr(), X.stride(0), X.stride(1),
                                    ctypes.byref(LC), _ptr(T), prec, _ptr(ws), ws.numel(), _stream(stream)))
    return T[:ne].view(info["num_jtuples"], info["num_prefixes"], info["block_elems"]), ws


def sttsm_rank_update_workspace_bytes(m: int, n: int, p: int, bA: int, bC: int, prec: int, rows: int,
                                      dtype: int = F32) -> int:
    LA, LC = layout(m, n, bA, dtype), layout(m, p, bC, F32)
    wsb = load().sttsm_rank_update_workspace_bytes(ctypes.byref(LA), ctypes.byref(LC), prec, rows)
    if wsb == 0:
        raise SttsmError(-1, load().sttsm_last_error().decode())
    return wsb


def sttsm_rank_update(A_bcss, X, m: int, n: int, p: int, bA: int, bC: int, prec: int = PREC_FP32, rows: int = 8,
                      C=None, ws=None, stream=None):
    """C := [A; X, ..., X] by the rank-update form: passes of `rows` block
    rows of A x_1 X ... x_{m-1} X, each added to C as a rank update.
    Returns (C, ws)."""
    import torch
    dt = _torch_dtype_code(A_bcss)
    if X.dtype != A_bcss.dtype or X.dim() != 2 or tuple(X.shape) != (p, n):
        raise ValueError("X must be a (p, n) tensor of A's dtype")
    LA, LC = layout(m, n, bA, dt), layout(m, p, bC, F32)
    if A_bcss.numel() < bcss_num_elems(m, n, bA, dt):
        raise ValueError("A too small for its layout")
    nc = bcss_num_elems(m, p, bC, F32)
    if C is None:
        C = torch.empty(nc, dtype=torch.float32, device=A_bcss.device)
    elif C.numel() < nc or C.dtype != torch.float32:
        raise ValueError("C too small or not float32")
    wsb = load().sttsm_rank_update_workspace_bytes(ctypes.byref(LA), ctypes.byref(LC), prec, rows)
    if wsb == 0:
        raise SttsmError(-1, load().sttsm_last_error().decode())
    if ws is None or ws.numel() < wsb:
        ws = torch.empty(wsb, dtype=torch.uint8, device=A_bcss.device)
    _check(load().sttsm_rank_update(ctypes.byref(LA), _ptr(A_bcss), X.data_ptr(), X.stride(0), X.stride(1),
                                    ctypes.byref(LC), _ptr(C), prec, rows, _ptr(ws), ws.numel(), _stream(stream)))
    return C, ws


def temporary(ws, m: int, n: int, p: int, bA: int, bC: int, prec: int, k: int, dtype: int = F32):
    """View of T^(k) inside a workspace sttsm has filled: a tensor of shape
    (num_jtuples, num_prefixes, block_elems), layout as in the header."""
    info = sttsm_workspace_temp(m, n, p, bA, bC, prec, k, dtype)
    tdt = _torch_dtype(info["dtype"])
    esz = 4 if info["dtype"] == F32 else 2
    count = info["num_jtuples"] * info["num_prefixes"] * info["block_elems"]
    raw = ws[info["byte_offset"]: info["byte_offset"] + count * esz]
    return raw.view(tdt).view(info["num_jtuples"], info["num_prefixes"], info["block_elems"])


def profile_enable(max_launches: int = 4096):
    _check(load().sttsm_profile_enable(max_launches))


def profile_read(max_levels: int = 8):
    """{level: (total_ms, launches)} recorded since enable / the last read."""
    ms = (ctypes.c_double * max_levels)()
    cnt = (ctypes.c_int64 * max_levels)()
    dropped = ctypes.c_int64()
    _check(load().sttsm_profile_read(ms, cnt, max_levels, ctypes.byref(dropped)))
    out = {d: (ms[d], cnt[d]) for d in range(max_levels) if cnt[d]}
    if dropped.value:
        out["dropped"] = dropped.value
    return out


def profile_disable():
    _check(load().sttsm_profile_disable())


# ------------------------------------------------------------------ serving
def make_request(A_bcss, X, m: int, n: int, p: int, bA: int, bC: int, prec: int) -> Request:
    """Request struct for device tensors A (BCSS) and X (p x n, row-major)."""
    dt = _torch_dtype_code(A_bcss)
    if X.dtype != A_bcss.dtype or tuple(X.shape) != (p, n) or X.stride(1) != 1:
        raise ValueError("X must be a row-major (p, n) tensor of A's dtype")
    return Request(layout(m, n, bA, dt), layout(m, p, bC, F32), _ptr(A_bcss), X.data_ptr(), X.stride(0), 1,
                   prec, 0)


def request_footprint(m: int, n: int, p: int, bA: int, bC: int, prec: int, dtype: int = F32) -> int:
    r = Request(layout(m, n, bA, dtype), layout(m, p, bC, F32), 1, 1, n, 1, prec, 0)
    return load().sttsm_request_footprint(ctypes.byref(r))


class Server:
    """Continuous-batching sttsm server over a device arena of arena_bytes
    (the HBM budget), allocated here with PyTorch."""

    def __init__(self, arena_bytes: int, max_inflight: int = 64, device="cuda"):
        import torch
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(load().sttsm_server_create(self.arena.data_ptr(), self.arena.numel(), max_inflight, ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, A_bcss, X, m: int, n: int, p: int, bA: int, bC: int, prec: int) -> int:
        """Queues a request.  Work the caller queued on its current stream
        (for example the kernels that produced A and X) is finished first:
        the server reads the inputs on its own stream."""
        import torch
        req = make_request(A_bcss, X, m, n, p, bA, bC, prec)
        torch.cuda.current_stream().synchronize()
        t = ctypes.c_uint64()
        _check(load().sttsm_submit(self.handle, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = (A_bcss, X, m, p, bC)   # inputs stay alive until fetched
        return t.value

    def poll(self, ticket: int) -> int:
        st = ctypes.c_int32()
        _check(load().sttsm_poll(self.handle, ticket, ctypes.byref(st)))
        return st.value

    def wait(self, ticket: int, timeout_s: float = -1.0) -> int:
        st = ctypes.c_int32()
        rc = load().sttsm_wait(self.handle, ticket, int(timeout_s * 1e6) if timeout_s >= 0 else -1, ctypes.byref(st))
        if rc not in (0, -4):
            _check(rc)
        return st.value

    def fetch(self, ticket: int, out=None):
        import torch
        if ticket not in self._keep:   # unknown or already fetched: the library says which
            _check(load().sttsm_fetch(self.handle, ticket, 1, 0))
        A, X, m, p, bC = self._keep[ticket]
        nc = bcss_num_elems(m, p, bC, F32)
        if out is None:
            out = torch.empty(nc, dtype=torch.float32, device=A.device)
        _check(load().sttsm_fetch(self.handle, ticket, _ptr(out), 0))
        del self._keep[ticket]
        return out

    def stats(self) -> dict:
        p50, p99, rps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        c, r, l = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(load().sttsm_server_stats(self.handle, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(rps),
                                         ctypes.byref(c), ctypes.byref(r), ctypes.byref(l)))
        return dict(p50_us=p50.value, p99_us=p99.value, req_per_s=rps.value, completed=c.value, rounds=r.value,
                    launches=l.value)

    def close(self):
        if self.handle:
            _check(load().sttsm_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version() -> str:
    return load().sttsm_version().decode()

"""The allocation-free entry point sttsm_noalloc, called through the raw C
ABI: the same C as sttsm (same kernels, so bit for bit) on two calls in a
row, the second on a smaller problem, and a problem larger than the static
scratch array rejected with EINVAL before anything is launched."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_util import P32, PBF, PX3F, check_entries, dev_dense, reference, say

pytestmark = pytest.mark.gpu


def st():
    import paper_1301_7744_amd
    return paper_1301_7744_amd


def _problem(m, n, p, bA, bC, seed, bf16=False):
    import torch
    A = synth.symmetric_uniform(m, n, (m, n, seed))
    X = synth.change_of_basis(p, n, (m, n, seed + 1))
    tdt = torch.float32
    if bf16:
        A, X, tdt = synth.round_to_bf16(A), synth.round_to_bf16(X), torch.bfloat16
    Ab = st().bcss_pack(dev_dense(np.asarray(A, np.float32), tdt), m, n, bA)
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(tdt).cuda()
    return A, X, Ab, Xd


def _noalloc_raw(Ab, Xd, m, n, p, bA, bC, prec, dt):
    """sttsm_noalloc through ctypes on the library handle; returns (rc, C)."""
    import torch
    lib = st().load()
    LA, LC = st().layout(m, n, bA, dt), st().layout(m, p, bC, st().F32)
    C = torch.full((st().bcss_num_elems(m, p, bC),), float("nan"), dtype=torch.float32, device="cuda")
    rc = lib.sttsm_noalloc(ctypes.byref(LA), Ab.data_ptr(), Xd.data_ptr(), Xd.stride(0), Xd.stride(1),
                           ctypes.byref(LC), C.data_ptr(), prec, None)
    torch.cuda.synchronize()
    return rc, C


# Two calls in a row, the second smaller, in each precision form.
SEQ = [((3, 256, 256, 16, 16, P32), (3, 35, 20, 16, 8, P32)),
       ((3, 256, 256, 16, 16, PBF), (4, 33, 20, 8, 8, PBF)),
       ((3, 200, 150, 16, 16, PX3F), (2, 70, 65, 64, 64, PX3F))]


@pytest.mark.parametrize("first,second", SEQ)
def test_noalloc_matches_sttsm_twice(first, second):
    import torch
    for (m, n, p, bA, bC, prec) in (first, second):
        say("noalloc", m, n, p, bA, bC, prec)
        bf = prec == PBF
        A, X, Ab, Xd = _problem(m, n, p, bA, bC, 5, bf16=bf)
        dt = st().BF16 if bf else st().F32
        rc, C = _noalloc_raw(Ab, Xd, m, n, p, bA, bC, prec, dt)
        assert rc == 0, st().load().sttsm_last_error()
        Cref, _ = st().sttsm(Ab, Xd, m, n, p, bA, bC, prec)
        torch.cuda.synchronize()
        assert torch.equal(C, Cref)
        nb = st().bcss_num_blocks(m, -(-p // bC))
        got = C.double().cpu().numpy().reshape(nb, bC ** m)
        ref, S = reference(A, X, bC)
        check_entries(got, ref, S, prec, -(-n // bA) * bA)


def test_noalloc_rejects_problems_beyond_the_scratch():
    """m = 3, n = p = 512, b = 16 in FP32 needs about 545 MiB of workspace:
    EINVAL with both sizes in the message, C untouched."""
    import torch
    m, n, p, b = 3, 512, 512, 16
    Ab = torch.zeros(st().bcss_num_elems(m, n, b), dtype=torch.float32, device="cuda")
    Xd = torch.zeros(p, n, dtype=torch.float32, device="cuda")
    rc, C = _noalloc_raw(Ab, Xd, m, n, p, b, b, P32, st().F32)
    assert rc == -1
    msg = st().load().sttsm_last_error().decode()
    assert "static array holds" in msg and str(st().NOALLOC_SCRATCH_BYTES) in msg
    assert torch.isnan(C).all()

"""Seeded synthetic inputs for sttsm workloads.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no blocks, no storage scheme, no mode products).  Both the
GPU path and the FP64 oracle are fed from here, so they see identical values.

Dense tensors are NumPy arrays in Fortran order indexed T[i_0, ..., i_{m-1}];
their memory order is dimensional order (mode 0 fastest).

Workload recipes (the paper's experiments use random FP64 data, §7.1):
  * symmetric A: i.i.d. uniform[-1, 1] on the sorted-index entries, mirrored to
    every permutation of each index;
  * X: i.i.d. N(0, 1) scaled by 1/sqrt(n) (p x n);
  * rank-r symmetric A = sum_i lam_i a_i^{o m}, a_i ~ N(0, I)/sqrt(n),
    lam_i ~ uniform[0.5, 2];
  * a served stream of requests with Poisson arrivals.
"""
from __future__ import annotations

import math

import numpy as np

_CHUNK = 1 << 22


def rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def round_to_bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as
    float32 holding bf16-representable values.  Inputs must be finite."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).reshape(np.shape(x))


def symmetric_uniform(m: int, n: int, seed, dtype=np.float32) -> np.ndarray:
    """Symmetric order-m tensor of extent n: each sorted-index entry drawn
    i.i.d. uniform[-1, 1], every other entry copied from the sorted entry of
    its index.  Values are drawn in float32 (exact in float64)."""
    g = rng(seed)
    total = n ** m
    draws = (g.random(total, dtype=np.float32) * np.float32(2.0) - np.float32(1.0))
    out = np.empty(total, dtype=np.float32)
    powers = np.array([n ** k for k in range(m)], dtype=np.int64)
    for start in range(0, total, _CHUNK):
        flat = np.arange(start, min(total, start + _CHUNK), dtype=np.int64)
        digits = (flat[:, None] // powers[None, :]) % n          # (i_0..i_{m-1})
        digits.sort(axis=1)
        src = digits @ powers                                    # offset of the sorted index
        out[start:start + flat.size] = draws[src]
    out = out.reshape((n,) * m, order="F")
    return out.astype(dtype, copy=False)


def splitmix64(z):
    """SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = (np.asarray(z, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def hashed_symmetric(m: int, n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Symmetric tensor whose entry at sorted index s_0 <= ... <= s_{m-1} is
    lo + (hi - lo) u, u = (h >> 40) 2^-24, h = f(...f(f(seed) ^ s_0)... ^ s_{m-1})
    with f = SplitMix64; float64, Fortran order.  For GPU-side generation of
    large served requests, which fill their compact storage with the same
    definition."""
    total = n ** m
    out = np.empty(total, dtype=np.float64)
    powers = np.array([n ** k for k in range(m)], dtype=np.int64)
    h0 = splitmix64(np.uint64(int(seed) & 0xFFFFFFFFFFFFFFFF))
    for start in range(0, total, _CHUNK):
        flat = np.arange(start, min(total, start + _CHUNK), dtype=np.int64)
        digits = (flat[:, None] // powers[None, :]) % n
        digits.sort(axis=1)
        h = np.full(flat.size, h0, dtype=np.uint64)
        for k in range(m):
            h = splitmix64(h ^ digits[:, k].astype(np.uint64))
        u = (h >> np.uint64(40)).astype(np.float64) * (1.0 / 16777216.0)
        out[start:start + flat.size] = lo + (hi - lo) * u
    return out.reshape((n,) * m, order="F")


def change_of_basis(p: int, n: int, seed, scale=None, dtype=np.float32) -> np.ndarray:
    """X (p x n), i.i.d. N(0,1) times `scale` (default 1/sqrt(n))."""
    g = rng(seed)
    s = 1.0 / math.sqrt(n) if scale is None else scale
    return (g.standard_normal((p, n)) * s).astype(dtype)


def rank_r_factors(n: int, r: int, seed):
    """lam_i ~ U[0.5, 2], a_i ~ N(0, I)/sqrt(n), i = 0..r-1 (float64)."""
    g = rng(seed)
    lams = g.uniform(0.5, 2.0, size=r)
    vecs = g.standard_normal((r, n)) / math.sqrt(n)
    return lams, vecs


def rank_r_symmetric(m: int, lams, vecs) -> np.ndarray:
    """Dense sum_i lam_i a_i^{o m} in float64 (Fortran order)."""
    out = None
    for lam, a in zip(lams, vecs):
        t = np.asarray(a, dtype=np.float64)
        for _ in range(m - 1):
            t = np.multiply.outer(t, a)
        t = lam * t
        out = t if out is None else out + t
    return np.asfortranarray(out)


def served_stream(num_requests: int, seed, rate_per_s: float):
    """Mixed request stream: m uniform in {3, 4}, n uniform in [32, 256],
    p uniform in [16, n], block size 16 when n >= 128 else 8 (bA = bC),
    arrival gaps exponential with the given rate.  Request r's tensor is the
    hashed symmetric tensor of seed 2r + 1 (see hashed_symmetric) and its X is
    drawn with seed (r, 1)."""
    g = rng(seed)
    reqs = []
    t = 0.0
    for r in range(num_requests):
        m = int(g.integers(3, 5))
        n = int(g.integers(32, 257))
        p = int(g.integers(16, n + 1))
        b = 16 if n >= 128 else 8
        t += float(g.exponential(1.0 / rate_per_s)) if rate_per_s > 0 else 0.0
        reqs.append(dict(id=r, m=m, n=n, p=p, b=b, arrival_s=t, seed_a=2 * r + 1, seed_x=(r, 1)))
    return reqs


# Named workloads (the sizes the method is measured and tested on).
CONFIGS = {
    "m3_n16_b4": dict(m=3, n=16, p=16, bA=4, bC=4, seed_a=101, seed_x=102, x_scale=1.0),
    "m3_n256_b16": dict(m=3, n=256, p=256, bA=16, bC=16, seed_a=201, seed_x=202),
    "m2_n4096_b64": dict(m=2, n=4096, p=4096, bA=64, bC=64, seed_a=301, seed_x=302),
    "m4_n64_b8": dict(m=4, n=64, p=64, bA=8, bC=8, seed_a=311, seed_x=312),
    "m5_n32_b4": dict(m=5, n=32, p=32, bA=4, bC=4, seed_a=321, seed_x=322),
    "m6_n24_b4": dict(m=6, n=24, p=24, bA=4, bC=4, seed_a=331, seed_x=332),
}


def rect_cases():
    """m=4, p=32, rank-8 A: n in {128, 130}, bA in {4, 8, 16}, bC in {4, 8}.
    The cases of one n share A and X (seed 401 + n), so the block sizes are
    compared on the same tensor."""
    out = []
    for n in (128, 130):
        for bA in (4, 8, 16):
            for bC in (4, 8):
                out.append(dict(name="m4_n%d_p32_bA%d_bC%d" % (n, bA, bC), m=4, n=n, p=32,
                                bA=bA, bC=bC, rank=8, seed=401 + n))
    return out


def rect_inputs(case):
    """(A, X, lams, vecs) of a rank-r rectangular case: A = sum_i lam_i
    a_i^{o m} rounded to float32, X with seed case seed + 1000."""
    lams, vecs = rank_r_factors(case["n"], case["rank"], case["seed"])
    A = rank_r_symmetric(case["m"], lams, vecs).astype(np.float32)
    X = change_of_basis(case["p"], case["n"], case["seed"] + 1000)
    return A, X, lams, vecs


def workload(name: str) -> dict:
    """Shape of a named workload: a CONFIGS entry or a rect_cases() name."""
    if name in CONFIGS:
        return CONFIGS[name]
    for c in rect_cases():
        if c["name"] == name:
            return c
    raise KeyError("unknown workload %r" % name)


def workload_data(name: str) -> str:
    """How a named workload's inputs are drawn (for reports)."""
    if name in CONFIGS:
        return "synthetic (seeded; symmetric A uniform[-1,1] mirrored from sorted-index entries, X N(0,1)/sqrt(n))"
    return "synthetic (seeded; rank-8 symmetric A = sum lam_i a_i^{o4}, a_i N(0,I)/sqrt(n), lam_i U[0.5,2]; X N(0,1)/sqrt(n))"


def make_config_inputs(name: str):
    """(A, X) float32 dense inputs for a named workload."""
    if name not in CONFIGS:
        A, X, _, _ = rect_inputs(workload(name))
        return A, X
    c = CONFIGS[name]
    A = symmetric_uniform(c["m"], c["n"], c["seed_a"])
    X = change_of_basis(c["p"], c["n"], c["seed_x"], scale=c.get("x_scale"))
    return A, X

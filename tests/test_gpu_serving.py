"""GPU tests of the continuous-batching server: results against the plain
path and the oracle, alone versus in a mix (bit-identical), admission under
a small budget, and ticket misuse."""
import numpy as np
import pytest

import oracle
from oracle import bcss_ref
import synth
from gpu_util import PBF, check_entries, reference, say, tol_bf16

pytestmark = pytest.mark.gpu


def st():
    import paper_1301_7744_amd
    return paper_1301_7744_amd


def make_inputs(m, n, p, b, seed, dtype="bf16"):
    """Device BCSS A and X for one request (bf16-valued inputs)."""
    import torch
    A = synth.round_to_bf16(synth.symmetric_uniform(m, n, (seed, 0)))
    X = synth.round_to_bf16(synth.change_of_basis(p, n, (seed, 1)))
    tdt = torch.bfloat16 if dtype == "bf16" else torch.float32
    Ad = torch.from_numpy(np.ascontiguousarray(A.ravel(order="F"))).to(tdt).cuda()
    Xd = torch.from_numpy(X).to(tdt).cuda()
    Ab = st().bcss_pack(Ad, m, n, b)
    torch.cuda.synchronize()
    return A, X, Ab, Xd


MIX = [(3, 40, 24, 8, 1), (4, 33, 20, 8, 2), (3, 70, 70, 16, 3), (4, 48, 16, 8, 4), (3, 130, 60, 16, 5),
       (4, 36, 36, 8, 6), (3, 35, 17, 8, 7)]


def run_server(reqs, arena_bytes=1 << 30, max_inflight=64):
    import torch
    srv = st().Server(arena_bytes, max_inflight)
    tickets = []
    for (m, n, p, b, seed) in reqs:
        _, _, Ab, Xd = make_inputs(m, n, p, b, seed)
        tickets.append(srv.submit(Ab, Xd, m, n, p, b, b, PBF))
    out = []
    for t in tickets:
        assert srv.wait(t, 60.0) == st().DONE
        out.append(srv.fetch(t).cpu().numpy().astype(np.float64))
    stats = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    return out, stats


def test_served_results_match_plain_path_and_oracle():
    import torch
    got, stats = run_server(MIX)
    say("stats", stats)
    assert stats["completed"] == len(MIX)
    for (m, n, p, b, seed), C in zip(MIX, got):
        A, X, Ab, Xd = make_inputs(m, n, p, b, seed)
        Cp, _ = st().sttsm(Ab, Xd, m, n, p, b, b, PBF)
        torch.cuda.synchronize()
        nb = st().bcss_num_blocks(m, -(-p // b))
        plain = Cp.double().cpu().numpy().reshape(nb, b ** m)
        ref, S = reference(A, X, b)
        e_plain = bcss_ref.rel_frobenius_bcss(C.reshape(nb, -1), plain, m, p, b)
        e_ref = bcss_ref.rel_frobenius_bcss(C.reshape(nb, -1), ref, m, p, b)
        say("  req", (m, n, p, b), "vs plain", e_plain, "vs oracle", e_ref)
        assert e_ref <= tol_bf16(m)
        assert e_plain <= tol_bf16(m)
        check_entries(C.reshape(nb, -1), ref, S, PBF, -(-n // b) * b)
        assert np.array_equal(C.reshape(nb, -1), plain)


def test_alone_equals_mix_bitwise():
    """A request's C is bit-identical alone and inside a mix of others."""
    target = MIX[2]
    alone, _ = run_server([target])
    mixed, _ = run_server(MIX[:2] + [target] + MIX[3:])
    assert np.array_equal(alone[0], mixed[2])


def test_admission_under_small_budget():
    """Budget for about one large request: all still complete, correctly."""
    m, n, p, b = 3, 70, 70, 16
    fp = st().request_footprint(m, n, p, b, b, PBF, st().BF16)
    reqs = [(m, n, p, b, 11 + i) for i in range(4)]
    got, stats = run_server(reqs, arena_bytes=int(fp * 1.5), max_inflight=8)
    ref, _ = run_server(reqs)
    assert stats["completed"] == 4
    for a, r in zip(got, ref):
        assert np.array_equal(a, r)


def test_never_fits_and_ticket_misuse():
    import torch
    m, n, p, b = 3, 70, 70, 16
    fp = st().request_footprint(m, n, p, b, b, PBF, st().BF16)
    srv = st().Server(fp // 2, 4)
    _, _, Ab, Xd = make_inputs(m, n, p, b, 21)
    with pytest.raises(st().SttsmError) as ei:
        srv.submit(Ab, Xd, m, n, p, b, b, PBF)
    assert ei.value.code == -2
    with pytest.raises(st().SttsmError) as ei:
        srv.poll(12345)
    assert ei.value.code == -5
    srv.close()
    srv = st().Server(4 * fp, 4)
    t = srv.submit(Ab, Xd, m, n, p, b, b, PBF)
    assert srv.wait(t, 60.0) == st().DONE
    srv.fetch(t)
    with pytest.raises(st().SttsmError) as ei:
        srv.fetch(t)
    assert ei.value.code == -5
    srv.close()
    torch.cuda.synchronize()


def test_destroy_with_requests_in_flight():
    """Destroying a server with queued and running requests returns cleanly."""
    import torch
    srv = st().Server(1 << 30, 2)
    for (m, n, p, b, seed) in MIX:
        _, _, Ab, Xd = make_inputs(m, n, p, b, seed)
        srv.submit(Ab, Xd, m, n, p, b, b, PBF)
    srv.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("m,n,b,dt", [(3, 9, 4, "f32"), (4, 7, 3, "f32"), (3, 40, 8, "bf16"), (2, 33, 16, "f64")])
def test_hashed_fill_matches_numpy_definition(m, n, b, dt):
    """The GPU's direct BCSS fill equals packing the numpy evaluation of the
    same SplitMix64 definition, bit for bit (served inputs are made this way)."""
    import torch
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f64": torch.float64}[dt]
    got = st().bcss_fill_hashed(m, n, b, seed=12345, dtype=tdt)
    torch.cuda.synchronize()
    A = synth.hashed_symmetric(m, n, 12345)
    if dt == "bf16":
        A = synth.round_to_bf16(A.astype(np.float32)).astype(np.float64)
    elif dt == "f32":
        A = A.astype(np.float32).astype(np.float64)
    ref = bcss_ref.pack(A, b)
    assert np.array_equal(got.to(torch.float64).cpu().numpy().reshape(ref.shape), ref)

"""The seeded input recipes shared by the tests and bench.py (no GPU)."""
import numpy as np
import pytest

import synth
from oracle import closed_forms


def test_named_workloads_resolve():
    for name in synth.CONFIGS:
        assert synth.workload(name) is synth.CONFIGS[name]
    names = [c["name"] for c in synth.rect_cases()]
    assert len(names) == 12 and len(set(names)) == 12
    for c in synth.rect_cases():
        assert synth.workload(c["name"]) == c
    with pytest.raises(KeyError):
        synth.workload("m9_n1_b1")


def test_rect_inputs_are_rank8():
    """rect_inputs' A is the rank-r sum its factors define (checked on one
    entry against the sum over the factors, and for symmetry), and X has
    p rows of n; a small case of the same recipe as the named m=4 cases."""
    case = dict(m=4, n=11, p=5, rank=8, seed=401)
    A, X, lams, vecs = synth.rect_inputs(case)
    assert A.shape == (11,) * 4 and A.dtype == np.float32
    assert X.shape == (5, 11)
    i = (3, 7, 7, 10)
    want = sum(l * v[i[0]] * v[i[1]] * v[i[2]] * v[i[3]] for l, v in zip(lams, vecs))
    assert abs(float(A[i]) - want) <= 1e-6 * max(1.0, abs(want))
    assert A[3, 7, 10, 7] == A[i] and A[10, 7, 3, 7] == A[i]
    C = closed_forms.rank_r(lams, vecs, X.astype(np.float64), 4)
    assert C.shape == (5,) * 4


def test_rect_workload_names_use_rect_inputs(monkeypatch):
    """make_config_inputs of a rectangular name takes its inputs from
    rect_inputs with that case (stubbed here: the full-size tensor is large)."""
    seen = {}

    def stub(case):
        seen["case"] = case
        return "A", "X", None, None
    monkeypatch.setattr(synth, "rect_inputs", stub)
    assert synth.make_config_inputs("m4_n130_p32_bA8_bC4") == ("A", "X")
    assert seen["case"] == synth.workload("m4_n130_p32_bA8_bC4")


def test_workload_data_describes_the_recipe():
    assert "uniform" in synth.workload_data("m3_n256_b16")
    assert "rank-8" in synth.workload_data("m4_n128_p32_bA4_bC4")

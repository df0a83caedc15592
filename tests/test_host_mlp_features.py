"""Host logic of the library: training samples of the learned proposer drawn
from a trace (bs32_mlp_features, no GPU call) against the oracle's samples."""
import math

import numpy as np
import pytest

import workloads
from oracle import mlp
from tests import mlp_cases as mc


@pytest.fixture(scope="module")
def binding():
    import paper_2605_23727_amd as b
    from paper_2605_23727_amd import build
    import os
    if not os.path.exists(b.LIB_PATH):
        build.build()
    return b


def _compare(b, tr, rtol):
    F, Y = b.mlp_features(tr, rtol)
    Fo, Yo = mlp.samples(tr, rtol)
    assert F.shape == Fo.shape
    # the library rounds each value once to FP32
    np.testing.assert_allclose(F, Fo, rtol=2 ** -23, atol=1e-6)
    np.testing.assert_allclose(Y, Yo, rtol=2 ** -23, atol=1e-6)
    return len(F)


def test_features_of_an_oracle_trace(binding, orc):
    w = workloads.kuramoto(24, seed=2101, t1=6.0)
    for rtol in (1e-5, 1e-8):
        _, st, tr = orc.bs32_solve(w["kind"], 24, w["y0"], 0.0, 6.0, rtol, A=w["A"], param=w["param"],
                                   gain=w["gain"], trace_cap=100000)
        assert _compare(binding, tr, rtol) > 20


def test_features_edge_cases(binding):
    rtol = 1e-6
    assert binding.mlp_features(mc.trace([], [], [], []), rtol)[0].shape == (0, 9)
    for n in range(1, 7):   # fewer records than a sample needs
        tr = mc.trace(np.full(n, 0.1), np.full(n, 0.5e-6), np.ones(n), np.ones(n, dtype=int))
        assert _compare(binding, tr, rtol) == max(0, n - 5)
    h = np.full(12, 0.01)
    err = np.full(12, 0.5 * rtol)
    err[5] = 0.0
    err[8] = np.nan
    acc = np.ones(12, dtype=int)
    acc[3] = 0
    tr = mc.trace(h, err, np.exp(np.arange(12.0)), acc)
    _compare(binding, tr, rtol)
    with pytest.raises(Exception):
        binding.mlp_features(tr, 0.0)

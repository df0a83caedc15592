"""Pins of the oracle's clock / cell-cycle model (paper Benchmark 3, eq. (CC),
Sec. 2.1): right-hand sides at points where every term has a closed form
(arctan(+-1) = +-pi/4, X_i2^h with h = 4), the odd pair term, cells that
cannot feel each other, the recipes' all-double reduction, and a solve
against an independent library integrator.
"""
import math

import numpy as np
import pytest
import scipy.integrate

import workloads

K0, K2, K3, A_, B_, C_, EPS = 2.0, 0.144832, 2.0, 2.0, 0.7, 0.8, 0.228249


def _rhs(orc, y, k1, K, I0, A=None):
    n = len(k1)
    return orc.rhs(orc.CLOCK4, n, np.asarray(y, float).reshape(-1), A=A, param=np.asarray(k1, float), gain=K,
                   stimulus=I0).reshape(n, 4)


def test_rhs_closed_form_two_cells(orc):
    # k1 = 2/3 gives theta^h = k1 / (k0 - k1) = 1/2
    k1 = [2.0 / 3.0, 2.0 / 3.0]
    K, I0 = 3.0, 1.5
    y = [[0.0, 0.0, 0.0, 0.0], [1.0, 2.0, 1.5, 0.5]]
    f = _rhs(orc, y, k1, K, I0)
    # cell 0: X_2 = 0, so k0 th / (th + 0) = k0 = 2 and the pair prefactor is k0 a = 4;
    # the pair term with cell 1 is arctan(1 - 0) = pi/4, weighted 1/N = 1/2
    np.testing.assert_allclose(f[0], [2.0 + 0.5 * 4.0 * K * math.pi / 4.0, 0.0, 0.0, EPS * B_], rtol=1e-15,
                               atol=1e-15)
    # cell 1: X_2^4 = 16, k0 th / (th + 16) = 1 / 16.5, prefactor a / 16.5; arctan(0 - 1) = -pi/4
    q = 1.0 / 16.5
    f1 = [q * (A_ * 1.0 + 1.0) - k1[1] * 1.0 + 0.5 * (q * A_) * K * (-math.pi / 4.0),
          K2 * (1.0 - 2.0),
          1.5 * (1.0 - 1.5 ** 2 / 3.0) - 0.5 + I0 * (1.0 - K3 ** 2 / (K3 ** 2 + 1.0)),
          EPS * (1.5 + B_ - C_ * 0.5)]
    np.testing.assert_allclose(f[1], f1, rtol=1e-14, atol=1e-15)


def test_pair_term_is_odd(orc):
    # same k1 and X_2 (same prefactor), uniform weights: the two coupling terms cancel
    k1 = [0.3, 0.3]
    y = [[0.2, 1.1, -1.0, -0.6], [-0.9, 1.1, -1.2, -0.5]]
    f = _rhs(orc, y, k1, K=2.0, I0=0.0)
    f0 = _rhs(orc, y, k1, K=0.0, I0=0.0)
    c = f[:, 0] - f0[:, 0]
    assert c[0] != 0.0 and c[0] == pytest.approx(-c[1], rel=1e-15)
    np.testing.assert_array_equal(f[:, 1:], f0[:, 1:])   # the pair term acts on the first component only


def test_dense_weights_scale_each_pair(orc):
    # with A the pair (i, j) enters with weight A_ij / N
    k1 = [0.35, 0.3, 0.4]
    y = np.array([[0.2, 1.1, -1.0, -0.6], [-0.9, 0.8, -1.2, -0.5], [0.5, 1.3, -1.1, -0.7]])
    A = np.array([[0.0, 2.0, 0.0], [0.0, 0.0, 0.0], [1.0, 1.0, 0.0]])
    f = _rhs(orc, y, k1, K=1.5, I0=0.5, A=A)
    f_uni = _rhs(orc, y, k1, K=1.5, I0=0.5)
    f0 = _rhs(orc, y, k1, K=0.0, I0=0.5)
    c_uni = f_uni[:, 0] - f0[:, 0]
    # cell 0 couples to cell 1 only, twice as strongly; cell 1 is uncoupled
    pre0 = K0 * (0.35 / (K0 - 0.35)) / (0.35 / (K0 - 0.35) + 1.1 ** 4) * A_
    assert f[0, 0] - f0[0, 0] == pytest.approx(2.0 * pre0 * 1.5 * math.atan(-0.9 - 0.2) / 3.0, rel=1e-14)
    assert f[1, 0] == f0[1, 0]
    assert f[2, 0] - f0[2, 0] == pytest.approx(c_uni[2], rel=1e-14)   # row 2 has ones where it matters


def test_identical_cells_do_not_interact(orc):
    n = 5
    w = workloads.clock4(1, seed=71, K=10.0, I0=1.5, t1=20.0)
    y0 = np.tile(w["y0"], n)
    k1 = np.full(n, w["param"][0])
    y, st, _ = orc.bs32_solve(orc.CLOCK4, n, y0, 0.0, 20.0, 1e-8, param=k1, gain=10.0, stimulus=1.5)
    y1, st1, _ = orc.bs32_solve(orc.CLOCK4, 1, w["y0"], 0.0, 20.0, 1e-8, param=k1[:1], gain=0.0, stimulus=1.5)
    assert st["status"] == st1["status"] == 0
    np.testing.assert_allclose(y.reshape(n, 4), np.tile(y1, (n, 1)), rtol=0, atol=1e-12)


def test_solve_matches_library_integrator(orc):
    w = workloads.clock4(3, seed=72, K=1.0, I0=1.5, t1=24.0)
    kw = dict(param=w["param"], gain=w["gain"], stimulus=w["stimulus"])
    y, st, _ = orc.bs32_solve(orc.CLOCK4, 3, w["y0"], 0.0, 24.0, 1e-11, **kw)
    sol = scipy.integrate.solve_ivp(lambda t, x: orc.rhs(orc.CLOCK4, 3, x, **kw), (0.0, 24.0), w["y0"],
                                    method="DOP853", rtol=1e-13, atol=1e-13)
    assert st["status"] == 0 and sol.success
    np.testing.assert_allclose(y, sol.y[:, -1], rtol=0, atol=2e-8)


def test_recipes_reduce_and_round(orc):
    w = workloads.clock4(40, seed=73, K=1.0, I0=1.5, dense=True)
    kw = dict(A=w["A"], param=w["param"], gain=w["gain"], stimulus=w["stimulus"])
    f = orc.rhs(orc.CLOCK4, 40, w["y0"], **kw)
    np.testing.assert_array_equal(orc.rhs_recipe(orc.CLOCK4, 40, w["y0"], 0, 0, 0, **kw), f)
    s = orc.rhs_recipe(orc.CLOCK4, 40, w["y0"], 1, 1, 1, **kw)
    assert np.all(s == s.astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(s, f, rtol=2e-5, atol=2e-5)
    m = orc.rhs_recipe(orc.CLOCK4, 40, w["y0"], 0, 0, 1, **kw)
    np.testing.assert_allclose(m, f, rtol=2e-6, atol=2e-6)
    assert np.max(np.abs(m - f)) > 0.0


def test_no_storage_formats_for_the_arctan_coupling(orc):
    # the reduced storage modes quantize a matrix of a matrix-vector product; the
    # arctan pair term has none, so the oracle refuses them for this model
    w = workloads.clock4(8, seed=74)
    with pytest.raises(ValueError):
        orc.bs32_solve(orc.CLOCK4, 8, w["y0"], 0.0, 1.0, 1e-6, param=w["param"], gain=w["gain"],
                       stimulus=w["stimulus"], mode=orc.PREC_RHS_BF16)


def test_large_populations_keep_theta_positive(orc):
    # k1 is redrawn into (0, k0), so theta^h = k1 / (k0 - k1) > 0 for every cell
    # even where the untruncated normal law would put a few cells below zero
    w = workloads.clock4(16384, seed=6000)
    k1 = w["param"]
    assert np.all(k1 > 0.0) and np.all(k1 < K0)
    assert abs(np.mean(k1) - 0.339278) < 0.005 and abs(np.std(k1) - 0.090909) < 0.005
    f = orc.rhs(orc.CLOCK4, 16384, w["y0"], param=k1, gain=0.0, stimulus=w["stimulus"])
    assert np.all(np.isfinite(f))

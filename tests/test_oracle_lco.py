"""Pins of the oracle's analytic solution of the coupled linear oscillators
(paper Benchmark 1, eq. (LCO), uniform weights) and of the real local error of
eq. (LCO-Local-Error).

The closed form is checked against the matrix exponential of the generator
read off the oracle's own pairwise right-hand side (the system is linear, so
L e_k = f(e_k)), against the one-agent case (a plain rotation), the flow
property, the invariants of the mean and deviation motions, and the order of
the BS3(2) step's true local error.
"""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import lco


def _generator(orc, n):
    """2N x 2N matrix of eq. (LCO) with M_ij = 1/N, one column per unit vector."""
    L = np.zeros((2 * n, 2 * n))
    for k in range(2 * n):
        e = np.zeros(2 * n)
        e[k] = 1.0
        L[:, k] = orc.rhs(orc.LCO_PAPER, n, e)
    return L


@pytest.mark.parametrize("n", [1, 2, 5, 7])
@pytest.mark.parametrize("h", [1e-3, 0.37, 2.0, 11.0])
def test_flow_equals_matrix_exponential(orc, n, h):
    rng = np.random.default_rng(100 + n)
    x = rng.uniform(0.0, 2.0, 2 * n)
    ref = scipy.linalg.expm(h * _generator(orc, n)) @ x
    np.testing.assert_allclose(lco.lco_flow(x, h), ref, rtol=1e-12, atol=1e-13)


def test_one_agent_rotates(orc):
    # N = 1: the coupling term vanishes and (x, v) turns on the unit circle
    x = np.array([0.6, -1.3])
    h = 0.9
    np.testing.assert_allclose(lco.lco_flow(x, h), [0.6 * math.cos(h) - 1.3 * math.sin(h),
                                                     -0.6 * math.sin(h) - 1.3 * math.cos(h)], rtol=1e-15)


def test_flow_property_and_zero_step():
    rng = np.random.default_rng(5)
    x = rng.uniform(0.0, 2.0, 2 * 40)
    np.testing.assert_array_equal(lco.lco_flow(x, 0.0), x)
    np.testing.assert_allclose(lco.lco_flow(lco.lco_flow(x, 0.4), 1.1), lco.lco_flow(x, 1.5), rtol=1e-13,
                               atol=1e-14)


def test_mean_circles_and_deviations_decay():
    rng = np.random.default_rng(6)
    x = rng.uniform(0.0, 2.0, 2 * 50)
    for h in (0.3, 4.0, 17.0):
        y = lco.lco_flow(x, h).reshape(-1, 2)
        X = x.reshape(-1, 2)
        # the means rotate: their squared length is conserved
        assert np.mean(y[:, 0]) ** 2 + np.mean(y[:, 1]) ** 2 == pytest.approx(
            np.mean(X[:, 0]) ** 2 + np.mean(X[:, 1]) ** 2, rel=1e-13)
        # the deviations have zero mean and shrink like e^{-h/2} (times a bounded factor)
        dev = y - y.mean(axis=0)
        assert abs(dev[:, 0].sum()) < 1e-12 and abs(dev[:, 1].sum()) < 1e-12
        dev0 = np.linalg.norm(X - X.mean(axis=0))
        assert np.linalg.norm(dev) <= 2.2 * math.exp(-0.5 * h) * dev0


def test_derivative_at_zero_is_the_right_hand_side(orc):
    rng = np.random.default_rng(7)
    n = 30
    x = rng.uniform(0.0, 2.0, 2 * n)
    f = orc.rhs(orc.LCO_PAPER, n, x)
    h = 1e-5
    fd = (lco.lco_flow(x, h) - lco.lco_flow(x, -h)) / (2 * h)
    np.testing.assert_allclose(fd, f, rtol=0, atol=1e-9)


def test_local_error_definition_on_a_planted_deviation():
    x = np.array([1.0, 0.5, 0.2, 1.5])
    h = 0.25
    ex = lco.lco_flow(x, h)
    bump = np.array([0.0, 3e-7, 0.0, 0.0])
    # max over components of |bump| / max(|X_ex|, delta)
    assert lco.lco_local_error(x, ex + bump, h, 1e-3) == pytest.approx(3e-7 / abs(ex[1]), rel=1e-9)
    # below delta the absolute deviation is divided by delta
    assert lco.lco_local_error(x, ex + bump, h, 1e3) == pytest.approx(3e-10, rel=1e-9)
    assert lco.lco_local_error(x, ex, h, 1e-3) == 0.0


def test_true_local_error_of_a_step_is_fourth_order(orc):
    # one BS3(2) step of the oracle from X: the real local error scales as h^4
    rng = np.random.default_rng(8)
    n = 20
    x = rng.uniform(0.0, 2.0, 2 * n)
    k1 = orc.rhs(orc.LCO_PAPER, n, x)
    errs = []
    for h in (0.04, 0.02, 0.01):
        xn, _, _ = orc.bs32_attempt(orc.LCO_PAPER, n, 0.0, h, x, k1, rtol=1e-6)
        errs.append(lco.lco_local_error(x, xn, h, 1.0))
    for a, b in zip(errs, errs[1:]):
        assert a / b == pytest.approx(16.0, rel=0.06)

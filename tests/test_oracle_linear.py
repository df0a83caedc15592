"""Pins of one BS3(2) step on linear problems (closed forms, Sec. 2.2).

For y' = M y every stage is a polynomial in Z = hM: the third-order solution
is (I + Z + Z^2/2 + Z^3/6) y and the stage-formed difference of the two
solutions is -(Z^3 + Z^4)/48 y.  These polynomials were derived by hand from
the tableau; a wrong coefficient anywhere in the stages, the weights or the
error weights changes them.
"""
import numpy as np
import pytest


def _osc_single(omega):
    # one uncoupled oscillator (N = 1, A = 0): x' = v, v' = -omega^2 x
    return np.array([[0.0, 1.0], [-omega * omega, 0.0]])


@pytest.mark.parametrize("h", [0.3, 0.05, 1e-3])
def test_step_polynomial_oscillator(orc, h):
    w = 1.7
    M = _osc_single(w)
    y0 = np.array([0.8, -0.3])
    K1 = M @ y0
    Xn, K4, err = orc.bs32_attempt(orc.OSC2, 1, 0.0, h, y0, K1, rtol=1e-6, A=np.zeros((1, 1)),
                                   param=np.array([w]))
    Z = h * M
    I = np.eye(2)
    R = I + Z + Z @ Z / 2 + Z @ Z @ Z / 6
    np.testing.assert_allclose(Xn, R @ y0, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(K4, M @ (R @ y0), rtol=1e-14, atol=1e-15)
    Z3 = Z @ Z @ Z
    ev = -(Z3 + Z3 @ Z) / 48 @ y0
    W = np.maximum(np.maximum(np.abs(y0), np.abs(Xn)), 1.0)
    np.testing.assert_allclose(err, np.max(np.abs(ev) / W), rtol=1e-9, atol=1e-18)


def test_step_polynomial_scalar_decay(orc):
    # Kuramoto with one agent is theta' = omega (constant): every stage equals omega,
    # the step is exact and the estimate vanishes (the error weights sum to zero).
    th0 = np.array([0.4])
    w = np.array([1.25])
    Xn, K4, err = orc.bs32_attempt(orc.KURAMOTO, 1, 0.0, 0.5, th0, w, rtol=1e-6, A=np.zeros((1, 1)), param=w)
    assert Xn[0] == pytest.approx(0.4 + 0.5 * 1.25, abs=1e-15)
    assert err < 1e-16


def test_local_error_orders(orc):
    # estimate ~ h^3 and true local error of the third-order solution ~ h^4
    w = 1.0
    M = _osc_single(w)
    y0 = np.array([1.0, 0.0])
    hs = np.array([0.1, 0.05, 0.025, 0.0125])
    ests, loc = [], []
    for h in hs:
        Xn, _, err = orc.bs32_attempt(orc.OSC2, 1, 0.0, h, y0, M @ y0, rtol=1.0, atol=1.0,
                                      A=np.zeros((1, 1)), param=np.array([w]))
        ests.append(err)
        exact = np.array([np.cos(h), -np.sin(h)])
        loc.append(np.max(np.abs(Xn - exact)))
    s_est = np.polyfit(np.log(hs), np.log(ests), 1)[0]
    s_loc = np.polyfit(np.log(hs), np.log(loc), 1)[0]
    assert abs(s_est - 3.0) < 0.1
    assert abs(s_loc - 4.0) < 0.1

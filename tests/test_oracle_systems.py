"""Pins of the oracle's right-hand sides and solves against closed forms,
invariants and hand-computed values (paper Sec. 2.1 and the dense-weight
generalisations of its benchmarks).
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg
import scipy.optimize

import workloads


# ---------------------------------------------------------------- hand values
def test_osc2_hand_values(orc):
    # N = 2, A = [[0, .5], [.5, 0]], omega = (1, 2), x = (1, 3), v = (4, 5)
    # v1' = -1*1 + (1/2)(.5*(3-1)) = -0.5 ; v2' = -4*3 + (1/2)(.5*(1-3)) = -12.5
    y = np.array([1.0, 4.0, 3.0, 5.0])
    f = orc.rhs(orc.OSC2, 2, y, A=[[0, 0.5], [0.5, 0]], param=[1.0, 2.0])
    np.testing.assert_array_equal(f, [4.0, -0.5, 5.0, -12.5])


def test_lco_paper_hand_values(orc):
    # paper eq. (LCO) with uniform weights, N = 3, x = (0, 1, 5), v = (2, 2, 2)
    # x_i' = v_i + mean(x) - x_i = 2 + 2 - x_i ; v_i' = -x_i
    y = np.array([0.0, 2.0, 1.0, 2.0, 5.0, 2.0])
    f = orc.rhs(orc.LCO_PAPER, 3, y)
    np.testing.assert_allclose(f, [4.0, 0.0, 3.0, -1.0, -1.0, -5.0], rtol=0, atol=1e-15)


def test_kuramoto_hand_values(orc):
    # N = 2, theta = (0, pi/2), A = [[0, 1], [.5, 0]], K = 2, omega = (.1, .2)
    # th1' = .1 + (2/2)(1*sin(pi/2)) = 1.1 ; th2' = .2 + (2/2)(.5*sin(-pi/2)) = -.3
    f = orc.rhs(orc.KURAMOTO, 2, [0.0, math.pi / 2], A=[[0, 1], [0.5, 0]], param=[0.1, 0.2], gain=2.0)
    np.testing.assert_allclose(f, [1.1, -0.3], rtol=1e-15, atol=1e-16)


def test_goodwin_hand_values(orc):
    # one agent, (x, y, z) = (.5, 1, 2), b = .2: x' = 1/1025 - .1, y' = .3, z' = .6
    f = orc.rhs(orc.GOODWIN3, 1, [0.5, 1.0, 2.0], A=[[0.0]], param=[0.2], gain=0.5)
    np.testing.assert_allclose(f, [1.0 / 1025.0 - 0.1, 0.3, 0.6], rtol=1e-15)
    # two agents, C = [[0, 1], [.5, 0]], kappa = .5, x = (.5, 1.5), z = (0, 0):
    # x1' = 1 - .2*.5 + (.5/2)(1*(1.5-.5)) = 1.15 ; x2' = 1 - .2*1.5 + (.5/2)(.5*(.5-1.5)) = .575
    y = np.array([0.5, 0.0, 0.0, 1.5, 0.0, 0.0])
    f = orc.rhs(orc.GOODWIN3, 2, y, A=[[0, 1], [0.5, 0]], param=[0.2, 0.2], gain=0.5)
    np.testing.assert_allclose(f[[0, 3]], [1.15, 0.575], rtol=1e-15)


# ------------------------------------------------------------ identities
def test_kuramoto_order_parameter_identity(orc):
    # uniform weights: sum_j sin(th_j - th_i) = N Im(Z e^{-i th_i}), Z = mean e^{i th}
    g = np.random.default_rng(3)
    n = 37
    th = g.random(n) * 20 - 10
    w = g.standard_normal(n)
    K = 1.7
    f = orc.rhs(orc.KURAMOTO, n, th, param=w, gain=K)
    Z = np.mean(np.exp(1j * th))
    np.testing.assert_allclose(f, w + K * np.imag(Z * np.exp(-1j * th)), rtol=0, atol=1e-13)


def test_rows_equal_full(orc):
    for make in (lambda: workloads.kuramoto(40, seed=5), lambda: workloads.osc2(33, seed=6),
                 lambda: workloads.goodwin3(29, seed=7)):
        w = make()
        f = orc.rhs(w["kind"], w["n"], w["y0"], A=w["A"], param=w["param"], gain=w["gain"])
        rows = np.array([0, 3, w["n"] - 1])
        fr = orc.rhs_rows(w["kind"], w["n"], rows, w["y0"], A_rows=w["A"][rows], param=w["param"], gain=w["gain"])
        d = orc.DIM[w["kind"]]
        np.testing.assert_array_equal(fr.reshape(-1, d), f.reshape(-1, d)[rows])


def test_goodwin_fixed_point(orc):
    # identical agents at the steady state x = b^2 z, y = b z, 1/(1+z^10) = b^3 z:
    # every derivative vanishes and the coupling sums are exactly zero.
    b = 0.2
    z = scipy.optimize.brentq(lambda z: 1.0 / (1.0 + z**10) - b**3 * z, 0.1, 5.0, xtol=1e-15)
    n = 9
    y = np.tile([b * b * z, b * z, z], n)
    C = np.random.default_rng(1).random((n, n))
    f = orc.rhs(orc.GOODWIN3, n, y, A=C, param=np.full(n, b), gain=0.5)
    assert np.max(np.abs(f)) < 1e-15
    assert abs(z - 1.549) < 1e-3  # the steady state quoted for the initial values


@pytest.mark.parametrize("kind", [1, 2, 3, 4])
def test_identical_agents_reduce_to_one(orc, kind):
    # equal parameters and initial values: the coupling is exactly zero, so the
    # N-agent solve equals the one-agent solve with the same step sequence.
    n = 6
    d = orc.DIM[kind]
    y1 = {1: [0.7, -0.2], 2: [0.7, -0.2], 3: [0.3], 4: [0.1, 0.4, 1.2]}[kind]
    p = {1: 1.3, 2: 1.0, 3: 0.8, 4: 0.2}[kind]
    A = np.random.default_rng(2).random((n, n))
    yN, stN, _ = orc.bs32_solve(kind, n, np.tile(y1, n), 0.0, 5.0, 1e-7, A=A, param=np.full(n, p), gain=1.5)
    y1s, st1, _ = orc.bs32_solve(kind, 1, np.array(y1), 0.0, 5.0, 1e-7, A=np.zeros((1, 1)), param=[p], gain=1.5)
    assert stN["n_accept"] == st1["n_accept"] and stN["n_reject"] == st1["n_reject"]
    np.testing.assert_allclose(yN.reshape(n, d), np.tile(y1s, (n, 1)), rtol=1e-13, atol=1e-15)


# ----------------------------------------------------------- closed forms
def test_uncoupled_kuramoto_exact(orc):
    n = 50
    g = np.random.default_rng(11)
    th0 = g.random(n) * 6.28
    w = g.standard_normal(n)
    y, st, tr = orc.bs32_solve(orc.KURAMOTO, n, th0, 0.0, 50.0, 1e-8, A=np.zeros((n, n)), param=w,
                               gain=2.0, trace_cap=1000)
    np.testing.assert_allclose(y, th0 + 50.0 * w, rtol=1e-14, atol=1e-12)
    assert st["n_reject"] == 0 and np.all(tr["err"] < 1e-15)
    # E = 0 every step: h grows by facmax until h_max = 0.1*(t1-t0) = 5
    hs = tr["h"]
    assert np.all(hs[1:] <= hs[:-1] * 5.0 * (1 + 1e-15) + 1e-300)
    assert hs[-2] == pytest.approx(5.0)


def test_lco_paper_mode_closed_form(orc):
    # paper eq. (LCO): the mean mode rotates, deviations follow d' = [[-1, 1], [-1, 0]] d
    n = 24
    w = workloads.lco_paper(n, seed=9, t1=3.0)
    T = 3.0
    y, st, _ = orc.bs32_solve(orc.LCO_PAPER, n, w["y0"], 0.0, T, 1e-9)
    X = w["y0"].reshape(n, 2)
    m = X.mean(axis=0)
    D = X - m
    Rm = scipy.linalg.expm(T * np.array([[0.0, 1.0], [-1.0, 0.0]]))
    Rd = scipy.linalg.expm(T * np.array([[-1.0, 1.0], [-1.0, 0.0]]))
    exact = (Rm @ m)[None, :] + D @ Rd.T
    err = np.max(np.abs(y.reshape(n, 2) - exact))
    assert st["status"] == 0 and err < 2e-7


@pytest.mark.parametrize("n", [4, 16, 64])
def test_osc2_eigendecomposition_closed_form(orc, n):
    # x'' = -M x with M = Omega^2 + (1/N)(D - A) symmetric positive definite
    w = workloads.osc2(n, seed=100 + n, t1=5.0)
    A, om = w["A"], w["param"]
    M = np.diag(om**2) + (np.diag(A.sum(axis=1)) - A) / n
    lam, Q = np.linalg.eigh(M)
    assert lam.min() > 0
    s = np.sqrt(lam)
    x0, v0 = w["y0"][0::2], w["y0"][1::2]
    T = 5.0
    a, b = Q.T @ x0, Q.T @ v0
    x_ex = Q @ (np.cos(s * T) * a + np.sin(s * T) / s * b)
    v_ex = Q @ (-s * np.sin(s * T) * a + np.cos(s * T) * b)
    errs = []
    for rtol in (1e-6, 1e-8, 1e-10):
        y, st, _ = orc.bs32_solve(orc.OSC2, n, w["y0"], 0.0, T, rtol, A=A, param=om)
        assert st["status"] == 0
        e = max(np.max(np.abs(y[0::2] - x_ex)), np.max(np.abs(y[1::2] - v_ex)))
        errs.append(e)
        assert e < 200 * rtol
    # tolerance proportionality: two decades of rtol buy more than a decade of error
    assert errs[2] < errs[0] / 30


def test_adler_two_oscillators(orc):
    # N = 2, symmetric weight a: phi = th2 - th1 obeys phi' = dw - K a sin(phi)
    # and th1 + th2 grows linearly.  Time to reach phi = 2 from phi = 0 by quadrature.
    dw, K, a = 2.0, 2.0, 0.5
    kappa = K * a  # (K/N) * a * 2 terms -> K a with N = 2
    T, _ = scipy.integrate.quad(lambda p: 1.0 / (dw - kappa * math.sin(p)), 0.0, 2.0, epsabs=1e-13, epsrel=1e-13, limit=200)
    w = np.array([-dw / 2 + 0.3, dw / 2 + 0.3])
    y, st, _ = orc.bs32_solve(orc.KURAMOTO, 2, np.zeros(2), 0.0, T, 1e-11, A=[[0, a], [a, 0]], param=w, gain=K)
    assert abs((y[1] - y[0]) - 2.0) < 1e-8
    assert abs((y[0] + y[1]) - 0.6 * T) < 1e-9


def test_kuramoto_linear_invariant(orc):
    # symmetric weights: sum_i theta_i - t sum_i omega_i is conserved by any RK method
    n = 30
    g = np.random.default_rng(4)
    U = g.random((n, n))
    A = np.triu(U, 1) + np.triu(U, 1).T
    th0 = g.random(n) * 6.28
    w = g.standard_normal(n)
    y, st, _ = orc.bs32_solve(orc.KURAMOTO, n, th0, 0.0, 10.0, 1e-6, A=A, param=w, gain=3.0)
    assert abs((y.sum() - 10.0 * w.sum()) - th0.sum()) < 1e-11


def test_observed_order_three(orc):
    # fixed steps on OSC2 (N = 4) against the eigendecomposition closed form: slope 3
    n = 4
    w = workloads.osc2(n, seed=77, t1=2.0)
    A, om = w["A"], w["param"]
    M = np.diag(om**2) + (np.diag(A.sum(axis=1)) - A) / n
    lam, Q = np.linalg.eigh(M)
    s = np.sqrt(lam)
    T = 2.0
    a, b = Q.T @ w["y0"][0::2], Q.T @ w["y0"][1::2]
    x_ex = Q @ (np.cos(s * T) * a + np.sin(s * T) / s * b)
    hs = np.array([1 / 8, 1 / 16, 1 / 32, 1 / 64])  # exact in binary: t lands on T
    errs = []
    for h in hs:
        y, st, _ = orc.bs32_solve(orc.OSC2, n, w["y0"], 0.0, T, 1.0, A=A, param=om, fixed_step=True, h0=h)
        assert st["n_accept"] == round(T / h)
        errs.append(np.max(np.abs(y[0::2] - x_ex)))
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert abs(slope - 3.0) < 0.1

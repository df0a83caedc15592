"""Pins of the oracle's adaptive loop: accept rule, counters, failure
conditions (paper Sec. 2.2), FSAL bookkeeping, the reduced-precision and
recipe evaluators' reductions, and DP5(4) against a library integrator.
"""
import math

import numpy as np
import pytest
import scipy.integrate

import workloads


def _kur(n=24, seed=21, K=2.0, t1=5.0):
    return workloads.kuramoto(n, seed=seed, K=K, t1=t1)


def test_accept_rule_and_counts(orc):
    w = _kur()
    y, st, tr = orc.bs32_solve(w["kind"], w["n"], w["y0"], 0.0, 5.0, 1e-7, A=w["A"], param=w["param"],
                               gain=w["gain"], trace_cap=100000)
    assert st["status"] == 0 and st["t_reached"] == 5.0
    acc = tr["accepted"] == 1
    assert np.all(tr["err"][acc] < 1e-7) and np.all(tr["err"][~acc] >= 1e-7)
    assert acc.sum() == st["n_accept"] and (~acc).sum() == st["n_reject"]
    # K1 + starting-step evaluation + three stages per attempt (FSAL reuses K4)
    assert st["n_fev"] == 2 + 3 * (st["n_accept"] + st["n_reject"])
    # accepted steps tile [t0, t1]
    assert abs(tr["h"][acc].sum() - 5.0) < 1e-12
    # a rejection shrinks the step, and the step after a rejection does not grow
    for k in range(len(tr) - 1):
        if not acc[k]:
            assert tr["h"][k + 1] < tr["h"][k]


def test_zero_interval_returns_initial_value(orc):
    w = _kur()
    y, st, _ = orc.bs32_solve(w["kind"], w["n"], w["y0"], 1.0, 1.0, 1e-6, A=w["A"], param=w["param"], gain=2.0)
    np.testing.assert_array_equal(y, w["y0"])
    assert st["n_fev"] == 0 and st["status"] == 0


def test_max_steps(orc):
    w = _kur()
    y, st, _ = orc.bs32_solve(w["kind"], w["n"], w["y0"], 0.0, 5.0, 1e-9, A=w["A"], param=w["param"], gain=2.0,
                              i_max=10)
    assert st["status"] == orc.MAX_STEPS and st["n_accept"] + st["n_reject"] == 11
    assert st["t_reached"] < 5.0


def test_max_rejects(orc):
    # an absurd initial step is rejected until h is small: > 0.85 * i_max rejections
    w = _kur()
    y, st, _ = orc.bs32_solve(w["kind"], w["n"], w["y0"], 0.0, 1e9, 1e-9, A=w["A"], param=w["param"], gain=2.0,
                              i_max=10, h0=1e8, h_max=1e9)
    assert st["status"] == orc.MAX_REJECTS and st["n_reject"] == 9 and st["n_accept"] == 0
    np.testing.assert_array_equal(y, w["y0"])  # the last accepted state is the initial one


def test_nonfinite(orc):
    w = _kur()
    y0 = w["y0"].copy()
    y0[3] = np.nan
    y, st, _ = orc.bs32_solve(w["kind"], w["n"], y0, 0.0, 5.0, 1e-6, A=w["A"], param=w["param"], gain=2.0)
    assert st["status"] == orc.NONFINITE


def test_h_too_small_single(orc):
    # Single stores the solution in FP32; at a tolerance below its resolution
    # the step collapses to h_min = 100 eps_32 (Sec. 2.2 failure condition)
    w = workloads.osc2(8, seed=3, t1=10.0)
    y, st, _ = orc.bs32_solve(w["kind"], 8, w["y0"], 0.0, 10.0, 1e-12, A=w["A"], param=w["param"],
                              mode=orc.PREC_PAPER_SINGLE)
    assert st["status"] == orc.H_TOO_SMALL
    y, st, _ = orc.bs32_solve(w["kind"], 8, w["y0"], 0.0, 10.0, 1e-12, A=w["A"], param=w["param"])
    assert st["status"] == 0


def test_recipe_all_double_equals_definition(orc):
    for w in (_kur(), workloads.osc2(20, seed=4), workloads.goodwin3(15, seed=5), workloads.lco_paper(12)):
        f = orc.rhs(w["kind"], w["n"], w["y0"], A=w["A"], param=w["param"], gain=w["gain"])
        g = orc.rhs_recipe(w["kind"], w["n"], w["y0"], 0, 0, 0, A=w["A"], param=w["param"], gain=w["gain"])
        np.testing.assert_array_equal(f, g)
        s = orc.rhs_recipe(w["kind"], w["n"], w["y0"], 1, 1, 1, A=w["A"], param=w["param"], gain=w["gain"])
        assert np.all(s.astype(np.float32).astype(np.float64) == s)  # single-precision values
        np.testing.assert_allclose(s, f, rtol=1e-5, atol=1e-5 * np.max(np.abs(f)))
        m = orc.rhs_recipe(w["kind"], w["n"], w["y0"], 0, 0, 1, A=w["A"], param=w["param"], gain=w["gain"])
        assert np.max(np.abs(m - f)) <= np.max(np.abs(s - f)) + 1e-12


def test_lowp_with_exact_weights_equals_definition(orc):
    # weights exactly representable in bf16 and a deep split: the matrix-vector
    # rewrite of the reduced-precision evaluator must equal the pairwise sums
    g = np.random.default_rng(7)
    n = 40
    A = g.integers(0, 256, (n, n)) / 256.0
    np.fill_diagonal(A, 0.0)
    for kind, y in ((3, g.random(n) * 6), (1, g.standard_normal(2 * n)), (4, g.random(3 * n))):
        p = g.uniform(0.5, 1.5, n)
        f = orc.rhs(kind, n, y, A=A, param=p, gain=1.3)
        q = orc.rhs_lowp(kind, n, y, 2, A=A, param=p, gain=1.3, split_terms=7, split_shift=8)
        np.testing.assert_allclose(q, f, rtol=0, atol=1e-13)


def test_lowp_storage_error_scales_with_format(orc):
    w = _kur(n=64)
    f = orc.rhs(3, 64, w["y0"], A=w["A"], param=w["param"], gain=2.0)
    errs = []
    for fmt in (1, 3, 2, 4):
        q = orc.rhs_lowp(3, 64, w["y0"], fmt, A=w["A"], param=w["param"], gain=2.0)
        errs.append(np.max(np.abs(q - f)))
    assert errs[0] < 1e-8 < errs[1] < errs[2] < errs[3] < 0.05


def test_dp54_against_library(orc):
    w = _kur(n=8, seed=31, t1=5.0)
    A, om, K, n = w["A"], w["param"], w["gain"], 8

    def f(t, th):
        return orc.rhs(3, n, th, A=A, param=om, gain=K)

    ref = scipy.integrate.solve_ivp(f, (0.0, 5.0), w["y0"], method="DOP853", rtol=1e-13, atol=1e-13).y[:, -1]
    y, st = orc.dp54_solve(3, n, w["y0"], 0.0, 5.0, 1e-11, A=A, param=om, gain=K)
    assert st["status"] == 0
    assert np.max(np.abs(y - ref)) < 1e-9
    # fifth order: two decades of tolerance cost about 10^(2/5) more steps
    _, st2 = orc.dp54_solve(3, n, w["y0"], 0.0, 5.0, 1e-9, A=A, param=om, gain=K)
    ratio = st["n_accept"] / st2["n_accept"]
    assert 1.8 < ratio < 3.5


def test_bs32_steps_scale_as_cube_root(orc):
    w = workloads.osc2(16, seed=8, t1=5.0)
    n_acc = []
    for rtol in (1e-6, 1e-9):
        _, st, _ = orc.bs32_solve(1, 16, w["y0"], 0.0, 5.0, rtol, A=w["A"], param=w["param"])
        n_acc.append(st["n_accept"])
    assert 7.0 < n_acc[1] / n_acc[0] < 14.0  # 10^(3/3) = 10


def test_rkf45_against_library(orc):
    """The oracle's Fehlberg 4(5) solve against scipy's DOP853 at a tight tolerance;
    fourth-order error estimate: two decades of tolerance cost about 10^(2/5) more steps."""
    w = _kur(n=8, seed=32, t1=5.0)
    A, om, K, n = w["A"], w["param"], w["gain"], 8

    def f(t, th):
        return orc.rhs(3, n, th, A=A, param=om, gain=K)

    ref = scipy.integrate.solve_ivp(f, (0.0, 5.0), w["y0"], method="DOP853", rtol=1e-13, atol=1e-13).y[:, -1]
    y, st = orc.rkf45_solve(3, n, w["y0"], 0.0, 5.0, 1e-11, A=A, param=om, gain=K)
    assert st["status"] == 0 and st["t_reached"] == 5.0
    assert np.max(np.abs(y - ref)) < 1e-8
    # every accepted step costs five new stages plus the fresh first stage
    assert st["n_fev"] == 2 + 5 * (st["n_accept"] + st["n_reject"]) + st["n_accept"]
    _, st2 = orc.rkf45_solve(3, n, w["y0"], 0.0, 5.0, 1e-9, A=A, param=om, gain=K)
    ratio = st["n_accept"] / st2["n_accept"]
    assert 1.8 < ratio < 3.5

"""GPU tests of the paper's precision recipes Single, Mixed1 and Mixed2
(Sec. 2.3, Table MP-Distrib) against the oracle's recipes.

The oracle evaluates the recipes on the pairwise definition (each pair term
and its weight rounded to FP32, the sum in the stated precision); the GPU
evaluates the matrix-vector form with A stored FP32 and a one-term FP32 vector
operand.  The two round different intermediate quantities, so parity is
statistical: element-wise within a rounding bound for one evaluation, and
solves whose final errors against an FP64 reference agree in magnitude.
"""
import math
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
# bs32_rhs evaluates the k4 row of a recipe: (F, Sigma, G) single flags
K4_ROW = {5: (1, 1, 1), 6: (0, 0, 1), 7: (0, 0, 1)}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bs():
    import paper_2605_23727_amd as b
    s = b.Solver(0)
    yield b, s
    s.close()


SYSTEMS = [
    ("kuramoto", lambda: workloads.kuramoto(300, seed=61, t1=2.0)),
    ("osc2", lambda: workloads.osc2(257, seed=62, t1=2.0)),
    ("goodwin3", lambda: workloads.goodwin3(130, seed=63, t1=20.0)),
    ("lco", lambda: workloads.lco_paper(200, t1=2.0, dense=True)),
]


@pytest.mark.parametrize("mode", [5, 6, 7])
@pytest.mark.parametrize("name,make", SYSTEMS)
def test_recipe_rhs_matches_oracle(bs, orc, mode, name, make):
    b, s = bs
    w = make()
    n = w["n"]
    say(f"[recipe rhs] {name} n={n} mode={mode}")
    s.set_workload(w)
    f = s.rhs(w["y0"], mode=mode)
    pF, pS, pG = K4_ROW[mode]
    fo = orc.rhs_recipe(w["kind"], n, w["y0"], pF, pS, pG, A=w["A"], param=w["param"], gain=w["gain"])
    fd = orc.rhs(w["kind"], n, w["y0"], A=w["A"], param=w["param"], gain=w["gain"])
    d = b.DIM[w["kind"]]
    A = np.ones((n, n)) if w["A"] is None else w["A"]
    x = w["y0"].reshape(n, d)[:, 0]
    vmax = 1.0 if w["kind"] == b.KURAMOTO else np.max(np.abs(x))
    coup = abs(w["gain"]) / n * np.sum(np.abs(A), axis=1) * vmax * 2.0   # bound on the pair terms' sum
    # summation error of an FP32 sum (N terms) or of FP32 groups, plus the operand and result roundings
    L = 2 * n + 64 if pS else 320
    tol = (U32 * (L * coup[:, None] + 8.0 * (np.abs(fd.reshape(n, d)) + 1.0))).reshape(-1)
    err = np.abs(f - fo)
    assert np.all(err <= tol), (name, mode, float(np.max(err / tol)))
    # a recipe differs from plain FP64 by about its rounding, and not by nothing
    assert np.max(np.abs(f - fd)) <= np.max(tol)
    if pG:
        assert np.max(np.abs(f - fd)) > 0.0


@pytest.mark.parametrize("mode", [5, 6, 7])
@pytest.mark.parametrize("name,make", SYSTEMS[:3])
def test_recipe_solves_track_the_oracle(bs, orc, mode, name, make):
    b, s = bs
    w = make()
    n, t1 = w["n"], w["t1"]
    kw = dict(A=w["A"], param=w["param"], gain=w["gain"])
    rtol = 1e-6
    say(f"[recipe solve] {name} n={n} mode={mode}")
    ref, _, _ = orc.bs32_solve(w["kind"], n, w["y0"], 0.0, t1, 1e-11, **kw)
    s.set_workload(w)
    y, st = s.solve(w["y0"], 0.0, t1, rtol, mode=mode)
    yo, sto, _ = orc.bs32_solve(w["kind"], n, w["y0"], 0.0, t1, rtol, mode=mode, **kw)
    assert st["status"] == 0 and sto["status"] == 0
    e_gpu = np.linalg.norm(y - ref) / math.sqrt(y.size)
    e_orc = np.linalg.norm(yo - ref) / math.sqrt(y.size)
    say(f"   error gpu {e_gpu:.3e} oracle {e_orc:.3e}; accepted {st['n_accept']} / {sto['n_accept']}")
    assert e_gpu <= 10.0 * e_orc + 1e-9 and e_orc <= 10.0 * e_gpu + 1e-9
    assert abs(st["n_accept"] - sto["n_accept"]) <= 0.1 * sto["n_accept"] + 2
    if mode == 5:   # Single keeps its solution in FP32
        assert np.all(y == y.astype(np.float32).astype(np.float64))


def test_mixed2_tracks_double_and_single_plateaus(bs, orc):
    """Mixed2 (every agent term and sum in FP64, pair terms in FP32) stays near
    FP64's error down to tight tolerances, as the oracle's Mixed2 does; Single's
    error stops falling (its state is FP32)."""
    b, s = bs
    w = workloads.kuramoto(300, seed=64, t1=2.0)
    kw = dict(A=w["A"], param=w["param"], gain=w["gain"])
    ref, _, _ = orc.bs32_solve(w["kind"], w["n"], w["y0"], 0.0, 2.0, 1e-12, **kw)
    s.set_workload(w)
    err = {}
    for mode in (0, 5, 7):
        for rtol in (1e-5, 1e-8):
            y, st = s.solve(w["y0"], 0.0, 2.0, rtol, mode=mode)
            assert st["status"] == 0
            err[mode, rtol] = np.linalg.norm(y - ref) / math.sqrt(y.size)
    yo, _, _ = orc.bs32_solve(w["kind"], w["n"], w["y0"], 0.0, 2.0, 1e-8, mode=7, **kw)
    e7o = np.linalg.norm(yo - ref) / math.sqrt(yo.size)
    say(f"[recipes] errors {err}, oracle Mixed2 at 1e-8 {e7o:.3e}")
    assert err[7, 1e-8] <= 5.0 * err[0, 1e-8] + 1e-12
    assert err[7, 1e-8] <= 10.0 * e7o + 1e-12
    assert err[5, 1e-8] > 10.0 * err[0, 1e-8]
    assert err[5, 1e-8] > 0.1 * err[5, 1e-5]


def test_single_h_too_small_matches_oracle(bs, orc):
    b, s = bs
    w = workloads.osc2(8, seed=3, t1=10.0)
    s.set_workload(w)
    _, st = s.solve(w["y0"], 0.0, 10.0, 1e-12, mode=5)
    _, sto, _ = orc.bs32_solve(w["kind"], 8, w["y0"], 0.0, 10.0, 1e-12, A=w["A"], param=w["param"],
                               mode=orc.PREC_PAPER_SINGLE)
    assert st["status"] == sto["status"] == b.H_TOO_SMALL


def test_recipes_not_in_ensembles(bs):
    b, s = bs
    ws = [workloads.kuramoto(64, seed=65 + q, t1=1.0) for q in range(2)]
    s.set_ensemble(ws)
    with pytest.raises(b.BS32Error):
        s.solve_batch(np.concatenate([w["y0"] for w in ws]), 0.0, 1.0, 1e-6, mode=6)


@pytest.mark.parametrize("mode", [5, 6, 7])
def test_recipe_rows_per_stage(bs, orc, mode):
    """Each stage of an attempt uses its own row of Table MP-Distrib.  Without coupling
    (K = 0) the Kuramoto right-hand side is omega, so the stages differ only in how F
    rounds it: FP64 rows give omega, single rows (float)omega, and the error estimate
    of the first attempt h |sum (b_l - bt_l) K_l| depends on which stages are single
    (for Mixed1, k4 in FP64 against k4 in FP32 changes it by a factor 2.8)."""
    b, s = bs
    w = workloads.kuramoto(64, seed=66, K=0.0, t1=1.0)
    s.set_workload(w)
    s.set_options(trace=1, trace_cap=1024, h0=0.01)
    try:
        _, st = s.solve(w["y0"], 0.0, 1.0, 1e-6, mode=mode)
        tr = s.trace()
    finally:
        s.set_options(trace=0, h0=0.0)
    _, sto, tro = orc.bs32_solve(w["kind"], 64, w["y0"], 0.0, 1.0, 1e-6, A=w["A"], param=w["param"], gain=0.0,
                                 mode=mode, trace_cap=1024, h0=0.01)
    assert st["status"] == 0 and sto["status"] == 0
    e_gpu, e_orc = tr["err"][0], tro["err"][0]
    say(f"[recipe rows] mode {mode}: first estimate {e_gpu:.6e} vs oracle {e_orc:.6e}")
    assert abs(e_gpu - e_orc) <= 1e-6 * e_orc + 1e-300

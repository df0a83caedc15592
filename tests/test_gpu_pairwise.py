"""GPU tests of the pairwise couplings (the paper's own form of its benchmarks,
Sec. 2.1): the clock / cell-cycle model of eq. (CC) with its arctan pair term,
and Kuramoto evaluated as K sin(th_j - th_i) pair by pair.

FP64: element-wise against the oracle's pairwise definition and solves at the
parity bar.  The recipes (G in single): element-wise within an FP32 rounding
bound of the oracle's pairwise recipe, solves at matched error magnitude.
"""
import math
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
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


def _kur_pair(n, seed, dense=True, t1=2.0):
    w = workloads.kuramoto(n, seed=seed, t1=t1)
    if not dense:
        w["A"] = None
    w["pairwise"] = True
    return w


CASES = [
    ("clock-uniform", lambda n: workloads.clock4(n, seed=80 + n, K=1.0, I0=1.5)),
    ("clock-dense", lambda n: workloads.clock4(n, seed=81 + n, K=10.0, I0=0.228249, dense=True)),
    ("kuramoto-uniform", lambda n: _kur_pair(n, 82 + n, dense=False)),
    ("kuramoto-dense", lambda n: _kur_pair(n, 83 + n)),
]


def _orc_kw(w):
    return dict(A=w["A"], param=w["param"], gain=w["gain"], stimulus=w.get("stimulus", 0.0))


def _coupling_scale(b, w):
    """Bound on the coupling sum of each row: |K| max|prefactor| (pi/2 or 1) sum_j |A_ij| / N."""
    n = w["n"]
    rows = np.full(n, float(n)) if w["A"] is None else np.sum(np.abs(w["A"]), axis=1)
    if w["kind"] == b.CLOCK4:
        k1 = w["param"]
        th = k1 / (2.0 - k1)
        pre = 2.0 * 2.0 * th / th  # k0 a at X_2 = 0 bounds the prefactor from above
        return abs(w["gain"]) * pre * (math.pi / 2) * rows / n
    return abs(w["gain"]) * rows / n


@pytest.mark.parametrize("n", [1, 5, 300, 1000])
@pytest.mark.parametrize("name,make", CASES)
def test_pair_rhs_fp64_matches_oracle(bs, orc, name, make, n):
    b, s = bs
    w = make(n)
    say(f"[pair rhs fp64] {name} n={n}")
    s.set_workload(w)
    f = s.rhs(w["y0"])
    fo = orc.rhs(w["kind"], n, w["y0"], **_orc_kw(w))
    d = b.DIM[w["kind"]]
    tol = 1e-14 * (_coupling_scale(b, w)[:, None] + np.abs(fo.reshape(n, d)) + 1.0)
    err = np.abs(f - fo).reshape(n, d)
    assert np.all(err <= tol), (name, n, float(np.max(err / tol)))


@pytest.mark.parametrize("name,make", CASES)
def test_pair_every_tile(bs, orc, name, make):
    b, s = bs
    w = make(257)
    s.set_workload(w)
    fo = orc.rhs(w["kind"], 257, w["y0"], **_orc_kw(w))
    tol = 1e-14 * (_coupling_scale(b, w)[:, None] + np.abs(fo.reshape(257, -1)) + 1.0)
    try:
        for tile in range(4):
            s.set_options(tile=tile)
            f = s.rhs(w["y0"])
            assert np.all(np.abs(f - fo).reshape(257, -1) <= tol), (name, tile)
            assert s.kernel_name(0, tile).startswith("k_contract_pair<")
    finally:
        s.set_options(tile=-1)


@pytest.mark.parametrize("name,make,t1,rtol", [
    ("clock-uniform", lambda: workloads.clock4(200, seed=90, K=1.0, I0=1.5), 24.0, 1e-7),
    ("clock-dense", lambda: workloads.clock4(130, seed=91, K=10.0, I0=10.0, dense=True), 12.0, 1e-7),
    ("kuramoto-dense", lambda: _kur_pair(300, 92), 2.0, 1e-8),
])
def test_pair_solve_fp64_matches_oracle(bs, orc, name, make, t1, rtol):
    b, s = bs
    w = make()
    say(f"[pair solve fp64] {name} n={w['n']}")
    s.set_workload(w)
    y, st = s.solve(w["y0"], 0.0, t1, rtol)
    yo, sto, _ = orc.bs32_solve(w["kind"], w["n"], w["y0"], 0.0, t1, rtol, **_orc_kw(w))
    assert st["status"] == 0 and sto["status"] == 0
    rel = np.linalg.norm(y - yo) / np.linalg.norm(yo)
    say(f"   rel {rel:.2e}, accepted {st['n_accept']} / {sto['n_accept']}")
    assert rel <= 1e-10
    assert abs(st["n_accept"] - sto["n_accept"]) <= max(1, 0.01 * sto["n_accept"])


def test_pairwise_kuramoto_equals_matrix_vector_form(bs):
    """The pairwise evaluation and the sin/cos identity of the matrix-vector path
    are the same function: FP64 solves agree to rounding."""
    b, s = bs
    w = workloads.kuramoto(400, seed=93, t1=2.0)
    s.set_workload(w)
    y_mv, st_mv = s.solve(w["y0"], 0.0, 2.0, 1e-8)
    w["pairwise"] = True
    s.set_workload(w)
    y_pw, st_pw = s.solve(w["y0"], 0.0, 2.0, 1e-8)
    assert np.linalg.norm(y_pw - y_mv) / np.linalg.norm(y_mv) <= 1e-10
    assert abs(st_pw["n_accept"] - st_mv["n_accept"]) <= 1


@pytest.mark.parametrize("mode", [5, 6, 7])
@pytest.mark.parametrize("name,make", CASES)
def test_pair_recipe_rhs_matches_oracle(bs, orc, mode, name, make):
    b, s = bs
    n = 300
    w = make(n)
    s.set_workload(w)
    f = s.rhs(w["y0"], mode=mode)
    pF, pS, pG = K4_ROW[mode]
    fo = orc.rhs_recipe(w["kind"], n, w["y0"], pF, pS, pG, **_orc_kw(w))
    fd = orc.rhs(w["kind"], n, w["y0"], **_orc_kw(w))
    d = b.DIM[w["kind"]]
    L = 2 * n + 64 if pS else 64
    tol = (U32 * (L * _coupling_scale(b, w)[:, None] + 16.0 * (np.abs(fd.reshape(n, d)) + 1.0))).reshape(-1)
    err = np.abs(f - fo)
    assert np.all(err <= tol), (name, mode, float(np.max(err / tol)))
    assert np.max(np.abs(f - fd)) > 0.0   # the pair terms really are single


@pytest.mark.parametrize("mode", [5, 6, 7])
def test_pair_recipe_solves_track_the_oracle(bs, orc, mode):
    b, s = bs
    w = workloads.clock4(150, seed=94, K=1.0, I0=1.5, t1=24.0)
    kw = _orc_kw(w)
    ref, _, _ = orc.bs32_solve(w["kind"], 150, w["y0"], 0.0, 24.0, 1e-11, **kw)
    s.set_workload(w)
    y, st = s.solve(w["y0"], 0.0, 24.0, 1e-6, mode=mode)
    yo, sto, _ = orc.bs32_solve(w["kind"], 150, w["y0"], 0.0, 24.0, 1e-6, mode=mode, **kw)
    assert st["status"] == 0 and sto["status"] == 0
    e_gpu = np.linalg.norm(y - ref) / math.sqrt(y.size)
    e_orc = np.linalg.norm(yo - ref) / math.sqrt(y.size)
    say(f"[pair recipe solve] mode {mode}: error gpu {e_gpu:.3e} oracle {e_orc:.3e}")
    assert e_gpu <= 10.0 * e_orc + 1e-9 and e_orc <= 10.0 * e_gpu + 1e-9
    assert abs(st["n_accept"] - sto["n_accept"]) <= 0.1 * sto["n_accept"] + 2


def test_pairwise_limits(bs):
    b, s = bs
    w = workloads.clock4(64, seed=95)
    s.set_workload(w)
    for mode in (1, 2, 3, 4):
        with pytest.raises(b.BS32Error):
            s.solve(w["y0"], 0.0, 1.0, 1e-6, mode=mode)
    with pytest.raises(b.BS32Error):   # uniform weights: no stored matrix
        s.packed_coupling(0)
    with pytest.raises(b.BS32Error):
        s.set_ensemble([w, workloads.clock4(32, seed=96)])
    y, st = s.solve(w["y0"], 0.0, 1.0, 1e-6)   # the context still works
    assert st["status"] == 0

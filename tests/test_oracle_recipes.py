"""Pins of the oracle's precision recipes (paper Sec. 2.3, Table MP-Distrib).

* The recipe table the integrator uses equals the paper's table, transcribed in
  ``tests/golden/mp_recipes.txt``.
* Each table row serves the stage it names: one fixed-step attempt of every
  recipe equals the attempt composed by hand from single evaluations with the
  fixture's flags (and differs when a row is swapped).
* Every single-precision branch of ``orc_rhs_recipe`` is pinned by values
  derived by hand: the inputs are chosen so that every rounding is known in
  closed form (powers of two, 1/3, sums that tie in FP32), so a flipped flag,
  a weight left in FP64, an FP64 sum where the recipe says single, a missing
  gain or an eq. (CC) prefactor in the wrong precision changes an expected bit
  pattern.  Notation: e = 2^-30; f32(1/3) = 11184811 * 2^-25 (0x3EAAAAAB);
  f64(1/3) = 6004799503160661 * 2^-54.
"""
import itertools
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mp_recipes.txt")
E = 2.0 ** -30
COMBOS = list(itertools.product((0, 1), repeat=3))  # (pF, pS, pG)


def _golden():
    t = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#")[0].split()
            if not line:
                continue
            solver, stage, *flags = line
            t[(solver, stage)] = tuple(1 if v == "S" else 0 for v in flags)
    return t


def _rne(x, p):
    """Round a rational to p significant bits, ties to even (normal range)."""
    x = Fr(x)
    if x == 0:
        return x
    s = -1 if x < 0 else 1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fr(2) ** e > a:
        e -= 1
    q = a / Fr(2) ** (e - p + 1)
    n = q.numerator // q.denominator
    r = q - n
    if r > Fr(1, 2) or (r == Fr(1, 2) and n % 2 == 1):
        n += 1
    return s * n * Fr(2) ** (e - p + 1)


def f32(x):
    return _rne(x, 24)


def f64(x):
    return _rne(x, 53)


def test_rne_helper_on_known_values():
    assert f32(Fr(1, 3)) == Fr(11184811, 2 ** 25)
    assert f64(Fr(1, 3)) == Fr(6004799503160661, 2 ** 54)
    assert f32(1 + Fr(1, 2 ** 24)) == 1            # a tie rounds to the even neighbour
    assert f32(1 + Fr(3, 2 ** 24)) == 1 + Fr(1, 2 ** 22)
    assert float(f64(Fr(1, 10))) == 0.1


# ---------------------------------------------------------------------------
# the table and the stage each row serves
# ---------------------------------------------------------------------------
def test_recipe_table_matches_the_paper(orc):
    g = _golden()
    t = orc.recipe_table()
    for solver in ("Single", "Mixed1", "Mixed2"):
        for stage in ("k2", "k3", "k4"):
            assert t[(solver, stage)] == g[(solver, stage)], (solver, stage)
    # the Double column is all double: the FP64 mode evaluates the plain definition
    assert all(g[("Double", s)] == (0, 0, 0) for s in ("k2", "k3", "k4"))


def test_library_recipe_rows_match_the_paper():
    # the GPU library's own table (host code; no device needed)
    import paper_2605_23727_amd as b
    g = _golden()
    for mode, solver in ((5, "Single"), (6, "Mixed1"), (7, "Mixed2")):
        for row, stage in enumerate(("k2", "k3", "k4")):
            assert b.recipe_row(mode, row) == g[(solver, stage)], (solver, stage)
    with pytest.raises(b.BS32Error):
        b.recipe_row(4, 0)


def _attempt_by_hand(orc, w, flags, h, single):
    kw = dict(A=w["A"], param=w["param"], gain=w["gain"])
    kind, n = w["kind"], w["n"]
    rnd = (lambda v: v.astype(np.float32).astype(np.float64)) if single else (lambda v: v)
    X = rnd(w["y0"].copy())
    K1 = orc.rhs_recipe(kind, n, X, *flags["k4"], **kw)  # the first K1 takes the k4 row
    Y = rnd(X + h * (0.5 * K1))
    K2 = orc.rhs_recipe(kind, n, Y, *flags["k2"], **kw)
    Y = rnd(X + h * (0.0 * K1 + 0.75 * K2))
    K3 = orc.rhs_recipe(kind, n, Y, *flags["k3"], **kw)
    Xn = rnd(X + h * (2.0 / 9.0 * K1 + 1.0 / 3.0 * K2 + 4.0 / 9.0 * K3))
    K4 = orc.rhs_recipe(kind, n, Xn, *flags["k4"], **kw)
    e = h * ((2.0 / 9.0 - 7.0 / 24.0) * K1 + (1.0 / 3.0 - 1.0 / 4.0) * K2 + (4.0 / 9.0 - 1.0 / 3.0) * K3
             + (0.0 - 1.0 / 8.0) * K4)
    rtol = 1e-6
    W = np.maximum(np.maximum(np.abs(X), np.abs(Xn)), 1.0)
    return Xn, float(np.max(np.abs(e) / W))


@pytest.mark.parametrize("mode,solver", [(5, "Single"), (6, "Mixed1"), (7, "Mixed2")])
def test_each_row_serves_its_stage(orc, mode, solver):
    import workloads
    w = workloads.osc2(7, seed=77, t1=1.0)
    g = _golden()
    flags = {s: g[(solver, s)] for s in ("k2", "k3", "k4")}
    h = 0.0625
    y, st, tr = orc.bs32_solve(w["kind"], w["n"], w["y0"], 0.0, h, 1e-6, A=w["A"], param=w["param"],
                               gain=w["gain"], mode=mode, fixed_step=True, h0=h, trace_cap=4)
    assert st["n_accept"] == 1 and st["status"] == 0
    Xn, err = _attempt_by_hand(orc, w, flags, h, single=solver == "Single")
    np.testing.assert_array_equal(y, Xn)
    assert tr["err"][0] == err
    # the rows are not interchangeable: k2 evaluated with the k4 row (Mixed1) or
    # all rows double changes the attempt
    swapped = dict(flags, k2=flags["k4"]) if solver == "Mixed1" else {s: (0, 0, 0) for s in flags}
    Xs, _ = _attempt_by_hand(orc, w, swapped, h, single=solver == "Single")
    assert np.any(Xs != Xn)


# ---------------------------------------------------------------------------
# hand-derived values of one evaluation, every (pF, pS, pG)
# ---------------------------------------------------------------------------
def _eval(orc, kind, y, pF, pS, pG, A, param, gain=1.0, stimulus=0.0):
    n = A.shape[0]
    return orc.rhs_recipe(kind, n, np.array(y, dtype=np.float64), pF, pS, pG, A=A, param=np.array(param, float),
                          gain=gain, stimulus=stimulus)


SWAP2 = np.array([[0.0, 1.0], [1.0, 0.0]])


@pytest.mark.parametrize("pF,pS,pG", COMBOS)
def test_pair_term_rounds_components_in_single_osc2(orc, pF, pS, pG):
    # x = (1 + e, 1): the FP64 difference is -e, the difference of FP32-rounded
    # components is 0; weights 1/2, so the coupling of agent 0 is -e/2 or 0
    f = _eval(orc, orc.OSC2, [1 + E, 0.0, 1.0, 0.0], pF, pS, pG, SWAP2, [0.0, 0.0])
    c = 0.0 if pG else E / 2
    np.testing.assert_array_equal(f, [0.0, -c, 0.0, c])


@pytest.mark.parametrize("pF,pS,pG", COMBOS)
def test_pair_term_and_agent_term_lco(orc, pF, pS, pG):
    # eq. (LCO): x' = v + coupling, v' = -x; the agent term -x of 1 + e is -1 in FP32
    f = _eval(orc, orc.LCO_PAPER, [1 + E, 0.0, 1.0, 0.0], pF, pS, pG, SWAP2, [1.0, 1.0])
    c = 0.0 if pG else E / 2
    np.testing.assert_array_equal(f, [-c, -1.0 if pF else -(1 + E), c, -1.0])


@pytest.mark.parametrize("pF,pS,pG", COMBOS)
def test_goodwin_gain_and_agent_term(orc, pF, pS, pG):
    # z = 1 gives 1/(1 + z^10) = 1/2 exactly, b = 0; kappa = 1/2 multiplies the
    # sum: agent 0 gets 1/2 - e/4 in FP64, which FP32 (ulp 2^-25 below 1/2) rounds to 1/2
    y = [1 + E, 0.0, 1.0, 1.0, 0.0, 1.0]
    f = _eval(orc, orc.GOODWIN3, y, pF, pS, pG, SWAP2, [0.0, 0.0], gain=0.5)
    c = 0.0 if pG else E / 4
    x0 = 0.5 - (0.0 if pF else c)
    x1 = 0.5 + (0.0 if pF else c)
    np.testing.assert_array_equal(f, [x0, 1.0 if pF else 1 + E, 0.0, x1, 1.0, 0.0])


@pytest.mark.parametrize("pF,pS,pG", COMBOS)
def test_kuramoto_gain_inside_the_pair_term(orc, pF, pS, pG):
    # theta = (1 + e, 1), K = 2, weights 1/2: sin(-e) = -e in both precisions, so
    # the coupling is K/2 * (-e) = -e (FP64 pair term) or 0 (FP32 components);
    # omega_0 = 1 + 2e rounds to 1 in FP32, and 1 - e rounds back to 1 there
    f = _eval(orc, orc.KURAMOTO, [1 + E, 1.0], pF, pS, pG, SWAP2, [1 + 2 * E, 0.0], gain=2.0)
    c = 0.0 if pG else E
    f0 = 1.0 if pF else (1 + 2 * E) - c
    np.testing.assert_array_equal(f, [f0, c])


@pytest.mark.parametrize("pF,pS,pG", COMBOS)
def test_weight_is_rounded_to_single(orc, pF, pS, pG):
    # A_01 = 1/3, N = 3: the single weight is f32(f32(1/3) * f32(1/3)), not f32(1/9)
    A = np.zeros((3, 3))
    A[0, 1] = 1.0 / 3.0
    f = _eval(orc, orc.OSC2, [0.0, 0.0, 1.0, 0.0, 0.0, 0.0], pF, pS, pG, A, [0.0, 0.0, 0.0])
    third32 = f32(Fr(1, 3))
    m32 = f32(third32 * third32)
    m64 = f64(f64(Fr(1, 3)) * f64(Fr(1, 3)))
    assert m32 != f32(Fr(1, 9)) and m32 != f32(m64)  # the inputs can tell the readings apart
    want = m32 if pG else (f32(m64) if (pF or pS) else m64)  # a single sum rounds the term too
    assert Fr(f[1]) == want
    np.testing.assert_array_equal(f[2:], 0.0)


@pytest.mark.parametrize("pF,pS,pG", COMBOS)
def test_single_sum_drops_what_the_double_sum_keeps(orc, pF, pS, pG):
    # weights 1/4 on x = (0, 4, 2^-22, 2^-22): pair terms 1, 2^-24, 2^-24, exact in
    # both precisions; the FP64 sum is 1 + 2^-23, the FP32 sum ties twice to 1
    A = np.zeros((4, 4))
    A[0, 1:] = 1.0
    y = [0.0, 0.0, 4.0, 0.0, 2.0 ** -22, 0.0, 2.0 ** -22, 0.0]
    f = _eval(orc, orc.OSC2, y, pF, pS, pG, A, [0.0] * 4)
    assert f[1] == (1.0 if pS else 1.0 + 2.0 ** -23)


@pytest.mark.parametrize("pF,pS,pG", COMBOS)
def test_agent_term_in_single(orc, pF, pS, pG):
    # omega = 1 + 2^-20 (exact in FP32), x = v = 1 + e; omega^2 = 1 + 2^-19 + 2^-40
    # rounds to 1 + 2^-19 in FP32, and times x (which FP32 rounds to 1) stays so;
    # in FP64 omega^2 x = 1 + 2^-19 + 2^-30 + 2^-40 + 2^-49 (+ 2^-70, rounded off)
    A = np.zeros((1, 1))
    f = _eval(orc, orc.OSC2, [1 + E, 1 + E], pF, pS, pG, A, [1 + 2.0 ** -20])
    if pF:
        want = [1.0, -(1 + 2.0 ** -19)]
    else:
        want = [1 + E, -(1 + 2.0 ** -19 + 2.0 ** -30 + 2.0 ** -40 + 2.0 ** -49)]
    np.testing.assert_array_equal(f, want)


@pytest.mark.parametrize("pF,pS,pG", COMBOS)
def test_clock_model_pair_and_agent_terms(orc, pF, pS, pG):
    # eq. (CC) with k1 = 1 (theta^h = 1) and X_2 = 1: the prefactor is
    # k0 th a / (th + 1) = 2 exactly; X_1 = (1 + e, 1) and K = 1 give the agent-0
    # pair term 1/2 * 2 * atan(-e) = -e in FP64, 0 from FP32 components.
    # Agent term of agent 0 in FP64: (2 (1+e)^2 + 1) - (1 + e) = 2 + 3e (the 2^-59 of
    # the square is rounded off); in FP32 (components rounded to 1): 2, and 2 - e
    # rounds back to 2 there.  k2 (X_1 - X_2) is k2 e, or 0 in FP32.
    y = [1 + E, 1.0, 0.0, 0.0, 1.0, 1.0, 0.0, 0.0]
    f = _eval(orc, orc.CLOCK4, y, pF, pS, pG, SWAP2, [1.0, 1.0], gain=1.0, stimulus=0.0)
    c = 0.0 if pG else E
    if pF:
        assert f[0] == 2.0 and f[1] == 0.0
    else:
        assert f[0] == (2 + 3 * E) - c
        assert f[1] == 0.144832 * E
    # the last two components (x3 = x4 = 0, I0 = 0): 0 and eps (b - 0) = 0.228249 * 0.7
    assert f[2] == 0.0
    eps_b = float(f32(f32(Fr(0.228249)) * f32(Fr(0.7)))) if pF else 0.228249 * 0.7
    assert f[3] == eps_b
    assert f[4] == (2.0 if pF else 2.0 + c)  # agent 1: (2 + 1) - 1 + coupling e
    assert f[5] == 0.0 and f[6] == 0.0 and f[7] == eps_b


@pytest.mark.parametrize("pG", (0, 1))
def test_clock_model_prefactor_precision(orc, pG):
    # k1 = 3/4 gives theta^h = f(3/5) and X_2 = 2 gives X_2^4 = 16, so the prefactor
    # 2 th / (th + 16) * 2 is rounded differently in FP32 and FP64 (and the FP32 one
    # is not the FP64 one rounded to FP32).  A weight of 2^40 (N = 2) and
    # X_1 = (0, 2^-30) make the pair term 2^39 * pre * atan(2^-30) = 512 pre, which
    # dominates agent 0's equation (its agent term is q = pre / 2).
    A = np.array([[0.0, 2.0 ** 40], [0.0, 0.0]])
    y = [0.0, 2.0, 0.0, 0.0, 2.0 ** -30, 2.0, 0.0, 0.0]
    f = _eval(orc, orc.CLOCK4, y, 0, 0, pG, A, [0.75, 0.75], gain=1.0)
    th64 = f64(Fr(3, 5))
    q64 = f64(f64(2 * th64) / f64(th64 + 16))
    th32 = f32(Fr(3, 5))
    pre32 = 2 * f32((2 * th32) / f32(th32 + 16))
    pre64 = 2 * q64
    assert pre32 != pre64 and pre32 != f32(pre64)
    pre = pre32 if pG else pre64
    assert Fr(f[0]) == f64(q64 + 512 * pre)


@pytest.mark.parametrize("pF,pS,pG", COMBOS)
def test_goodwin_gain_multiplies_the_single_sum(orc, pF, pS, pG):
    # x = (1, 3), z = 1, b = 0, kappa = 1/2, weights 1/2: sums +1 and -1, coupling
    # +-1/2, so x' = 1/2 +- 1/2; every value is exact in both precisions
    y = [1.0, 0.0, 1.0, 3.0, 0.0, 1.0]
    f = _eval(orc, orc.GOODWIN3, y, pF, pS, pG, SWAP2, [0.0, 0.0], gain=0.5)
    np.testing.assert_array_equal(f, [1.0, 1.0, 0.0, 0.0, 3.0, 0.0])

"""Pins of the oracle's Butcher tables (paper Sec. 2.2, Table Butcher-O23).

The BS3(2) table is compared entry by entry with the table printed in the
paper (tests/golden/bs32_butcher.txt) and checked against the order
conditions, in exact rational arithmetic.
"""
import os
from fractions import Fraction as Fr

import numpy as np

GOLD = os.path.join(os.path.dirname(__file__), "golden", "bs32_butcher.txt")


def _frac(x):
    return Fr(x).limit_denominator(10**6)


def _golden():
    rows = {}
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, *vals = line.split()
        rows[key] = [Fr(v) for v in vals]
    return rows


def test_bs32_table_matches_paper(orc):
    c, a, b, bt = orc.bs32_tableau()
    g = _golden()
    assert [_frac(v) for v in c] == g["c"]
    assert [_frac(v) for v in b] == g["b"]
    assert [_frac(v) for v in bt] == g["bt"]
    for l in (2, 3, 4):
        row = [_frac(v) for v in a[l - 1, : l - 1]]
        assert row == g[f"a{l}"][: l - 1] + [Fr(0)] * (l - 1 - len(g[f"a{l}"]))
    # the doubles are the correctly rounded fractions
    for v in list(c) + list(b) + list(bt) + list(a.ravel()):
        assert float(_frac(v)) == v


def test_bs32_order_conditions(orc):
    c, a, b, bt = orc.bs32_tableau()
    c = [_frac(v) for v in c]
    b = [_frac(v) for v in b]
    bt = [_frac(v) for v in bt]
    A = [[_frac(v) for v in row] for row in a]
    # row sums equal c (consistency of the stages)
    for i in range(4):
        assert sum(A[i]) == c[i]
    # third order for b
    assert sum(b) == 1
    assert sum(bi * ci for bi, ci in zip(b, c)) == Fr(1, 2)
    assert sum(bi * ci * ci for bi, ci in zip(b, c)) == Fr(1, 3)
    Ac = [sum(A[i][j] * c[j] for j in range(4)) for i in range(4)]
    assert sum(bi * x for bi, x in zip(b, Ac)) == Fr(1, 6)
    # second order for the embedded weights, and not third
    assert sum(bt) == 1
    assert sum(x * y for x, y in zip(bt, c)) == Fr(1, 2)
    assert sum(x * y * y for x, y in zip(bt, c)) != Fr(1, 3) or sum(x * y for x, y in zip(bt, Ac)) != Fr(1, 6)
    # FSAL: the last stage row equals b, and c4 = 1
    assert A[3][:3] == b[:3] and c[3] == 1 and b[3] == 0
    # error weights e = b - bt
    e = [x - y for x, y in zip(b, bt)]
    assert e == [Fr(-5, 72), Fr(1, 12), Fr(1, 9), Fr(-1, 8)]
    assert sum(e) == 0


def test_dp54_order_conditions(orc):
    c, a, b, bt = orc.dp54_tableau()
    c = [Fr(v).limit_denominator(10**7) for v in c]
    A = [[Fr(v).limit_denominator(10**7) for v in row] for row in a]
    b = [Fr(v).limit_denominator(10**7) for v in b]
    bt = [Fr(v).limit_denominator(10**7) for v in bt]
    for i in range(7):
        assert sum(A[i]) == c[i]
    Ac = [sum(A[i][j] * c[j] for j in range(7)) for i in range(7)]
    Ac2 = [sum(A[i][j] * c[j] ** 2 for j in range(7)) for i in range(7)]
    AAc = [sum(A[i][j] * Ac[j] for j in range(7)) for i in range(7)]
    for w, order in ((b, 5), (bt, 4)):
        assert sum(w) == 1
        assert sum(x * y for x, y in zip(w, c)) == Fr(1, 2)
        assert sum(x * y ** 2 for x, y in zip(w, c)) == Fr(1, 3)
        assert sum(x * y for x, y in zip(w, Ac)) == Fr(1, 6)
        assert sum(x * y ** 3 for x, y in zip(w, c)) == Fr(1, 4)
        assert sum(x * y * z for x, y, z in zip(w, c, Ac)) == Fr(1, 8)
        assert sum(x * y for x, y in zip(w, Ac2)) == Fr(1, 12)
        assert sum(x * y for x, y in zip(w, AAc)) == Fr(1, 24)
        if order == 5:
            assert sum(x * y ** 4 for x, y in zip(w, c)) == Fr(1, 5)
    assert A[6][:6] == b[:6]


def _order_sums(w, c, A):
    """The elementary-weight sums of the Runge-Kutta order conditions up to order 5,
    as (value, required) pairs keyed by order."""
    s = len(c)
    Ac = [sum(A[i][j] * c[j] for j in range(s)) for i in range(s)]
    Ac2 = [sum(A[i][j] * c[j] ** 2 for j in range(s)) for i in range(s)]
    Ac3 = [sum(A[i][j] * c[j] ** 3 for j in range(s)) for i in range(s)]
    AAc = [sum(A[i][j] * Ac[j] for j in range(s)) for i in range(s)]
    AcAc = [sum(A[i][j] * c[j] * Ac[j] for j in range(s)) for i in range(s)]
    AAc2 = [sum(A[i][j] * Ac2[j] for j in range(s)) for i in range(s)]
    AAAc = [sum(A[i][j] * AAc[j] for j in range(s)) for i in range(s)]

    def dot(*vs):
        return sum(w[i] * np.prod([v[i] for v in vs]) for i in range(s))

    cc = [x * x for x in c]
    c3 = [x ** 3 for x in c]
    c4 = [x ** 4 for x in c]
    Ac_sq = [x * x for x in Ac]
    ones = [Fr(1)] * s
    return {
        1: [(dot(ones), Fr(1))],
        2: [(dot(c), Fr(1, 2))],
        3: [(dot(cc), Fr(1, 3)), (dot(Ac), Fr(1, 6))],
        4: [(dot(c3), Fr(1, 4)), (dot(c, Ac), Fr(1, 8)), (dot(Ac2), Fr(1, 12)), (dot(AAc), Fr(1, 24))],
        5: [(dot(c4), Fr(1, 5)), (dot(cc, Ac), Fr(1, 10)), (dot(Ac_sq), Fr(1, 20)), (dot(c, Ac2), Fr(1, 15)),
            (dot(Ac3), Fr(1, 20)), (dot(c, AAc), Fr(1, 30)), (dot(AcAc), Fr(1, 40)), (dot(AAc2), Fr(1, 60)),
            (dot(AAAc), Fr(1, 120))],
    }


def test_rkf45_order_conditions(orc):
    """Fehlberg 4(5): the propagated weights b satisfy every condition up to order four
    and not all of order five; the embedded weights bh satisfy all of order five."""
    c0, a0, b0, bh0 = orc.rkf45_tableau()
    raw = list(c0) + list(b0) + list(bh0) + list(a0.ravel())
    c = [Fr(v).limit_denominator(10**6) for v in c0]
    A = [[Fr(v).limit_denominator(10**6) for v in row] for row in a0]
    b = [Fr(v).limit_denominator(10**6) for v in b0]
    bh = [Fr(v).limit_denominator(10**6) for v in bh0]
    # the doubles are the correctly rounded fractions
    for v in raw:
        assert float(Fr(v).limit_denominator(10**6)) == v
    for i in range(6):
        assert sum(A[i]) == c[i]
        assert all(A[i][j] == 0 for j in range(i, 6))  # explicit
    sb = _order_sums(b, c, A)
    sh = _order_sums(bh, c, A)
    for order in (1, 2, 3, 4):
        assert all(v == r for v, r in sb[order]), order
    assert not all(v == r for v, r in sb[5])
    for order in (1, 2, 3, 4, 5):
        assert all(v == r for v, r in sh[order]), order
    assert b[5] == 0 and bh[5] == Fr(2, 55)

"""Analytic solution of the coupled linear oscillators and their real local error.

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the product
library.

Paper Benchmark 1, eq. (LCO), with the paper's uniform weights M_ij = 1/N:

    X_i1' = X_i2 + (1/N) sum_j (X_j1 - X_i1),      X_i2' = -X_i1.

The system is linear, X' = L X, and the paper notes that it has an analytic
solution (Sec. 2.1).  Written with the means m = (1/N) sum_j X_j1 and
w = (1/N) sum_j X_j2, the coupling is m - X_i1, so

  * the means move as an undamped oscillator:  m' = w,      w' = -m;
  * the deviations d_i = X_i1 - m, e_i = X_i2 - w as a damped one:
        d' = e - d,  e' = -d,
    whose matrix B = [[-1, 1], [-1, 0]] has trace -1 and determinant 1, hence
    exp(hB) = e^{-h/2} (cos(wh) I + sin(wh)/w (B + I/2)) with w = sqrt(3)/2.

exp(hL) X is the sum of the two motions.  The real local error of a step
(Sec. 2.4, eq. (LCO-Local-Error)) compares the numerical solution after the
step with this flow started from the solution before it.
"""
from __future__ import annotations

import math

import numpy as np

OMEGA = math.sqrt(3.0) / 2.0


def lco_flow(x, h):
    """exp(hL) x for one agent-major state x (2N values: X_11, X_12, X_21, ...), FP64."""
    X = np.asarray(x, dtype=np.float64).reshape(-1, 2)
    m = X[:, 0].mean()
    w = X[:, 1].mean()
    # mean motion: rotation by angle h
    c, s = math.cos(h), math.sin(h)
    m_h = c * m + s * w
    w_h = -s * m + c * w
    # deviation motion: exp(hB) applied to (d, e)
    d = X[:, 0] - m
    e = X[:, 1] - w
    damp = math.exp(-0.5 * h)
    co = math.cos(OMEGA * h)
    so = math.sin(OMEGA * h) / OMEGA
    # (B + I/2)(d, e) = (-d/2 + e, -d + e/2)
    d_h = damp * (co * d + so * (-0.5 * d + e))
    e_h = damp * (co * e + so * (-d + 0.5 * e))
    out = np.empty_like(X)
    out[:, 0] = m_h + d_h
    out[:, 1] = w_h + e_h
    return out.reshape(-1)


def lco_local_error(x_n, x_next, h, delta):
    """eq. (LCO-Local-Error): max_k |X^{n+1}_k - X_ex,k| / max(|X_ex,k|, delta) with
    X_ex = exp(h L) X^n, over all 2N components."""
    ex = lco_flow(x_n, h)
    xn1 = np.asarray(x_next, dtype=np.float64).reshape(-1)
    return float(np.max(np.abs(xn1 - ex) / np.maximum(np.abs(ex), delta)))

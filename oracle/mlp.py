"""FP64 reference of the learned step-size proposer: network, training loss,
gradient and the training samples drawn from a solver trace.

TEST INFRASTRUCTURE ONLY: imported by the test suite alone.

The proposer is an extension of the method.  Sec. 2.2 of the paper fixes only
that the error estimate E drives the step-size correction and that a step is
accepted iff E < Rel; nothing here touches acceptance.

Network: 9 -> 64 -> 64 -> 1, tanh hidden layers, linear output, applied to the
standardized features x_k = (f_k - mu_k) inv_sd_k.  Parameter vector, in order:
W1[64][9], b1[64], W2[64][64], b2[64], w3[64], b3, mu[9], inv_sd[9]; training
changes the network weights only.

Features after an accepted attempt n (most recent first):
    f[0..3] = log h_n, log h_{n-1}, log h_{n-2}, log h_{n-3}
    f[4..7] = log(max(E, 1e-30 Rel) / Rel) of the same attempts
    f[8]    = log max(fnorm_n, 1e-300), fnorm_n = max_k |K1_k| / max(|X^n_k|, Ab/Rel)
Output: delta = log(h_{n+1} / h_n), used by the solver only when every
standardized feature lies in [-4, 4] and delta is inside [log 0.2, log 5] and
within log 2 of the classical rule's step ratio.

Label of sample n: the step that would have put attempt n+1's estimate at
0.8 Rel if E grows like h^3 (the local error of the second-order embedded
solution is O(h^3)):
    label_n = log(h_{n+1} / h_n) + (1/3) log(0.8 Rel / E_{n+1}).
Loss over a set of samples: (1/n) sum_s w_s (y_s - label_s)^2 with w_s = 4 when
the prediction overshoots (y_s > label_s; a rejected attempt costs three RHS
evaluations) and 1 otherwise.
"""
from __future__ import annotations

import math

import numpy as np

IN, HID = 9, 64
NET = HID * IN + HID + HID * HID + HID + HID + 1
PARAMS = NET + 2 * IN
OVER_W = 4.0
TARGET = 0.8


def unpack(w):
    """(W1 [64,9], b1 [64], W2 [64,64], b2 [64], w3 [64], b3, mu [9], inv_sd [9]) of a parameter vector."""
    w = np.asarray(w, dtype=np.float64)
    assert w.size == PARAMS
    o = 0
    W1 = w[o:o + HID * IN].reshape(HID, IN)
    o += HID * IN
    b1 = w[o:o + HID]
    o += HID
    W2 = w[o:o + HID * HID].reshape(HID, HID)
    o += HID * HID
    b2 = w[o:o + HID]
    o += HID
    w3 = w[o:o + HID]
    o += HID
    b3 = w[o]
    o += 1
    return W1, b1, W2, b2, w3, b3, w[o:o + IN], w[o + IN:o + 2 * IN]


def forward(w, F):
    """Network outputs for the feature rows of F [n, 9]; returns (y [n], (x, h1, h2))."""
    W1, b1, W2, b2, w3, b3, mu, inv_sd = unpack(w)
    X = (np.asarray(F, dtype=np.float64).reshape(-1, IN) - mu) * inv_sd
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ w3 + b3, (X, h1, h2)


def loss(w, F, Y, over_w=OVER_W):
    y, _ = forward(w, F)
    r = y - np.asarray(Y, dtype=np.float64)
    wt = np.where(r > 0.0, over_w, 1.0)
    return float(np.mean(wt * r * r))


def grad(w, F, Y, over_w=OVER_W):
    """Gradient of `loss` with respect to the network weights (backpropagation);
    zero for mu and inv_sd, which training leaves alone."""
    W1, b1, W2, b2, w3, b3, mu, inv_sd = unpack(w)
    y, (X, h1, h2) = forward(w, F)
    n = X.shape[0]
    r = y - np.asarray(Y, dtype=np.float64)
    dy = 2.0 * np.where(r > 0.0, over_w, 1.0) * r / n  # dL/dy
    g_w3 = h2.T @ dy
    g_b3 = dy.sum()
    dz2 = np.outer(dy, w3) * (1.0 - h2 * h2)  # through tanh: d tanh(z)/dz = 1 - tanh(z)^2
    g_W2 = dz2.T @ h1
    g_b2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (1.0 - h1 * h1)
    g_W1 = dz1.T @ X
    g_b1 = dz1.sum(axis=0)
    return np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3], np.zeros(2 * IN)])


def features_at(trace, q, rtol):
    """Features of the proposal after attempt q of a trace (fields h, err, fnorm)."""
    f = [math.log(float(trace["h"][q - k])) for k in range(4)]
    f += [math.log(max(float(trace["err"][q - k]), 1e-30 * rtol) / rtol) for k in range(4)]
    f.append(math.log(max(float(trace["fnorm"][q]), 1e-300)))
    return np.array(f, dtype=np.float64)


def samples(trace, rtol):
    """(features [m, 9], labels [m]) from a trace with fields h, err, fnorm, accepted.

    One sample per accepted attempt n >= 3 whose next attempt is not the last
    record and has 0 < E < inf (the last attempt is clipped onto t1, so its
    step says nothing about the controller)."""
    F, Y = [], []
    n = len(trace)
    for q in range(3, n - 2):
        if not trace["accepted"][q]:
            continue
        h_next, e_next = float(trace["h"][q + 1]), float(trace["err"][q + 1])
        if not (e_next > 0.0 and math.isfinite(e_next) and h_next > 0.0):
            continue
        if not all(float(trace["h"][q - k]) > 0.0 and math.isfinite(float(trace["err"][q - k])) for k in range(4)):
            continue
        F.append(features_at(trace, q, rtol))
        Y.append(math.log(h_next / float(trace["h"][q])) + math.log(TARGET * rtol / e_next) / 3.0)
    return np.array(F, dtype=np.float64).reshape(-1, IN), np.array(Y, dtype=np.float64)

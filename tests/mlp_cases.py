"""Inputs of the learned-proposer tests: parameter vectors and trace records.

Networks are inputs here, never expected values: a seeded random network and a
hand-built one whose output follows the classical step-size rule closely.
"""
import math

import numpy as np

IN, HID = 9, 64
NET = HID * IN + HID + HID * HID + HID + HID + 1
PARAMS = NET + 2 * IN
OFF_W1 = 0
OFF_B1 = OFF_W1 + HID * IN
OFF_W2 = OFF_B1 + HID
OFF_B2 = OFF_W2 + HID * HID
OFF_W3 = OFF_B2 + HID
OFF_B3 = OFF_W3 + HID
OFF_MU = NET
OFF_ISD = NET + IN


def _net(inv_sd=1.0):
    w = np.zeros(PARAMS)
    w[OFF_ISD:OFF_ISD + IN] = inv_sd   # mu = 0
    return w


# hand-built networks read x = f / 64, so that any feature up to |f| = 256 lies
# inside the region where the solver uses a proposal (|x| <= 4)
WIDE = 1.0 / 64.0

TRACE_DTYPE = np.dtype([("t", "f8"), ("h", "f8"), ("err", "f8"), ("fnorm", "f8"), ("accepted", "i4"),
                        ("proposer", "i4")])


def random_net(seed, scale=1.0):
    """Glorot-uniform weights and small random biases, seeded."""
    rng = np.random.default_rng(seed)
    w = _net()
    lim1 = math.sqrt(6.0 / (IN + HID))
    lim2 = math.sqrt(6.0 / (2 * HID))
    lim3 = math.sqrt(6.0 / (HID + 1))
    w[OFF_W1:OFF_B1] = rng.uniform(-lim1, lim1, HID * IN) * scale
    w[OFF_B1:OFF_W2] = rng.uniform(-0.1, 0.1, HID)
    w[OFF_W2:OFF_B2] = rng.uniform(-lim2, lim2, HID * HID) * scale
    w[OFF_B2:OFF_W3] = rng.uniform(-0.1, 0.1, HID)
    w[OFF_W3:OFF_B3] = rng.uniform(-lim3, lim3, HID) * scale
    w[OFF_B3] = rng.uniform(-0.1, 0.1)
    return w


def controller_net(gain=1.0 / 3.0, target=0.8):
    """Network whose output is close to gain * (log target - f[4]): one unit per
    layer in its near-linear range, i.e. h_next ~ h (target Rel / E)^gain."""
    w = _net(WIDE)
    a1, a2 = 0.01, 0.01
    w[OFF_W1 + 0 * IN + 4] = a1 / WIDE  # hidden unit 0 of layer 1 reads f[4] = log(E_n / Rel)
    w[OFF_W2 + 0 * HID + 0] = a2      # hidden unit 0 of layer 2 reads unit 0 of layer 1
    w[OFF_W3 + 0] = -gain / (a1 * a2)
    w[OFF_B3] = gain * math.log(target)
    return w


def constant_net(c):
    """Network whose output is the constant c."""
    w = _net(WIDE)
    w[OFF_B3] = c
    return w


def trace(h, err, fnorm, accepted):
    tr = np.zeros(len(h), dtype=TRACE_DTYPE)
    tr["t"] = np.concatenate([[0.0], np.cumsum(h)[:-1]])
    tr["h"] = h
    tr["err"] = err
    tr["fnorm"] = fnorm
    tr["accepted"] = accepted
    return tr

"""Pins of the oracle's learned step-size proposer (an extension of the
method: the paper's Sec. 2.2 leaves the step-size correction open and makes the
error estimate the only judge of acceptance).

- backpropagation against central finite differences of the loss;
- the network's parameter layout against hand-built networks with a known
  output (a transposed weight block or a swapped feature index changes it);
- the two oracle evaluations of the network (C and numpy) against each other;
- features and labels against traces whose logarithms are integers, and the
  label against the cubic error model it is derived from;
- the oracle solver's use of the proposal: constant-output networks give
  h_{n+1} = h_n e^c exactly where the proposal applies, the classical rule
  everywhere else, and no accepted attempt ever has E >= Rel.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import mlp
from tests import mlp_cases as mc


def _data(seed, n):
    rng = np.random.default_rng(seed)
    X = rng.normal(0.0, 1.0, (n, mc.IN))
    Y = rng.normal(0.0, 0.5, n)
    return X, Y


def test_parameter_count():
    assert mlp.PARAMS == mc.PARAMS == 4883 and mlp.NET == 4865


def test_gradient_matches_finite_differences():
    w = mc.random_net(11)
    X, Y = _data(12, 37)
    g = mlp.grad(w, X, Y)
    rng = np.random.default_rng(13)
    idx = np.concatenate([rng.choice(mlp.PARAMS, 120, replace=False),
                          [mc.OFF_B1, mc.OFF_B2 + 5, mc.OFF_W3 + 63, mc.OFF_B3, mc.OFF_W1 + 8]])
    eps = 1e-6
    scale = np.max(np.abs(g))
    for p in idx:
        wp = w.copy()
        wm = w.copy()
        wp[p] += eps
        wm[p] -= eps
        fd = (mlp.loss(wp, X, Y) - mlp.loss(wm, X, Y)) / (2 * eps)
        assert abs(fd - g[p]) <= 1e-7 * scale + 1e-7 * abs(g[p]), (p, fd, g[p])


def test_loss_weights_overshoot_four_times():
    # one sample, zero network except the output bias: y = b3
    w = mc.constant_net(0.25)
    X = np.zeros((1, mc.IN))
    assert mlp.loss(w, X, [0.0]) == pytest.approx(4 * 0.25 ** 2, rel=1e-15)   # overshoot
    assert mlp.loss(w, X, [0.5]) == pytest.approx(0.25 ** 2, rel=1e-15)       # undershoot
    g = mlp.grad(w, X, [0.0])
    assert g[mc.OFF_B3] == pytest.approx(2 * 4 * 0.25, rel=1e-15)


@pytest.mark.parametrize("j,i,k", [(0, 0, 0), (37, 11, 4), (63, 62, 8), (5, 40, 2)])
def test_forward_layout_hand_built(orc, j, i, k):
    """Layer-1 unit j reads feature k, layer-2 unit i reads unit j; output 0.5."""
    w = mc.constant_net(0.0)
    w[mc.OFF_ISD:mc.OFF_ISD + mc.IN] = 1.0
    w[mc.OFF_W1 + j * mc.IN + k] = 1.0
    w[mc.OFF_W2 + i * mc.HID + j] = 1.0
    w[mc.OFF_B2 + i] = math.atanh(0.75) - 0.5
    w[mc.OFF_W3 + i] = 2.0
    w[mc.OFF_B3] = -1.0
    f = np.full(mc.IN, 3.0)
    f[k] = math.atanh(0.5)   # tanh(z1_j) = 0.5, every other layer-1 unit is tanh(0) = 0
    y, _ = mlp.forward(w, f[None, :])
    assert y[0] == pytest.approx(0.5, abs=1e-15)
    assert orc.mlp_forward(w, f) == pytest.approx(0.5, abs=1e-15)
    # the same network on a feature vector that moves only another feature is unchanged
    f2 = f.copy()
    f2[(k + 1) % mc.IN] = -7.0
    assert orc.mlp_forward(w, f2) == pytest.approx(0.5, abs=1e-15)


@pytest.mark.parametrize("k", [0, 4, 8])
def test_forward_standardizes_features(orc, k):
    """mu and inv_sd act as x = (f - mu) inv_sd on every feature before layer 1."""
    w = mc.random_net(31 + k)   # identity standardization
    rng = np.random.default_rng(k)
    mu = rng.normal(0.0, 3.0, mc.IN)
    isd = rng.uniform(0.2, 4.0, mc.IN)
    ws = w.copy()
    ws[mc.OFF_MU:mc.OFF_MU + mc.IN] = mu
    ws[mc.OFF_ISD:mc.OFF_ISD + mc.IN] = isd
    F = rng.normal(0.0, 3.0, (5, mc.IN))
    y_std, _ = mlp.forward(ws, F)
    y_id, _ = mlp.forward(w, (F - mu) * isd)
    np.testing.assert_allclose(y_std, y_id, rtol=1e-14, atol=1e-14)
    for r in range(5):
        assert orc.mlp_forward(ws, F[r]) == pytest.approx(y_std[r], rel=1e-13, abs=1e-13)
    # training leaves the standardization alone
    assert np.all(mlp.grad(ws, F, np.zeros(5))[mlp.NET:] == 0.0)


def test_c_and_numpy_forward_agree(orc):
    for seed in range(4):
        w = mc.random_net(100 + seed, scale=1.5)
        X, _ = _data(200 + seed, 16)
        y, _ = mlp.forward(w, X)
        for r in range(16):
            assert orc.mlp_forward(w, X[r]) == pytest.approx(y[r], rel=1e-13, abs=1e-13)


def test_samples_integer_logs():
    rtol = 1e-6
    # h = e^-1 .. e^-8, E / Rel = e^-1, e^-2, ...; fnorm = e^(q)
    h = np.exp(-np.arange(1.0, 9.0))
    err = rtol * np.exp(-np.arange(1.0, 9.0))
    fn = np.exp(np.arange(8.0))
    acc = np.array([1, 1, 1, 1, 0, 1, 1, 1])
    tr = mc.trace(h, err, fn, acc)
    F, Y = mlp.samples(tr, rtol)
    # candidates q = 3..5: q = 4 is rejected, so samples come from q = 3 and q = 5
    assert F.shape == (2, 9)
    np.testing.assert_allclose(F[0], [-4, -3, -2, -1, -4, -3, -2, -1, 3], atol=1e-14)
    np.testing.assert_allclose(F[1], [-6, -5, -4, -3, -6, -5, -4, -3, 5], atol=1e-14)
    # label q: log(h_{q+1}/h_q) + (1/3) log(0.8 Rel / E_{q+1}) = -1 + (log 0.8 + q + 2) / 3
    np.testing.assert_allclose(Y, [-1 + (math.log(0.8) + 5) / 3, -1 + (math.log(0.8) + 7) / 3], atol=1e-14)


def test_samples_skip_zero_and_nonfinite_estimates():
    rtol = 1e-8
    h = np.full(9, 0.01)
    err = np.full(9, 0.5 * rtol)
    err[5] = 0.0          # the next attempt of q = 4 has no estimate to learn from
    err[2] = np.inf       # q = 3, 4, 5 see it in their history
    tr = mc.trace(h, err, np.ones(9), np.ones(9, dtype=int))
    F, _ = mlp.samples(tr, rtol)
    assert F.shape[0] == 1   # only q = 6 (q = 7 is followed by the last record)
    # the floor 1e-30 Rel keeps log finite for E = 0
    tr2 = mc.trace(h, np.where(np.isinf(err), 0.0, err), np.ones(9), np.ones(9, dtype=int))
    f = mlp.features_at(tr2, 5, rtol)
    assert f[4] == pytest.approx(math.log(1e-30), rel=1e-15)


def test_label_is_the_step_of_the_cubic_model():
    """If E = C h^3 exactly, every label points at the same h* with C h*^3 = 0.8 Rel."""
    rtol, C = 1e-7, 3.7e4
    rng = np.random.default_rng(5)
    h = np.exp(rng.uniform(math.log(1e-4), math.log(1e-3), 40))
    tr = mc.trace(h, C * h ** 3, np.ones(40), np.ones(40, dtype=int))
    F, Y = mlp.samples(tr, rtol)
    h_star = (0.8 * rtol / C) ** (1.0 / 3.0)
    np.testing.assert_allclose(Y + F[:, 0], math.log(h_star), atol=1e-12)


def _kur_solve(orc, mlp_w, rtol=1e-7, n=32, t1=8.0, seed=2100, **kw):
    w = workloads.kuramoto(n, seed=seed, t1=t1)
    return orc.bs32_solve(w["kind"], n, w["y0"], 0.0, t1, rtol, A=w["A"], param=w["param"], gain=w["gain"],
                          trace_cap=200000, mlp_w=mlp_w, **kw)


@pytest.mark.parametrize("c", [math.log(1.1), math.log(1.02), math.log(0.7)])
def test_solver_applies_constant_proposal(orc, c):
    rtol = 1e-7
    y, st, tr = _kur_solve(orc, mc.constant_net(c), rtol=rtol)
    assert st["status"] == 0
    acc = tr["accepted"] == 1
    assert np.all(tr["err"][acc] < rtol) and np.all(tr["err"][~acc] >= rtol)
    h_max = 0.1 * 8.0
    used = fallback = 0
    for q in range(len(tr) - 1):
        nxt = tr["h"][q + 1]
        last = tr["t"][q + 1] + nxt >= 8.0 - 1e-12   # the final attempt may be clipped onto t1
        if acc[q] and q >= 3 and tr["proposer"][q + 1]:
            want = min(tr["h"][q] * math.exp(c), h_max)
            if not last:
                assert nxt == want
            used += 1
        elif acc[q] and q >= 3:
            # the classical step was taken: the proposal lay more than a factor 2 from it
            if not last and nxt < h_max:
                assert abs(math.log(nxt / tr["h"][q]) - c) > math.log(2.0) * (1 - 1e-12)
            fallback += 1
        else:
            assert tr["proposer"][q + 1] == 0
            if not acc[q]:
                assert nxt < tr["h"][q]  # the classical rule shrinks a rejected step
    assert used > 10


def _far_feature(k):
    w = mc.constant_net(math.log(1.05))
    w[mc.OFF_MU + k] = 1000.0   # feature k standardizes to about -16: outside the trained region
    return w


def test_solver_ignores_out_of_range_proposal(orc):
    """Outputs outside [log 0.2, log 5], and any output whose features lie outside
    [-4, 4] after standardization, fall back to the classical controller."""
    ref = _kur_solve(orc, None)
    nets = [mc.constant_net(c) for c in (math.log(5.0) * 1.01, math.log(0.2) * 1.01, float("nan"))]
    nets += [_far_feature(k) for k in (0, 4, 8)]
    assert _kur_solve(orc, mc.constant_net(math.log(1.05)))[2]["proposer"].sum() > 10
    for w in nets:
        y, st, tr = _kur_solve(orc, w)
        assert not np.any(tr["proposer"])
        np.testing.assert_array_equal(y, ref[0])
        assert st["n_accept"] == ref[1]["n_accept"]


def test_solver_proposal_uses_the_trace_features(orc):
    rtol = 1e-7
    w = mc.controller_net()
    y, st, tr = _kur_solve(orc, w, rtol=rtol)
    assert st["status"] == 0
    n_used = 0
    for q in range(3, len(tr) - 2):
        if tr["proposer"][q + 1]:
            delta = orc.mlp_forward(w, mlp.features_at(tr, q, rtol))
            assert tr["h"][q + 1] == pytest.approx(tr["h"][q] * math.exp(delta), rel=1e-14)
            n_used += 1
    assert n_used > 10
    acc = tr["accepted"] == 1
    assert np.all(tr["err"][acc] < rtol)
    # the solution stays within tolerance of the classical solve
    y0, _, _ = _kur_solve(orc, None, rtol=rtol)
    assert np.max(np.abs(y - y0)) < 1e-4

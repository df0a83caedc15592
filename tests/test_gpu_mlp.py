"""GPU tests of the learned step-size proposer: the training kernels' gradient
and loss against the FP64 oracle, training on solver traces, and solves with
the proposer in the loop against the oracle solver driven by the same network.

Acceptance never depends on the proposer: every accepted attempt of every
trace below has E < Rel.
"""
import math
import sys

import numpy as np
import pytest

import workloads
from oracle import mlp
from tests import mlp_cases as mc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bs():
    import paper_2605_23727_amd as b
    s = b.Solver(0)
    yield b, s
    s.close()


def _bf16(orc, w):
    """The network weights rounded to BF16 (the standardization is used as given)."""
    w = np.asarray(w, dtype=np.float64).copy()
    w[:mc.NET] = orc.round_fmt(w[:mc.NET], orc.FMT_BF16)
    return w


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000])
def test_grad_matches_oracle(bs, orc, n):
    b, s = bs
    say(f"[mlp grad] n={n}")
    w = _bf16(orc, mc.random_net(7 + n, scale=1.3)).astype(np.float32)
    rng = np.random.default_rng(n)
    X = rng.normal(0.0, 1.5, (n, 9)).astype(np.float32)
    Y = rng.normal(0.0, 0.7, n).astype(np.float32)
    g, L = s.mlp_grad(w, X, Y)
    go = mlp.grad(w.astype(np.float64), X.astype(np.float64), Y.astype(np.float64))
    Lo = mlp.loss(w.astype(np.float64), X.astype(np.float64), Y.astype(np.float64))
    assert abs(L - Lo) <= 1e-5 * Lo
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    assert rel < 2e-5, rel
    # every block of the parameter vector, on its own scale
    for lo, hi in ((mc.OFF_W1, mc.OFF_B1), (mc.OFF_B1, mc.OFF_W2), (mc.OFF_W2, mc.OFF_B2), (mc.OFF_B2, mc.OFF_W3),
                   (mc.OFF_W3, mc.OFF_B3), (mc.OFF_B3, mc.PARAMS)):
        assert np.max(np.abs(g[lo:hi] - go[lo:hi])) <= 1e-4 * np.max(np.abs(go[lo:hi])) + 1e-12


def test_grad_rounds_weights_to_bf16(bs, orc):
    b, s = bs
    w = mc.random_net(3).astype(np.float32)
    rng = np.random.default_rng(4)
    X = rng.normal(0.0, 1.0, (200, 9)).astype(np.float32)
    Y = rng.normal(0.0, 0.5, 200).astype(np.float32)
    g, L = s.mlp_grad(w, X, Y)
    Lo = mlp.loss(_bf16(orc, w), X.astype(np.float64), Y.astype(np.float64))
    assert abs(L - Lo) <= 1e-5 * Lo


def _kur(n, seed, t1=8.0):
    return workloads.kuramoto(n, seed=seed, t1=t1)


def _gpu_solve(s, w, rtol, net=None, trace=True):
    s.set_workload(w)
    if net is None:
        s.set_controller(0)
    else:
        s.set_controller(1, net)
    s.set_options(trace=1 if trace else 0, trace_cap=1 << 18)
    y, st = s.solve(w["y0"], 0.0, w["t1"], rtol)
    tr = s.trace() if trace else None
    s.set_options(trace=0)
    s.set_controller(0)
    return y, st, tr


@pytest.mark.parametrize("which", ["constant", "controller"])
def test_learned_solve_matches_oracle(bs, orc, which):
    b, s = bs
    rtol = 1e-7
    w = _kur(300, 2201, t1=8.0)
    net = mc.constant_net(math.log(1.08)) if which == "constant" else mc.controller_net()
    netq = _bf16(orc, net)
    say(f"[mlp solve] {which} kuramoto n=300 rtol={rtol}")
    y, st, tr = _gpu_solve(s, w, rtol, netq.astype(np.float32))
    yo, sto, tro = orc.bs32_solve(w["kind"], w["n"], w["y0"], 0.0, w["t1"], rtol, A=w["A"], param=w["param"],
                                  gain=w["gain"], trace_cap=1 << 18, mlp_w=netq)
    assert st["status"] == 0 and sto["status"] == 0
    assert np.all(tr["err"][tr["accepted"] == 1] < rtol)
    assert tr["proposer"].sum() > 0.5 * len(tr)
    assert st["n_learned"] == tr["proposer"].sum()
    assert abs(st["n_accept"] - sto["n_accept"]) <= 0.01 * sto["n_accept"]
    rel = np.linalg.norm(y - yo) / np.linalg.norm(yo)
    say(f"   accepted {st['n_accept']} / {sto['n_accept']}, proposer {tr['proposer'].sum()}, rel {rel:.2e}")
    if which == "constant":
        # the proposal is the same double on both sides: the same attempts; steps differ
        # only through the classical rule after a rejection, which sees E with the
        # rounding of the stage sums (E is a difference of nearly equal solutions)
        assert len(tr) == len(tro)
        np.testing.assert_array_equal(tr["proposer"], tro["proposer"])
        np.testing.assert_array_equal(tr["accepted"], tro["accepted"])
        np.testing.assert_allclose(tr["h"], tro["h"], rtol=1e-8)
    assert rel < 1e-10


def test_set_controller_errors(bs):
    b, s = bs
    w = _kur(64, 2202)
    s.set_workload(w)
    with pytest.raises(ValueError):   # the binding checks the count ...
        s.set_controller(1, np.zeros(10, dtype=np.float32))
    short = np.zeros(10, dtype=np.float32)   # ... and so does the library
    assert b.lib().bs32_set_controller(s._ctx, 1, short.ctypes.data, short.size) == b.EINVAL
    assert b.lib().bs32_set_controller(s._ctx, 1, None, b.MLP_PARAMS) == b.EINVAL
    bad = mc.constant_net(0.0).astype(np.float32)
    bad[5] = np.nan
    with pytest.raises(b.BS32Error):
        s.set_controller(1, bad)
    with pytest.raises(b.BS32Error):
        s.set_controller(2, mc.constant_net(0.0))
    # a standard solve afterwards is unaffected
    y, st = s.solve(w["y0"], 0.0, 1.0, 1e-7)
    assert st["status"] == 0


def _training_set(b, s, seeds, rtols, n=256, t1=8.0):
    F, Y = [], []
    for sd in seeds:
        w = _kur(n, sd, t1=t1)
        for rtol in rtols:
            _, st, tr = _gpu_solve(s, w, rtol)
            f, y = b.mlp_features(tr, rtol)
            F.append(f)
            Y.append(y)
    return np.concatenate(F), np.concatenate(Y)


def test_training_reduces_loss_and_exports_the_trained_network(bs, orc):
    b, s = bs
    say("[mlp train] traces")
    F, Y = _training_set(b, s, [2301, 2302], [1e-6, 1e-8])
    say(f"[mlp train] {len(F)} samples")
    assert len(F) > 500
    W, losses = s.mlp_train(F, Y, epochs=30, batch=128, lr=1e-3, seed=9)
    say(f"   loss {losses[0]:.4g} -> {losses[-1]:.4g}")
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.5 * losses[0]
    # the exported vector carries its standardization: on raw features it is the trained network
    _, L = s.mlp_grad(W, F, Y)
    assert abs(L - losses[-1]) <= 1e-6 * losses[-1]
    Lo = mlp.loss(_bf16(orc, W), F.astype(np.float64), Y.astype(np.float64))
    assert abs(L - Lo) <= 1e-3 * Lo
    mu, isd = W[mc.OFF_MU:mc.OFF_MU + 9], W[mc.OFF_ISD:mc.OFF_ISD + 9]
    np.testing.assert_allclose(mu, F.astype(np.float64).mean(axis=0), rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(1.0 / isd, F.astype(np.float64).std(axis=0), rtol=1e-4)
    # same seed, same weights
    W2, losses2 = s.mlp_train(F, Y, epochs=30, batch=128, lr=1e-3, seed=9)
    np.testing.assert_array_equal(W, W2)


def test_learned_solve_of_trained_network(bs, orc):
    """A trained proposer, deployed: E alone decides, the result stays within the
    tolerance-level distance of the standard solve, the oracle agrees."""
    b, s = bs
    F, Y = _training_set(b, s, [2311, 2312], [1e-6, 1e-7, 1e-8])
    W, losses = s.mlp_train(F, Y, epochs=40, batch=128, lr=1e-3, seed=3)
    rtol = 1e-7
    w = _kur(256, 2399)
    y0, st0, _ = _gpu_solve(s, w, rtol)
    y1, st1, tr = _gpu_solve(s, w, rtol, W)
    say(f"[mlp deploy] fev standard {st0['n_fev']} learned {st1['n_fev']}; "
        f"rejects {st0['n_reject']} / {st1['n_reject']}; proposer {tr['proposer'].mean():.2f}")
    assert st1["status"] == 0
    assert np.all(tr["err"][tr["accepted"] == 1] < rtol)
    assert np.max(np.abs(y1 - y0)) < 1e-4
    yo, sto, _ = orc.bs32_solve(w["kind"], w["n"], w["y0"], 0.0, w["t1"], rtol, A=w["A"], param=w["param"],
                                gain=w["gain"], mlp_w=_bf16(orc, W))
    assert abs(st1["n_accept"] - sto["n_accept"]) <= 0.01 * sto["n_accept"] + 1
    assert np.linalg.norm(y1 - yo) / np.linalg.norm(yo) < 1e-9


def test_ensemble_with_learned_proposer_matches_single(bs):
    b, s = bs
    ws = [_kur(int(n), 2400 + q, t1=3.0) for q, n in enumerate([100, 257, 64, 700])]
    net = mc.controller_net().astype(np.float32)
    s.set_options(tile=2)
    try:
        s.set_ensemble(ws)
        s.set_controller(1, net)
        y, st, _ = s.solve_batch(np.concatenate([w["y0"] for w in ws]), 0.0, 3.0, 1e-7)
        s.set_controller(0)
        assert np.all(st == 0)
        single = b.Solver(0)
        single.set_options(tile=2)
        off = 0
        for q, w in enumerate(ws):
            single.set_workload(w)
            single.set_controller(1, net)
            ys, sts = single.solve(w["y0"], 0.0, 3.0, 1e-7)
            m = w["n"]
            np.testing.assert_array_equal(y[off:off + m], ys)
            bst = s.batch_stats(q)
            assert bst["n_accept"] == sts["n_accept"] and bst["n_reject"] == sts["n_reject"]
            off += m
        single.close()
    finally:
        s.set_options(tile=-1)


def _safety_traces(b, s, seeds, rtols, n=384, t1=10.0):
    """Traces at three controller safety factors, so that the features cover steps on
    both sides of the classical choice (the labels are the steps that would have put
    the next estimate at 0.8 Rel)."""
    F, Y = [], []
    for sd in seeds:
        w = _kur(n, sd, t1=t1)
        s.set_workload(w)
        for rtol in rtols:
            for safety in (0.75, 0.9, 0.97):
                s.set_options(trace=1, trace_cap=1 << 18, safety=safety)
                s.solve(w["y0"], 0.0, t1, rtol)
                f, y = b.mlp_features(s.trace(), rtol)
                F.append(f)
                Y.append(y)
    s.set_options(trace=0, safety=0.9)
    return np.concatenate(F), np.concatenate(Y)


def test_trained_proposer_saves_evaluations_on_held_out_system(bs, orc):
    """Trained on traces of two Kuramoto systems, the proposer solves a held-out one
    (another seed and size) with fewer RHS evaluations than the standard controller,
    at a final error within 2x of the standard controller's against the oracle's
    Dormand-Prince 5(4) solution at rtol 1e-12; the estimate alone decides acceptance."""
    b, s = bs
    F, Y = _safety_traces(b, s, [2501, 2502], [1e-6, 1e-7, 1e-8])
    W, losses = s.mlp_train(F, Y, epochs=40, batch=256, lr=1e-3, seed=5)
    say(f"[mlp gain] {len(F)} samples, loss {losses[0]:.3g} -> {losses[-1]:.3g}")
    rtol = 1e-7
    w = _kur(640, 2599, t1=20.0)
    y0, st0, _ = _gpu_solve(s, w, rtol)
    y1, st1, tr = _gpu_solve(s, w, rtol, W)
    ref, rst = orc.dp54_solve(w["kind"], w["n"], w["y0"], 0.0, w["t1"], 1e-12, A=w["A"], param=w["param"],
                              gain=w["gain"], i_max=10_000_000)
    assert rst["status"] == 0
    e0 = np.linalg.norm(y0 - ref) / math.sqrt(w["n"])
    e1 = np.linalg.norm(y1 - ref) / math.sqrt(w["n"])
    say(f"[mlp gain] RHS evaluations standard {st0['n_fev']} learned {st1['n_fev']} "
        f"({100.0 * (1.0 - st1['n_fev'] / st0['n_fev']):.1f} % fewer); rejected {st0['n_reject']} / {st1['n_reject']}; "
        f"steps chosen by the network {st1['n_learned']}; error {e0:.3e} / {e1:.3e}")
    assert st0["status"] == 0 and st1["status"] == 0
    assert st1["n_learned"] > 0
    assert np.all(tr["err"][tr["accepted"] == 1] < rtol)
    assert st1["n_fev"] < st0["n_fev"]
    assert e1 <= 2.0 * e0

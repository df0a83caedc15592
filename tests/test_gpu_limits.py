"""The wall-clock failure conditions of Sec. 2.2 (a time limit, and a slow-solver
limit when less than 10 % of the interval is done), forced from the host with
tiny limits so that every kernel exits normally.  The host checks the clock
between chunks of attempts, so the chunk already in flight still runs: the
solve then returns the last accepted state, and the statistics report the time
and the counts it reached."""
import sys

import numpy as np
import pytest

import workloads

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


@pytest.mark.parametrize("which", ["timeout", "too_slow"])
def test_single_solve_wall_clock_limit(bs, which):
    import torch
    b, s = bs
    w = workloads.kuramoto(512, seed=81, t1=200.0)
    say(f"[wall-clock limit] {which} kuramoto n=512 t=[0,200]")
    s.set_workload(w)
    rec = torch.zeros((256, w["n"]), dtype=torch.float64, device="cuda")
    s.set_record(rec)
    if which == "timeout":
        s.set_options(time_limit_s=1e-9, slow_limit_s=0.0)
        want = b.TIMEOUT
    else:
        s.set_options(time_limit_s=0.0, slow_limit_s=1e-9)
        want = b.TOO_SLOW
    try:
        y, st = s.solve(w["y0"], 0.0, 200.0, 1e-6)
    finally:
        s.set_options(time_limit_s=5400.0, slow_limit_s=2700.0)
        s.set_record(None)
    say(f"   status {st['status']} t_reached {st['t_reached']:.4g} accepted {st['n_accept']} rejected {st['n_reject']}")
    assert st["status"] == want
    assert 0.0 < st["t_reached"] < 0.1 * 200.0
    assert 1 <= st["n_accept"] <= 255 and st["n_accept"] + st["n_reject"] <= 2 + 2 * 64
    # y_out is the state after the last accepted step, as the record holds it
    last = rec[st["n_accept"]].cpu().numpy()
    assert np.array_equal(y, last)
    assert np.all(rec[st["n_accept"] + 1:].cpu().numpy() == 0.0)
    # and the solve continues from there to the same place as an unlimited run would go
    y2, st2 = s.solve(w["y0"], 0.0, 200.0, 1e-6)
    assert st2["status"] == 0 and st2["t_reached"] == 200.0


def test_batch_wall_clock_limit(bs):
    b, s = bs
    ws = [workloads.kuramoto(int(n), seed=90 + q, t1=100.0) for q, n in enumerate((200, 350, 128, 512))]
    say("[wall-clock limit] batch of 4")
    s.set_ensemble(ws)
    y0 = np.concatenate([w["y0"] for w in ws])
    s.set_options(time_limit_s=1e-9)
    try:
        y, st, tot = s.solve_batch(y0, 0.0, np.full(4, 100.0), 1e-6)
    finally:
        s.set_options(time_limit_s=5400.0)
    say(f"   statuses {list(st)}")
    assert np.all(st == b.TIMEOUT)
    for q in range(4):
        bst = s.batch_stats(q)
        assert bst["status"] == b.TIMEOUT and 0.0 < bst["t_reached"] < 100.0
    assert np.all(np.isfinite(y))

"""GPU tests of the accuracy diagnostics: the solution record of a solve, the
analytic flow of the coupled linear oscillators (paper Benchmark 1, eq. (LCO))
and the real local error of eq. (LCO-Local-Error), against the oracle's closed
form (oracle/lco.py) on the same inputs.
"""
import ctypes as C
import math
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


def _accepted_h(tr):
    return np.array([r["h"] for r in tr if r["accepted"] == 1])


@pytest.mark.parametrize("n", [1, 3, 257, 1000])
def test_flow_matches_oracle(bs, n):
    import torch
    from oracle import lco
    b, s = bs
    rng = np.random.default_rng(300 + n)
    count = 5
    X = rng.uniform(0.0, 2.0, (count, 2 * n))
    h = np.array([0.0, 1e-3, 0.3, 2.5, 40.0])
    say(f"[lco flow] n={n}")
    out = s.lco_flow(n, torch.from_numpy(X.reshape(-1)).cuda(), torch.from_numpy(h).cuda()).cpu().numpy()
    ref = np.concatenate([lco.lco_flow(X[k], h[k]) for k in range(count)])
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-14)


def _recorded_solve(b, s, w, mode, rtol, cap=None):
    import torch
    n = w["n"]
    s.set_workload(w)
    s.set_options(trace=1, trace_cap=1 << 17)
    cap = cap or 20000
    rec = torch.full((cap * 2 * n,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()  # the fill is done before the library's stream writes the record
    s.set_record(rec)
    try:
        y, st = s.solve(w["y0"], 0.0, w["t1"], rtol, mode=mode)
        tr = s.trace()
    finally:
        s.set_record(None)
        s.set_options(trace=0)
    return rec, y, st, tr


def test_record_holds_the_trajectory(bs):
    b, s = bs
    w = workloads.lco_paper(200, seed=1301, t1=3.0)
    rec, y, st, tr = _recorded_solve(b, s, w, b.PREC_FP64, 1e-6)
    assert st["status"] == 0
    na = st["n_accept"]
    R = rec.cpu().numpy().reshape(-1, 400)
    np.testing.assert_array_equal(R[0], w["y0"])
    np.testing.assert_array_equal(R[na], y)
    assert np.all(np.isfinite(R[: na + 1])) and np.all(np.isnan(R[na + 1:]))
    assert len(_accepted_h(tr)) == na


def test_record_capacity_and_single_rounding(bs):
    b, s = bs
    w = workloads.lco_paper(64, seed=1302, t1=3.0)
    rec, y, st, _ = _recorded_solve(b, s, w, b.PREC_PAPER_SINGLE, 1e-5, cap=7)
    assert st["status"] == 0 and st["n_accept"] > 7
    R = rec.cpu().numpy().reshape(7, 128)
    assert np.all(np.isfinite(R))
    # the Single recipe holds its state in FP32 from the start
    np.testing.assert_array_equal(R[0], w["y0"].astype(np.float32).astype(np.float64))
    # a solve without a record leaves the buffer alone and gives the same answer
    y2, st2 = s.solve(w["y0"], 0.0, 3.0, 1e-5, mode=b.PREC_PAPER_SINGLE)
    np.testing.assert_array_equal(y2, y)


@pytest.mark.parametrize("mode", [0, 5, 6, 7])
def test_local_error_matches_oracle(bs, mode):
    import torch
    from oracle import lco
    b, s = bs
    n = 300
    w = workloads.lco_paper(n, seed=1303, t1=4.0)
    rtol = 1e-7
    rec, y, st, tr = _recorded_solve(b, s, w, mode, rtol)
    assert st["status"] == 0
    na = st["n_accept"]
    h = _accepted_h(tr)
    say(f"[lco local error] mode {mode}: {na} steps")
    err = s.lco_local_error(n, rec, torch.from_numpy(h).cuda(), 1.0).cpu().numpy()
    R = rec.cpu().numpy().reshape(-1, 2 * n)
    ref = np.array([lco.lco_local_error(R[k], R[k + 1], h[k], 1.0) for k in range(na)])
    assert np.all(np.abs(err - ref) <= 1e-13 + 1e-6 * ref), float(np.max(np.abs(err - ref)))
    E_bs = np.array([r["err"] for r in tr if r["accepted"] == 1])
    assert np.all(E_bs < rtol)


def test_single_real_error_plateaus_above_the_tolerance(bs):
    """Sec. 3 (fig. LCO-Local-Error-Comp): at a strict tolerance the estimate of
    every solver stays below Rel, but Single's real local error does not, while
    FP64's and Mixed2's do."""
    import torch
    b, s = bs
    n = 200
    w = workloads.lco_paper(n, seed=1304, t1=3.0)
    rtol = 1e-9
    mean = {}
    for mode in (0, 5, 7):
        rec, y, st, tr = _recorded_solve(b, s, w, mode, rtol)
        assert st["status"] == 0
        h = _accepted_h(tr)
        err = s.lco_local_error(n, rec, torch.from_numpy(h).cuda(), 1.0).cpu().numpy()
        mean[mode] = (float(np.mean(err)), float(np.mean([r["err"] for r in tr if r["accepted"] == 1])))
    say(f"[lco real vs estimate] {mean}")
    assert mean[5][0] > 10.0 * rtol and mean[5][1] < rtol
    assert mean[0][0] < rtol and mean[7][0] < 3.0 * rtol


def test_diagnostic_arguments(bs):
    import torch
    b, s = bs
    L = b.lib()
    w = workloads.lco_paper(16, seed=1305, t1=1.0)
    s.set_workload(w)
    host = np.zeros(64)
    assert L.bs32_set_record(s._ctx, host.ctypes.data, 2) == b.EINVAL
    assert L.bs32_set_record(s._ctx, None, -1) == b.EINVAL
    d = torch.zeros(64, dtype=torch.float64, device="cuda")
    hh = torch.ones(1, dtype=torch.float64, device="cuda")
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    assert L.bs32_lco_local_error(s._ctx, 16, 1, d.data_ptr(), hh.data_ptr(), 0.0, e.data_ptr()) == b.EINVAL
    assert L.bs32_lco_local_error(s._ctx, 0, 1, d.data_ptr(), hh.data_ptr(), 1.0, e.data_ptr()) == b.EINVAL
    assert L.bs32_lco_flow(s._ctx, 16, 1, host.ctypes.data, hh.data_ptr(), d.data_ptr()) == b.EINVAL
    assert L.bs32_lco_flow(s._ctx, 16, 0, None, None, None) == b.OK
    # a non-finite state reads as NaN, not as a small error
    d[3] = float("nan")
    torch.cuda.synchronize()
    assert L.bs32_lco_local_error(s._ctx, 16, 1, d.data_ptr(), hh.data_ptr(), 1.0, e.data_ptr()) == b.OK
    assert math.isnan(float(e[0]))
    # an ensemble context has no single-system record
    s.set_ensemble([workloads.lco_paper(16, seed=1306), workloads.lco_paper(8, seed=1307)])
    dd = torch.zeros(64, dtype=torch.float64, device="cuda")
    assert L.bs32_set_record(s._ctx, C.c_void_p(dd.data_ptr()), 2) == b.ESTATE

"""GPU parity of the FP64 path against the CPU oracle, through the C ABI.

Right-hand sides are compared element by element (relative to the sum of the
absolute pair terms, the scale of FP64 summation-order differences); solves
are compared at t_end with the ℓ2-relative bar 1e-10 and accepted-step counts
within 1 %.
"""
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


def _pair_scale(w):
    """sum_j |A_ij| * (|v_j| + |v_i|) scale of the coupling sum, per row (FP64 rounding scale)."""
    A = np.abs(w["A"]) if w["A"] is not None else np.ones((w["n"], w["n"]))
    d = workloads.DIM[w["kind"]]
    x = w["y0"][0::d]
    v = np.ones_like(x) if w["kind"] == workloads.KURAMOTO else np.abs(x)
    return (A @ v + A.sum(1) * np.abs(x)) / w["n"] * max(1.0, abs(w["gain"]))


CASES = [
    ("osc2", lambda: workloads.osc2(300, seed=11)),
    ("kuramoto", lambda: workloads.kuramoto(1000, seed=12)),
    ("goodwin3", lambda: workloads.goodwin3(333, seed=13)),
    ("lco_paper", lambda: workloads.lco_paper(257, seed=14)),
    ("kuramoto_n1", lambda: workloads.kuramoto(1, seed=15)),
    ("osc2_n4097", lambda: workloads.osc2(4097, seed=16)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_rhs_fp64_matches_oracle(bs, orc, name, make):
    b, s = bs
    w = make()
    say(f"[rhs fp64] {name} n={w['n']}")
    s.set_workload(w)
    f = s.rhs(w["y0"])
    ref = orc.rhs(w["kind"], w["n"], w["y0"], A=w["A"], param=w["param"], gain=w["gain"])
    d = workloads.DIM[w["kind"]]
    tol = 1e-14 * np.repeat(_pair_scale(w), d) + 1e-15 * np.abs(ref)
    assert np.all(np.abs(f - ref) <= tol + 1e-300), np.max(np.abs(f - ref) / (tol + 1e-300))


SOLVES = [
    ("osc2_n256_cfg1", lambda: workloads.osc2(256, seed=1000, t1=10.0, rtol=1e-6)),
    ("kuramoto_n600", lambda: workloads.kuramoto(600, seed=21, t1=10.0, rtol=1e-7)),
    ("goodwin3_n300", lambda: workloads.goodwin3(300, seed=22, t1=60.0, rtol=1e-6)),
    ("lco_paper_n200", lambda: workloads.lco_paper(200, seed=23, t1=10.0, rtol=1e-8)),
    ("osc2_n1_tight", lambda: workloads.osc2(1, seed=24, t1=10.0, rtol=1e-10)),
]


@pytest.mark.parametrize("name,make", SOLVES, ids=[c[0] for c in SOLVES])
def test_solve_fp64_matches_oracle(bs, orc, name, make):
    b, s = bs
    w = make()
    say(f"[solve fp64] {name} n={w['n']}")
    s.set_workload(w)
    y, st = s.solve(w["y0"], w["t0"], w["t1"], w["rtol"], w["atol"])
    ref, rst, _ = orc.bs32_solve(w["kind"], w["n"], w["y0"], w["t0"], w["t1"], w["rtol"], w["atol"], A=w["A"],
                                 param=w["param"], gain=w["gain"])
    assert st["status"] == 0 and rst["status"] == 0
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    say(f"   rel l2 {rel:.3e}  accepted gpu {st['n_accept']} cpu {rst['n_accept']}  rejected {st['n_reject']}/{rst['n_reject']}")
    assert rel <= 1e-10
    assert abs(st["n_accept"] - rst["n_accept"]) <= max(1, 0.01 * rst["n_accept"])
    assert st["t_reached"] == w["t1"]
    assert st["n_fev"] == 2 + 3 * (st["n_accept"] + st["n_reject"])


def test_solve_is_bitwise_reproducible(bs):
    b, s = bs
    w = workloads.kuramoto(2048, seed=31, t1=2.0, rtol=1e-6)
    say("[determinism] kuramoto n=2048 x3")
    s.set_workload(w)
    outs = [s.solve(w["y0"], 0.0, 2.0, 1e-6)[0] for _ in range(3)]
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


def test_graph_and_stream_launch_agree(bs):
    b, s = bs
    w = workloads.osc2(512, seed=32, t1=3.0)
    say("[graph vs stream] osc2 n=512")
    s.set_workload(w)
    y1, st1 = s.solve(w["y0"], 0.0, 3.0, 1e-7)
    s.set_options(use_graph=0)
    try:
        y2, st2 = s.solve(w["y0"], 0.0, 3.0, 1e-7)
    finally:
        s.set_options(use_graph=1)
    assert np.array_equal(y1, y2) and st1["n_accept"] == st2["n_accept"]


def test_stats_name_the_tile_and_kernel(bs):
    b, s = bs
    w = workloads.kuramoto(300, seed=34, t1=0.5)
    s.set_workload(w)
    for mode, prefix in ((0, "k_contract_f64<2, "), (2, "k_contract_mfma<2, 2, 2, "), (4, "k_contract_mfma<4, 2, 3, ")):
        _, st = s.solve(w["y0"], 0.0, 0.5, 1e-6, mode=mode)
        assert st["tile"] >= 0 and st["n_learned"] == 0
        assert s.kernel_name(mode, st["tile"]).startswith(prefix)
    s.set_options(tile=3)
    try:
        _, st = s.solve(w["y0"], 0.0, 0.5, 1e-6)
        assert st["tile"] == 3
    finally:
        s.set_options(tile=-1)
    with pytest.raises(b.BS32Error):
        s.kernel_name(0, 10_000)


def test_device_pointers(bs):
    import torch
    b, s = bs
    w = workloads.kuramoto(700, seed=33, t1=1.0)
    say("[device pointers] kuramoto n=700")
    A = torch.from_numpy(w["A"]).cuda()
    p = torch.from_numpy(w["param"]).cuda()
    y0 = torch.from_numpy(w["y0"]).cuda()
    # same tile both times: the autotuner may pick another split of k, which
    # changes the FP64 summation order
    s.set_options(tile=0)
    try:
        s.set_system(w["kind"], w["n"], A, p, w["gain"])
        out = torch.empty_like(y0)
        s.solve(y0, 0.0, 1.0, 1e-6, out=out)
        s.set_workload(w)
        y_h, _ = s.solve(w["y0"], 0.0, 1.0, 1e-6)
    finally:
        s.set_options(tile=-1)
    assert np.array_equal(out.cpu().numpy(), y_h)


def test_zero_interval_and_errors(bs):
    b, s = bs
    w = workloads.osc2(64, seed=34)
    say("[edge cases] osc2 n=64")
    s.set_workload(w)
    y, st = s.solve(w["y0"], 2.0, 2.0, 1e-6)
    assert np.array_equal(y, w["y0"]) and st["n_fev"] == 0
    with pytest.raises(b.BS32Error):
        s.solve(w["y0"], 2.0, 1.0, 1e-6)
    with pytest.raises(b.BS32Error):
        s.solve(w["y0"], 0.0, 1.0, 0.0)
    with pytest.raises(b.BS32Error):
        s.solve(w["y0"], 0.0, 1.0, 1e-6, mode=11)


def test_failure_codes_match_oracle(bs, orc):
    b, s = bs
    w = workloads.kuramoto(24, seed=21, t1=5.0)
    say("[failure codes] kuramoto n=24")
    s.set_workload(w)
    s.set_options(i_max=10)
    try:
        y, st = s.solve(w["y0"], 0.0, 5.0, 1e-9)
        ref, rst, _ = orc.bs32_solve(3, 24, w["y0"], 0.0, 5.0, 1e-9, A=w["A"], param=w["param"], gain=2.0, i_max=10)
        assert st["status"] == b.MAX_STEPS == rst["status"]
        assert st["n_accept"] + st["n_reject"] == 11
        assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-12
        s.set_options(i_max=10, h0=1e8, h_max=1e9)
        y, st = s.solve(w["y0"], 0.0, 1e9, 1e-9)
        assert st["status"] == b.MAX_REJECTS and st["n_reject"] == 9
        assert np.array_equal(y, w["y0"])
    finally:
        s.set_options(i_max=100000, h0=0.0, h_max=0.0)
    y0 = w["y0"].copy()
    y0[5] = math.nan
    y, st = s.solve(y0, 0.0, 5.0, 1e-6)
    assert st["status"] == b.NONFINITE


def test_trace_records(bs):
    b, s = bs
    w = workloads.kuramoto(256, seed=41, t1=5.0)
    say("[trace] kuramoto n=256")
    s.set_workload(w)
    s.set_options(trace=1, trace_cap=4096)
    try:
        y, st = s.solve(w["y0"], 0.0, 5.0, 1e-7)
        tr = s.trace()
    finally:
        s.set_options(trace=0)
    assert len(tr) == st["n_accept"] + st["n_reject"]
    acc = tr["accepted"] == 1
    assert np.all(tr["err"][acc] < 1e-7) and np.all(tr["err"][~acc] >= 1e-7)
    assert abs(tr["h"][acc].sum() - 5.0) < 1e-12

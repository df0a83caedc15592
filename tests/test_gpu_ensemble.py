"""GPU tests of the batched ensemble path (grouped launches over many instances).

Each instance of a batch must equal the single-system GPU solve of the same
instance bit for bit when both use the same contraction tile (same kernels,
same summation order), and match the oracle at the FP64 parity bar.
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


def _members(B, seed, t1=2.0, kind="kuramoto"):
    g = np.random.default_rng(seed)
    ns = g.integers(33, 700, B)
    ws = []
    for q, n in enumerate(ns):
        if kind == "kuramoto":
            ws.append(workloads.kuramoto(int(n), seed=seed * 100 + q, K=float(g.uniform(0.5, 4.0)), t1=t1))
        else:
            ws.append(workloads.osc2(int(n), seed=seed * 100 + q, t1=t1))
    return ws


@pytest.mark.parametrize("kind", ["kuramoto", "osc2"])
def test_batch_fp64_matches_oracle_and_single(bs, orc, kind):
    b, s = bs
    ws = _members(9, 5 if kind == "kuramoto" else 6, kind=kind)
    t1 = np.array([w["t1"] for w in ws])
    t1[3] = 0.0  # empty interval: returns y0
    t1[5] = 0.7
    say(f"[batch fp64] {kind} B={len(ws)} n={[w['n'] for w in ws]}")
    s.set_options(tile=2)
    try:
        s.set_ensemble(ws)
        y0 = np.concatenate([w["y0"] for w in ws])
        y, st, tot = s.solve_batch(y0, 0.0, t1, 1e-7)
        assert np.all(st == 0)
        off = 0
        single = b.Solver(0)
        single.set_options(tile=2)
        for q, w in enumerate(ws):
            m = w["y0"].size
            yq = y[off:off + m]
            off += m
            bst = s.batch_stats(q)
            if t1[q] == 0.0:
                assert np.array_equal(yq, w["y0"]) and bst["n_fev"] == 0
                continue
            ref, rst, _ = orc.bs32_solve(w["kind"], w["n"], w["y0"], 0.0, t1[q], 1e-7, A=w["A"],
                                         param=w["param"], gain=w["gain"])
            rel = np.linalg.norm(yq - ref) / np.linalg.norm(ref)
            assert rel <= 1e-10, (q, rel)
            assert abs(bst["n_accept"] - rst["n_accept"]) <= max(1, 0.01 * rst["n_accept"])
            single.set_workload(w)
            ys, sst = single.solve(w["y0"], 0.0, t1[q], 1e-7)
            assert np.array_equal(ys, yq), q
            assert sst["n_accept"] == bst["n_accept"] and sst["n_reject"] == bst["n_reject"]
        single.close()
        assert tot["n_fev"] == sum(s.batch_stats(q)["n_fev"] for q in range(len(ws)))
    finally:
        s.set_options(tile=-1)


@pytest.mark.parametrize("mode", [1, 2, 4])
def test_batch_reduced_equals_single(bs, mode):
    b, s = bs
    ws = _members(6, 7)
    say(f"[batch mode {mode}] kuramoto B=6")
    s.set_options(tile=1)
    try:
        s.set_ensemble(ws)
        y, st, _ = s.solve_batch(np.concatenate([w["y0"] for w in ws]), 0.0, 1.0, 1e-6, mode=mode)
        assert np.all(st == 0)
        single = b.Solver(0)
        single.set_options(tile=1)
        off = 0
        for w in ws:
            m = w["y0"].size
            single.set_workload(w)
            ys, _ = single.solve(w["y0"], 0.0, 1.0, 1e-6, mode=mode)
            assert np.array_equal(ys, y[off:off + m])
            off += m
        single.close()
    finally:
        s.set_options(tile=-1)


@pytest.mark.parametrize("mode", [0, 1, 2, 4])
def test_batch_every_tile_tracks_oracle(bs, orc, mode):
    """Every grouped contraction tile, forced one by one: a short batch solve of
    instances of ragged N against the oracle's solve in the same storage mode (a
    tile that left rows or operand columns unfinished would fail it)."""
    b, s = bs
    ws = _members(4, 11, t1=0.3)
    refs = [orc.bs32_solve(w["kind"], w["n"], w["y0"], 0.0, 0.3, 1e-6, A=w["A"], param=w["param"],
                           gain=w["gain"], mode=mode)[0] for w in ws]
    y0 = np.concatenate([w["y0"] for w in ws])
    bar = 1e-10 if mode == 0 else 2e-5
    s.set_ensemble(ws)
    k, checked = 0, 0
    try:
        while True:
            s.set_options(tile=k)
            say(f"[batch tile] mode {mode} tile {k}")
            try:
                y, st, _ = s.solve_batch(y0, 0.0, 0.3, 1e-6, mode=mode)
            except b.BS32Error as e:
                if e.code == b.EUNSUPPORTED:  # single-system tile (epilogue wave)
                    k += 1
                    continue
                assert e.code == b.EINVAL and k > 0  # past the last candidate
                break
            assert np.all(st == 0), k
            off = 0
            for w, ref in zip(ws, refs):
                m = w["y0"].size
                rel = np.linalg.norm(y[off:off + m] - ref) / np.linalg.norm(ref)
                assert rel <= bar, (k, w["n"], rel)
                off += m
            k += 1
            checked += 1
    finally:
        s.set_options(tile=-1)
    assert checked >= 8


# (mode, tile index) pairs with four-wave tiles: FP64 (1,4,1,4) and (4,2,2,2, non-temporal);
# FP32 matrix cores (2,4,1,4, non-temporal); BF16 (2,4,1,2, non-temporal) and (1,4,1,4)
PERSISTENT_CASES = [(0, 0), (0, 13), (1, 25), (2, 20), (2, 17), (3, 16), (4, 16), (4, 20)]


@pytest.mark.parametrize("mode,tile", PERSISTENT_CASES)
def test_persistent_launch_equals_grouped(bs, mode, tile):
    """One persistent launch per chunk of attempts (instances claim their own row tiles
    and finalize slices from device counters) gives every instance exactly the result
    of the grouped launches: same kernels, same summation order, same decisions."""
    b, s = bs
    ws = _members(9, 12, t1=1.2)
    t1 = np.array([w["t1"] for w in ws])
    t1[2] = 0.0   # empty interval
    t1[4] = 0.35  # finishes early
    t1[7] = 0.8
    y0 = np.concatenate([w["y0"] for w in ws])
    say(f"[persistent] mode {mode} tile {tile} n={[w['n'] for w in ws]}")
    out = {}
    try:
        s.set_ensemble(ws)
        for launch in (0, 1):
            s.set_options(tile=tile, ensemble_launch=launch)
            y, st, tot = s.solve_batch(y0, 0.0, t1, 1e-6, mode=mode)
            assert np.all(st == 0), (launch, st)
            out[launch] = (y, [s.batch_stats(q) for q in range(len(ws))], tot)
    finally:
        s.set_options(tile=-1, ensemble_launch=0)
    assert np.array_equal(out[0][0], out[1][0])
    for q in range(len(ws)):
        g, p = out[0][1][q], out[1][1][q]
        assert (g["n_accept"], g["n_reject"], g["n_fev"]) == (p["n_accept"], p["n_reject"], p["n_fev"]), q
    assert out[0][2]["n_fev"] == out[1][2]["n_fev"]


@pytest.mark.parametrize("mode,tile", [(1, 25), (0, 13)])
def test_persistent_launch_large_instances(bs, mode, tile):
    """Instances large enough that a stage spans several tasks (runs of row tiles of
    about 4 MB) and the finalize several runs of slices, mixed with small ones: the
    persistent launch still equals the grouped launches bit for bit."""
    b, s = bs
    g = np.random.default_rng(14)
    ns = [8192, 33, 4100, 700, 2500, 64, 8191, 300]
    ws = [workloads.kuramoto(n, seed=1400 + q, K=float(g.uniform(0.5, 4.0)), t1=0.15) for q, n in enumerate(ns)]
    y0 = np.concatenate([w["y0"] for w in ws])
    say(f"[persistent large] mode {mode} tile {tile} n={ns}")
    out = {}
    try:
        s.set_ensemble(ws)
        for launch in (0, 1):
            s.set_options(tile=tile, ensemble_launch=launch)
            y, st, _ = s.solve_batch(y0, 0.0, 0.15, 1e-6, mode=mode)
            assert np.all(st == 0), (launch, st)
            out[launch] = (y, [s.batch_stats(q)["n_fev"] for q in range(len(ws))])
    finally:
        s.set_options(tile=-1, ensemble_launch=0)
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


def test_persistent_launch_learned_controller(bs):
    """The learned proposer runs inside the finalize tasks of the persistent launch
    (one workgroup's forward pass per finalize slice) exactly as in the grouped
    finalize launch: same steps, same solutions."""
    from tests import mlp_cases as mc
    b, s = bs
    ws = _members(6, 15, t1=1.0)
    y0 = np.concatenate([w["y0"] for w in ws])
    say(f"[persistent learned] n={[w['n'] for w in ws]}")
    out = {}
    try:
        s.set_ensemble(ws)
        s.set_controller(1, mc.random_net(5, scale=0.3))
        for launch in (0, 1):
            s.set_options(tile=25, ensemble_launch=launch)
            y, st, _ = s.solve_batch(y0, 0.0, 1.0, 1e-6, mode=1)
            assert np.all(st == 0), (launch, st)
            out[launch] = (y, [(s.batch_stats(q)["n_accept"], s.batch_stats(q)["n_learned"]) for q in range(len(ws))])
    finally:
        s.set_controller(0)
        s.set_options(tile=-1, ensemble_launch=0)
    assert sum(nl for _, nl in out[0][1]) > 0
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


def test_persistent_launch_rejects_other_tiles(bs):
    """Tiles of other than four waves have no persistent form: a forced one is refused."""
    b, s = bs
    ws = _members(3, 13, t1=0.2)
    s.set_ensemble(ws)
    try:
        s.set_options(tile=1, ensemble_launch=1)   # BF16 (1,1,8,4): eight waves
        with pytest.raises(b.BS32Error) as e:
            s.solve_batch(np.concatenate([w["y0"] for w in ws]), 0.0, 0.2, 1e-6, mode=2)
        assert e.value.code == b.EUNSUPPORTED
    finally:
        s.set_options(tile=-1, ensemble_launch=0)
    with pytest.raises(b.BS32Error):
        s.set_options(ensemble_launch=2)


def test_batch_autotuned_and_failures(bs, orc):
    b, s = bs
    ws = _members(12, 8, t1=1.5)
    y0 = np.concatenate([w["y0"] for w in ws])
    k = sum(w["y0"].size for w in ws[:4])
    y0[k + 2] = math.nan  # instance 4 starts from a NaN
    say("[batch autotuned + NaN instance] kuramoto B=12")
    s.set_ensemble(ws)
    y, st, tot = s.solve_batch(y0, 0.0, 1.5, 1e-6)
    assert st[4] == b.NONFINITE
    assert np.all(np.delete(st, 4) == 0)
    off = 0
    for q, w in enumerate(ws):
        m = w["y0"].size
        if q != 4:
            ref, _, _ = orc.bs32_solve(w["kind"], w["n"], w["y0"], 0.0, 1.5, 1e-6, A=w["A"], param=w["param"],
                                       gain=w["gain"])
            assert np.linalg.norm(y[off:off + m] - ref) / np.linalg.norm(ref) <= 1e-10
        off += m


def test_batch_rejects_mixed_kinds(bs):
    b, s = bs
    with pytest.raises(b.BS32Error):
        s.set_ensemble([workloads.kuramoto(40, seed=1), workloads.osc2(40, seed=2)])


def test_format_switch_leaves_no_stale_operand_bytes(bs):
    """Padding columns of the operand buffers are read against zero weights; after
    a solve in another storage format they must not hold that format's bytes (an
    FP32 value's low half read as BF16 / FP16 can be Inf or NaN, and 0 * Inf = NaN)."""
    b, s = bs
    ws = _members(12, 9)
    y0 = np.concatenate([w["y0"] for w in ws])
    s.set_options(tile=7)
    try:
        fresh = {}
        for mode in (2, 3):
            s.set_ensemble(ws)
            y, st, _ = s.solve_batch(y0, 0.0, 2.0, 1e-6, mode=mode)
            assert np.all(st == 0)
            fresh[mode] = y
        s.set_ensemble(ws)
        for mode in (1, 2, 1, 3):
            say(f"[format switch] ensemble mode {mode}")
            y, st, _ = s.solve_batch(y0, 0.0, 2.0, 1e-6, mode=mode)
            assert np.all(st == 0), (mode, st)
            if mode in fresh:
                np.testing.assert_array_equal(y, fresh[mode])
    finally:
        s.set_options(tile=-1)


def test_format_switch_single_system(bs):
    b, s = bs
    w = workloads.kuramoto(300, seed=71, t1=2.0)   # N not a multiple of 256: padded rows
    s.set_options(tile=0)
    try:
        s.set_workload(w)
        y2, st2 = s.solve(w["y0"], 0.0, 2.0, 1e-6, mode=2)
        s.set_workload(w)
        for mode in (1, 2, 4, 3, 2):
            y, st = s.solve(w["y0"], 0.0, 2.0, 1e-6, mode=mode)
            assert st["status"] == 0, (mode, st["status"])
        np.testing.assert_array_equal(y, y2)
    finally:
        s.set_options(tile=-1)


def test_range_stop_is_per_instance(bs):
    """One instance whose operand leaves the e4m3 range (|x| > 448) stops with
    BS32_RANGE; the others run on and equal their single-system solves."""
    b, s = bs
    ws = [workloads.osc2(int(n), seed=140 + q, t1=2.0) for q, n in enumerate((200, 150, 260, 90))]
    ws[2]["y0"] = ws[2]["y0"].copy()
    ws[2]["y0"][0::2] *= 1000.0  # positions far outside e4m3's range
    say("[range per instance] osc2 B=4, instance 2 out of range, e4m3")
    s.set_options(tile=0)
    try:
        s.set_ensemble(ws)
        y0 = np.concatenate([w["y0"] for w in ws])
        y, st, tot = s.solve_batch(y0, 0.0, np.full(4, 2.0), 1e-6, mode=4)
        say(f"   statuses {list(st)}")
        assert st[2] == b.RANGE
        assert all(st[q] == 0 for q in (0, 1, 3))
        single = b.Solver(0)
        single.set_options(tile=0)
        off = 0
        for q, w in enumerate(ws):
            m = w["y0"].size
            if q != 2:
                single.set_workload(w)
                ys, sst = single.solve(w["y0"], 0.0, 2.0, 1e-6, mode=4)
                assert sst["status"] == 0
                assert np.array_equal(ys, y[off:off + m]), q
            off += m
        single.close()
    finally:
        s.set_options(tile=-1)

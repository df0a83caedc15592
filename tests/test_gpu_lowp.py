"""GPU parity of the reduced-precision contraction modes against the oracle.

* the stored coupling matrix is bit-exact with the oracle's rounding of A/s and
  the power-of-two scale s equals the oracle's;
* one right-hand side per mode matches the oracle's reduced-precision
  definition (stored weights, split vector operand, exact sums) within the
  FP32-accumulation bound 4 * 2^-24 * L * (gain/N) sum_j |A_ij||v_j|, with L the
  number of products one FP32 partial sum holds (128 for FP32, 256 for the
  BF16/FP16 matrix cores, 512 for e4m3);
* short solves track the oracle's reduced-precision solve.
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

MODES = {1: ("rhs_fp32", 1, 128), 2: ("rhs_bf16", 2, 256), 3: ("rhs_fp16", 3, 256), 4: ("rhs_fp8", 4, 512)}
NP_DT = {1: np.float32, 2: np.uint16, 3: np.uint16, 4: np.uint8}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bs():
    import paper_2605_23727_amd as b
    s = b.Solver(0)
    yield b, s
    s.close()


@pytest.mark.parametrize("mode", [1, 2, 3, 4])
def test_packed_matrix_bit_exact(bs, orc, mode):
    b, s = bs
    g = np.random.default_rng(50 + mode)
    n = 96
    A = g.random((n, n)) * 10.0 ** g.integers(-5, 1, (n, n))
    A[0, :8] = [1.0 + 2.0**-9, 1.0 + 3 * 2.0**-9, 0.5 + 2.0**-6, 2.0**-130, 1.0 + 2.0**-12, 0.0, 1e-9, 0.999]
    A *= np.where(g.random((n, n)) < 0.3, -1.0, 1.0)
    say(f"[packed] mode {MODES[mode][0]} n={n}")
    s.set_system(workloads.KURAMOTO, n, A, np.zeros(n), 1.0)
    bits, scale = s.packed_coupling(mode)
    fmt = MODES[mode][1]
    ref_scale = orc.matrix_scale(A, fmt)
    assert scale == ref_scale
    if mode == 1:
        np.testing.assert_array_equal(bits.astype(np.float64), orc.round_fmt(A / scale, fmt))
    else:
        ref = orc.encode_fmt(A / scale, fmt).astype(NP_DT[mode])
        assert np.array_equal(bits, ref), np.argwhere(bits != ref)[:5]


CASES = [
    ("kuramoto_n1000", lambda: workloads.kuramoto(1000, seed=61)),
    ("osc2_n700", lambda: workloads.osc2(700, seed=62)),
    ("goodwin3_n515", lambda: workloads.goodwin3(515, seed=63)),
    ("kuramoto_n4096", lambda: workloads.kuramoto(4096, seed=64)),
]


@pytest.mark.parametrize("mode", [1, 2, 3, 4])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_rhs_lowp_matches_oracle(bs, orc, name, make, mode):
    b, s = bs
    w = make()
    mname, fmt, L = MODES[mode]
    say(f"[rhs {mname}] {name}")
    s.set_workload(w)
    f = s.rhs(w["y0"], mode=mode)
    ref = orc.rhs_lowp(w["kind"], w["n"], w["y0"], fmt, A=w["A"], param=w["param"], gain=w["gain"])
    d = workloads.DIM[w["kind"]]
    x = w["y0"][0::d]
    v = np.abs(np.concatenate([np.sin(x), np.cos(x)])) if d == 1 else np.abs(x)
    Aabs = np.abs(w["A"])
    S = (Aabs @ (v[: w["n"]] + (v[w["n"]:] if d == 1 else 0.0))) * abs(w["gain"]) / w["n"]
    tol = 4 * 2.0**-24 * L * np.repeat(S, d) + 1e-13 * np.abs(ref) + 1e-15
    err = np.abs(f - ref)
    assert np.all(err <= tol), (np.max(err / tol), np.max(err))


SOLVES = [
    ("osc2_n300", lambda: workloads.osc2(300, seed=71, t1=3.0, rtol=1e-6)),
    ("kuramoto_n512", lambda: workloads.kuramoto(512, seed=72, t1=2.0, rtol=1e-6)),
    ("goodwin3_n256", lambda: workloads.goodwin3(256, seed=73, t1=20.0, rtol=1e-6)),
]


@pytest.mark.parametrize("mode", [1, 2, 3, 4])
@pytest.mark.parametrize("name,make", SOLVES, ids=[c[0] for c in SOLVES])
def test_solve_lowp_tracks_oracle(bs, orc, name, make, mode):
    b, s = bs
    w = make()
    mname, fmt, L = MODES[mode]
    say(f"[solve {mname}] {name}")
    s.set_workload(w)
    y, st = s.solve(w["y0"], w["t0"], w["t1"], w["rtol"], w["atol"], mode=mode)
    ref, rst, _ = orc.bs32_solve(w["kind"], w["n"], w["y0"], w["t0"], w["t1"], w["rtol"], w["atol"], A=w["A"],
                                 param=w["param"], gain=w["gain"], mode=mode)
    assert st["status"] == 0 and rst["status"] == 0
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    say(f"   rel l2 {rel:.2e} accepted {st['n_accept']} / {rst['n_accept']}")
    assert rel <= 2e-5
    assert abs(st["n_accept"] - rst["n_accept"]) <= max(2, 0.03 * rst["n_accept"])


@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4])
def test_every_tile_matches_oracle(bs, orc, mode):
    """Every instantiated contraction tile (the autotuner's candidates), forced one
    by one, on a ragged size; FP64 to summation-order rounding, others to the bound."""
    b, s = bs
    w = workloads.kuramoto(777, seed=76)
    s.set_workload(w)
    if mode == 0:
        ref = orc.rhs(w["kind"], w["n"], w["y0"], A=w["A"], param=w["param"], gain=w["gain"])
        tol = 1e-13 * (np.abs(w["A"]).sum(1) * abs(w["gain"]) / w["n"]) + 1e-15
    else:
        mname, fmt, L = MODES[mode]
        ref = orc.rhs_lowp(w["kind"], w["n"], w["y0"], fmt, A=w["A"], param=w["param"], gain=w["gain"])
        tol = 4 * 2.0**-24 * L * (np.abs(w["A"]).sum(1) * 2 * abs(w["gain"]) / w["n"]) + 1e-15
    k = 0
    try:
        while True:
            s.set_options(tile=k)
            say(f"[tile] mode {mode} tile {k}")
            try:
                f = s.rhs(w["y0"], mode=mode)
            except b.BS32Error as e:
                assert e.code == b.EINVAL and k > 0  # past the last candidate
                break
            err = np.abs(f - ref)
            assert np.all(err <= tol), (k, np.max(err / tol))
            k += 1
    finally:
        s.set_options(tile=-1)
    assert k >= 8


@pytest.mark.parametrize("mode", [1, 2, 4])
def test_every_tile_solve_tracks_oracle(bs, orc, mode):
    """Every contraction tile, forced one by one, through a short solve (every stage
    kind, both operand columns, the controller) against the oracle's solve in the same
    storage mode."""
    b, s = bs
    w = workloads.kuramoto(777, seed=77, t1=0.3)
    s.set_workload(w)
    ref, rst, _ = orc.bs32_solve(w["kind"], w["n"], w["y0"], 0.0, 0.3, 1e-6, A=w["A"], param=w["param"],
                                 gain=w["gain"], mode=mode)
    assert rst["status"] == 0
    k = 0
    try:
        while True:
            s.set_options(tile=k)
            say(f"[tile solve] mode {mode} tile {k}")
            try:
                y, st = s.solve(w["y0"], 0.0, 0.3, 1e-6, mode=mode)
            except b.BS32Error as e:
                assert e.code == b.EINVAL and k > 0  # past the last candidate
                break
            rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
            assert st["status"] == 0 and rel <= 2e-5, (k, rel)
            assert abs(st["n_accept"] - rst["n_accept"]) <= 2, k
            k += 1
    finally:
        s.set_options(tile=-1)
    assert k >= 8


def test_lowp_reproducible(bs):
    b, s = bs
    w = workloads.kuramoto(1024, seed=74, t1=1.0)
    s.set_workload(w)
    say("[lowp determinism] kuramoto n=1024 bf16 x2")
    y1, _ = s.solve(w["y0"], 0.0, 1.0, 1e-6, mode=2)
    y2, _ = s.solve(w["y0"], 0.0, 1.0, 1e-6, mode=2)
    assert np.array_equal(y1, y2)


def test_fp8_range_check(bs):
    b, s = bs
    n = 64
    w = workloads.osc2(n, seed=75)
    y0 = w["y0"].copy()
    y0[0] = 1000.0  # x beyond the e4m3 range of the vector terms
    s.set_workload(w)
    say("[fp8 range] osc2 n=64")
    y, st = s.solve(y0, 0.0, 1.0, 1e-6, mode=4)
    assert st["status"] == b.RANGE
    with pytest.raises(b.BS32Error):
        s.rhs(y0, mode=4)

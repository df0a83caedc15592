"""GPU tests of shared-coupling ensembles: many instances with one coupling
matrix and their own parameters, gains, initial values and intervals, whose
stage contractions run as one matrix product on the matrix cores.

Every instance is checked against the oracle's solve of that instance alone:
FP64 at the parity bar (relative l2 <= 1e-10, accepted steps within 1 %),
the reduced storage formats against the oracle's reduced-precision solve (the
oracle quantizes A and the operand terms the same way and sums exactly).
"""
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


def _sweep(kind, n, B, seed):
    """B instances on one network: per-instance parameters, gains and initial values."""
    g = np.random.default_rng(seed)
    if kind == "kuramoto":
        base = workloads.kuramoto(n, seed=seed, t1=2.0)
        params = g.standard_normal((B, n))
        gains = g.uniform(0.5, 4.0, B)
        y0 = g.random((B, n)) * 2 * np.pi
    elif kind == "osc2":
        base = workloads.osc2(n, seed=seed, t1=2.0)
        params = g.uniform(0.5, 1.5, (B, n))
        gains = np.ones(B)
        y0 = g.standard_normal((B, 2 * n))
    elif kind == "goodwin3":
        base = workloads.goodwin3(n, seed=seed, t1=20.0)
        params = g.uniform(0.18, 0.22, (B, n))
        gains = g.uniform(0.2, 1.0, B)
        y0 = (g.random((B, n, 3)) * 2 * np.array([0.062, 0.310, 1.549])).reshape(B, -1)
    else:
        base = workloads.lco_paper(n, seed=seed, t1=2.0, dense=True)
        params = None
        gains = np.ones(B)
        y0 = g.random((B, 2 * n)) * 2.0
    return base, params, gains, y0


def _check_against_oracle(b, s, orc, kind, base, params, gains, y0, t1, rtol, mode, rel_bar, acc_bar):
    B = y0.shape[0]
    n = base["n"]
    s.set_shared_ensemble(base["kind"], n, B, A=base["A"], params=params, gains=gains)
    y, st, tot = s.solve_batch(y0.reshape(-1), 0.0, t1, rtol, mode=mode)
    assert np.all(st == 0), st
    Y = y.reshape(B, -1)
    worst = 0.0
    for q in range(B):
        bst = s.batch_stats(q)
        if t1[q] == 0.0:
            assert np.array_equal(Y[q], y0[q]) and bst["n_fev"] == 0
            continue
        ref, rst, _ = orc.bs32_solve(base["kind"], n, y0[q], 0.0, t1[q], rtol, A=base["A"],
                                     param=None if params is None else params[q], gain=gains[q], mode=mode)
        assert rst["status"] == 0
        rel = np.linalg.norm(Y[q] - ref) / np.linalg.norm(ref)
        worst = max(worst, rel)
        assert rel <= rel_bar, (kind, mode, q, rel)
        assert abs(bst["n_accept"] - rst["n_accept"]) <= max(acc_bar[0], acc_bar[1] * rst["n_accept"]), q
    say(f"   worst rel {worst:.2e}")
    assert tot["n_fev"] == sum(s.batch_stats(q)["n_fev"] for q in range(B))


@pytest.mark.parametrize("kind,n,B", [("kuramoto", 300, 7), ("osc2", 257, 5), ("goodwin3", 130, 4),
                                      ("lco", 200, 3), ("kuramoto", 1, 2)])
def test_shared_fp64_matches_oracle(bs, orc, kind, n, B):
    b, s = bs
    base, params, gains, y0 = _sweep(kind, n, B, 400 + n)
    t1 = np.full(B, base["t1"])
    if B >= 4:
        t1[1] = 0.0              # an empty interval returns y0
        t1[2] = 0.4 * base["t1"]  # instances finish at different attempts
    say(f"[shared fp64] {kind} n={n} B={B}")
    _check_against_oracle(b, s, orc, kind, base, params, gains, y0, t1, 1e-7, 0, 1e-10, (1, 0.01))


LIBRARY_TILE = 6   # hipBLASLt product + the kernel's row epilogues (16-bit storage), 64 x 128 tiles
LIBRARY_TILES = (6, 7, 8)   # the same with 64 x 128, 64 x 64 and 64 x 32 epilogue tiles
GEMM_TILES = (9, 10, 11)   # LDS-tiled products of 16-bit storage: 128 x 128, 128 x 64, 64 x 128


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4, 5, *LIBRARY_TILES, *GEMM_TILES])
@pytest.mark.parametrize("mode", [0, 1, 2, 3, 8])
def test_shared_every_tile(bs, orc, tile, mode):
    """Every instantiated product tile in every storage format, on a ragged N and a
    batch that does not fill the last column block; the library product too."""
    b, s = bs
    base, params, gains, y0 = _sweep("kuramoto", 333, 37, 77)
    y0 = y0[:37]
    t1 = np.full(37, 0.5)
    say(f"[shared tile {tile}] mode {mode}")
    s.set_options(tile=tile)
    try:
        s.set_shared_ensemble(base["kind"], 333, 37, A=base["A"], params=params, gains=gains)
        served = (2, 3, 8) if tile in LIBRARY_TILES + GEMM_TILES else (2, 3) if tile >= 4 else (0, 1, 2, 3, 8)
        if mode not in served:   # the 256-row tiles serve BF16 and FP16, the library 16-bit storage
            with pytest.raises(b.BS32Error):
                s.kernel_name(mode, tile)
            return
        name = s.kernel_name(mode, tile)
        assert name.startswith("hipBLASLt product + k_shared_contract<" if tile in LIBRARY_TILES else
                               "k_shared_gemm<" if tile in GEMM_TILES else "k_shared_contract<")
        y, st, _ = s.solve_batch(y0.reshape(-1), 0.0, t1, 1e-6, mode=mode)
        assert np.all(st == 0)
        Y = y.reshape(37, -1)
        for q in (0, 17, 36):
            ref, rst, _ = orc.bs32_solve(base["kind"], 333, y0[q], 0.0, 0.5, 1e-6, A=base["A"], param=params[q],
                                         gain=gains[q], mode=mode)
            rel = np.linalg.norm(Y[q] - ref) / np.linalg.norm(ref)
            assert rel <= (1e-10 if mode == 0 else 2e-5), (q, rel)
    finally:
        s.set_options(tile=-1)


@pytest.mark.parametrize("mode", [1, 2, 3, 8])
def test_shared_reduced_tracks_oracle(bs, orc, mode):
    b, s = bs
    base, params, gains, y0 = _sweep("kuramoto", 520, 6, 91)
    t1 = np.full(6, 2.0)
    say(f"[shared reduced] mode {mode}")
    _check_against_oracle(b, s, orc, "kuramoto", base, params, gains, y0, t1, 1e-6, mode, 2e-5, (2, 0.03))


@pytest.mark.parametrize("mode", [2, 3, 8])
def test_library_product_matches_fused(bs, mode):
    """The library product (FP32 accumulation over the whole k) and the fused kernel
    solve the same fixed-step sweep to FP32 summation-order differences."""
    b, s = bs
    base, params, gains, y0 = _sweep("kuramoto", 700, 37, 92)
    say(f"[shared library vs fused] mode {mode}")
    out = {}
    try:
        s.set_options(fixed_step=1, h0=0.02)
        for tile in (1, LIBRARY_TILE):
            s.set_options(tile=tile)
            s.set_shared_ensemble(base["kind"], 700, 37, A=base["A"], params=params, gains=gains)
            y, st, _ = s.solve_batch(y0.reshape(-1), 0.0, 1.0, 1e-6, mode=mode)
            assert np.all(st == 0)
            assert all(s.batch_stats(q)["n_accept"] == 50 for q in range(37))
            out[tile] = y
    finally:
        s.set_options(tile=-1, fixed_step=0, h0=0.0)
    rel = np.linalg.norm(out[1] - out[LIBRARY_TILE]) / np.linalg.norm(out[1])
    say(f"   rel {rel:.2e}")
    assert rel <= 1e-6


def test_shared_equals_grouped_ensemble(bs):
    """The product path and the grouped path (one matrix copy per instance) solve the
    same instances to FP64 rounding."""
    b, s = bs
    base, params, gains, y0 = _sweep("osc2", 300, 5, 93)
    s.set_shared_ensemble(base["kind"], 300, 5, A=base["A"], params=params, gains=gains)
    y_sh, st_sh, _ = s.solve_batch(y0.reshape(-1), 0.0, 2.0, 1e-8)
    ws = [dict(kind=base["kind"], n=300, A=base["A"], param=params[q], gain=gains[q]) for q in range(5)]
    s.set_ensemble(ws)
    y_gr, st_gr, _ = s.solve_batch(y0.reshape(-1), 0.0, 2.0, 1e-8)
    assert np.all(st_sh == 0) and np.all(st_gr == 0)
    assert np.linalg.norm(y_sh - y_gr) / np.linalg.norm(y_gr) <= 1e-11


def test_shared_rejections(bs):
    b, s = bs
    base, params, gains, y0 = _sweep("kuramoto", 64, 3, 95)
    s.set_shared_ensemble(base["kind"], 64, 3, A=base["A"], params=params, gains=gains)
    with pytest.raises(b.BS32Error):   # e4m3's three operand terms do not tile the product
        s.solve_batch(y0.reshape(-1), 0.0, 1.0, 1e-6, mode=4)
    with pytest.raises(b.BS32Error):   # the recipes are single-system paths
        s.solve_batch(y0.reshape(-1), 0.0, 1.0, 1e-6, mode=6)
    w = workloads.clock4(32, seed=96)
    with pytest.raises(b.BS32Error):
        s.set_shared_ensemble(w["kind"], 32, 2)
    # the context still works after the rejections
    s.set_shared_ensemble(base["kind"], 64, 3, A=base["A"], params=params, gains=gains)
    y, st, _ = s.solve_batch(y0.reshape(-1), 0.0, 1.0, 1e-6)
    assert np.all(st == 0)


def test_bf16_pair_planes_bit_exact(bs, orc):
    """The BF16-pair planes of the stored coupling equal the oracle's quantizer bit for
    bit: hi = RNE_bf16(A/s), lo = RNE_bf16(A/s - hi), s the power-of-two scale."""
    b, s = bs
    w = workloads.kuramoto(300, seed=97)
    s.set_workload(w)
    planes, sc = s.packed_coupling(b.PREC_RHS_BF16X2)
    assert sc == orc.matrix_scale(w["A"], orc.FMT_BF16X2)
    x = w["A"] / sc
    hi = orc.encode_fmt(x, orc.FMT_BF16).astype(np.uint16)
    lo = orc.encode_fmt(x - orc.decode_fmt(hi, orc.FMT_BF16), orc.FMT_BF16).astype(np.uint16)
    np.testing.assert_array_equal(planes[0], hi)
    np.testing.assert_array_equal(planes[1], lo)


def test_bf16_pair_only_for_shared_products(bs):
    b, s = bs
    w = workloads.kuramoto(64, seed=98, t1=1.0)
    s.set_workload(w)
    with pytest.raises(b.BS32Error):
        s.solve(w["y0"], 0.0, 1.0, 1e-6, mode=b.PREC_RHS_BF16X2)
    s.set_ensemble([w, workloads.kuramoto(32, seed=99, t1=1.0)])
    with pytest.raises(b.BS32Error):
        s.solve_batch(np.concatenate([w["y0"], workloads.kuramoto(32, seed=99)["y0"]]), 0.0, 1.0, 1e-6,
                      mode=b.PREC_RHS_BF16X2)

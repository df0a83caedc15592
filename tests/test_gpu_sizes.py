"""GPU parity at the benchmark configurations' own sizes.

* FP64 solves against the oracle (Sec. 2.2, eq. (Stage-ODE23)) on the default
  benchmark workload itself (Kuramoto N = 4096, dense weights, t in [0, 50],
  rtol = atol = 1e-6) and on the Goodwin network N = 16384 over [0, 5]: relative
  l2 difference at t_end <= 1e-10 and accepted-step counts within 1 %.  The
  Kuramoto workload does not amplify rounding differences: the oracle's solution
  from y0 perturbed by 1e-13 (relative) differs from the unperturbed one by
  7.7e-15 at t = 50, so the FP64 bar needs no allowance for chaos.
* Sampled rows of one right-hand side at N = 16384 (Goodwin) and N = 32768
  (Kuramoto, coupled oscillators) in FP64 and every storage format, against the
  oracle's pairwise FP64 definition (bar: 16 sqrt(N) units of FP64 roundoff
  times the sum of the pair terms' magnitudes, the two sides adding N terms in
  different orders) and its reduced-precision definition evaluated for those
  rows only (the stored weights of each row from the per-tensor scale of the
  whole matrix; bar: the FP32-accumulation bound of the storage modes).  The systems are drawn on the GPU
  (torch Philox) and the sampled rows copied back.
* One ensemble with an N = 8192 instance among 64 (sizes log-uniform in
  [256, 8192]) against the oracle, FP64.
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

MODES = {1: (1, 128), 2: (2, 256), 3: (3, 256), 4: (4, 512)}  # mode: (storage format, products per FP32 sum)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bs():
    import paper_2605_23727_amd as b
    s = b.Solver(0)
    yield b, s
    s.close()


def _solve_pair(b, s, orc, w, name):
    say(f"[{name}] n={w['n']} t=[0,{w['t1']}] rtol={w['rtol']}")
    s.set_workload(w)
    y, st = s.solve(w["y0"], w["t0"], w["t1"], w["rtol"], w["atol"], mode=b.PREC_FP64)
    ref, rst, _ = orc.bs32_solve(w["kind"], w["n"], w["y0"], w["t0"], w["t1"], w["rtol"], w["atol"], A=w["A"],
                                 param=w["param"], gain=w["gain"])
    rel = float(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    say(f"   rel l2 {rel:.3e}  accepted gpu {st['n_accept']} oracle {rst['n_accept']}  "
        f"rejected {st['n_reject']} / {rst['n_reject']}")
    assert st["status"] == 0 and rst["status"] == 0
    assert st["t_reached"] == w["t1"]
    assert rel <= 1e-10
    assert abs(st["n_accept"] - rst["n_accept"]) <= max(1, 0.01 * rst["n_accept"])


def test_default_workload_fp64_solve_matches_oracle(bs, orc):
    b, s = bs
    _solve_pair(b, s, orc, workloads.kuramoto(4096, seed=2000, K=2.0, t1=50.0, rtol=1e-6), "kuramoto c2 fp64")


def test_goodwin_n16384_fp64_solve_matches_oracle(bs, orc):
    b, s = bs
    _solve_pair(b, s, orc, workloads.goodwin3(16384, seed=3000, kappa=0.5, t1=5.0, rtol=1e-6), "goodwin c3 fp64")


def _rows(n, seed, k=40):
    g = np.random.default_rng(seed)
    r = np.unique(np.concatenate([[0, 1, n - 2, n - 1], g.integers(0, n, k)]))
    return r.astype(np.int64)


def _host(x):
    return x.detach().cpu().numpy() if hasattr(x, "detach") else np.asarray(x)


SAMPLED = [
    ("goodwin3_n16384", lambda: workloads.goodwin3_device(16384, seed=3000)),
    ("kuramoto_n32768", lambda: workloads.kuramoto_device(32768, seed=5000)),
    ("osc2_n32768", lambda: workloads.osc2_device(32768, seed=5001)),
]


@pytest.mark.parametrize("name,make", SAMPLED, ids=[c[0] for c in SAMPLED])
def test_sampled_rows_at_full_size(bs, orc, name, make):
    import torch
    b, s = bs
    w = make()
    n, kind, d = w["n"], w["kind"], workloads.DIM[w["kind"]]
    say(f"[sampled rows] {name}")
    s.set_workload(w)
    rows = _rows(n, n + kind)
    Ar = _host(w["A"][torch.from_numpy(rows).to(w["A"].device)])
    y = _host(w["y0"])
    p = _host(w["param"])
    amax = float(torch.max(torch.abs(w["A"])).item())
    x = y[0::d]
    v = np.abs(np.concatenate([np.sin(x), np.cos(x)])) if kind == workloads.KURAMOTO else np.abs(x)
    Aabs = np.abs(Ar)
    g = abs(w["gain"])
    if kind == workloads.KURAMOTO:
        S = (Aabs @ (v[:n] + v[n:])) * g / n
        pair = (Aabs.sum(1) * 2.0) * g / n
    else:
        S = (Aabs @ v) * max(1.0, g) / n
        pair = (Aabs @ v + Aabs.sum(1) * np.abs(x[rows])) * max(1.0, g) / n
    for mode in (0, 1, 2, 3, 4):
        f = s.rhs(y, mode=mode).reshape(-1, d)[rows].reshape(-1)
        if mode == 0:
            # both sides sum n FP64 terms in different orders (the oracle left to right):
            # a bound of 16 sqrt(n) units of roundoff times the sum of the terms' magnitudes
            ref = orc.rhs_rows(kind, n, rows, y, A_rows=Ar, param=p, gain=w["gain"])
            tol = 16 * 2.0**-53 * np.sqrt(n) * np.repeat(pair, d) + 1e-15 * np.abs(ref)
        else:
            fmt, L = MODES[mode]
            scale = orc.matrix_scale(np.array([amax]), fmt)
            ref = orc.rhs_lowp_rows(kind, n, rows, y, fmt, scale, A_rows=Ar, param=p, gain=w["gain"])
            tol = 4 * 2.0**-24 * L * np.repeat(S, d) + 1e-13 * np.abs(ref) + 1e-15
        err = np.abs(f - ref)
        say(f"   mode {mode}: max err / tol {np.max(err / (tol + 1e-300)):.3f}")
        assert np.all(err <= tol + 1e-300), (mode, np.max(err / (tol + 1e-300)))
    del w
    torch.cuda.empty_cache()


def test_ensemble_with_n8192_instance_matches_oracle(bs, orc):
    b, s = bs
    B = 64
    ns, ks = workloads.ensemble_sizes(B, seed=4100)
    ns[0] = 8192
    ws = [workloads.ensemble_member(int(n), float(k), seed=4100 * 10 + q, t1=1.0) for q, (n, k) in
          enumerate(zip(ns, ks))]
    say(f"[ensemble] B={B} sum N^2 = {float(np.sum(ns.astype(float) ** 2)):.3e}, largest {int(ns.max())}")
    s.set_ensemble(ws)
    y0 = np.concatenate([w["y0"] for w in ws])
    y, st, tot = s.solve_batch(y0, 0.0, np.full(B, 1.0), 1e-6)
    assert np.all(st == 0)
    offs = np.concatenate([[0], np.cumsum([w["y0"].size for w in ws])])
    check = [0] + list(np.argsort(ns)[:: B // 8][:8])
    for q in check:
        w = ws[q]
        yq = y[offs[q]:offs[q + 1]]
        ref, rst, _ = orc.bs32_solve(w["kind"], w["n"], w["y0"], 0.0, 1.0, 1e-6, A=w["A"], param=w["param"],
                                     gain=w["gain"])
        bst = s.batch_stats(int(q))
        rel = float(np.linalg.norm(yq - ref) / np.linalg.norm(ref))
        say(f"   instance {q} n={w['n']}: rel l2 {rel:.3e} accepted {bst['n_accept']} / {rst['n_accept']}")
        assert rel <= 1e-10
        assert abs(bst["n_accept"] - rst["n_accept"]) <= max(1, 0.01 * rst["n_accept"])

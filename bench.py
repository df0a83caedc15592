#!/usr/bin/env python3
"""Benchmark of the gfx950 BS3(2) hot path.

Default workload (--config c2), the Kuramoto network N = 4096 (paper Benchmark 2
with dense weights): theta_i' = w_i + (K/N) sum_j A_ij sin(theta_j - theta_i),
A ~ U[0,1) with zero diagonal, w ~ N(0,1), theta0 ~ U[0,2pi), K = 2,
t in [0, 50], rtol = atol = 1e-6, seed 2000.

One "step" is one complete solve t0 -> t_end (every stage of the method:
vector operand, N^2 contractions, stage combinations, FSAL, error norm,
controller) with the system already packed and the inputs resident in HBM.
value = pair interactions per second over the timed steps, where one pair is
one (i, j) term of one right-hand-side evaluation (n_fev * N^2 per solve).

Also reported: time-to-t_end of each precision mode next to plain FP64, the
normalized final error ||y - y_ref||_2 / sqrt(N) (paper eq. (Metric)) against an
FP64 reference at a tight tolerance (the oracle's Dormand-Prince 5(4) solution at
rtol 1e-12 for the default workload, tests/golden/kuramoto_n4096_ref.npy, with
the GPU's own FP64 Dormand-Prince 5(4) reference and its distance to the
oracle's; the GPU reference elsewhere), each reduced mode's error split into a
storage part (the reference integrator on the dequantized stored matrix against
the reference on A) and an arithmetic part (the mode against the reference on
the dequantized matrix), a tolerance sweep 1e-4 .. 1e-8 of FP64, FP32 and BF16
(default workload), the roofline of the contraction kernel (algorithmic bytes
N^2 * bytes(A) per launch over its event-timed mean duration, whether the matrix
fits the Infinity Cache, and the HBM traffic the PMC counters measured for the
same kernel when the committed summary matches the kernel sources), and the
CPU oracle timed on a bounded sample.

Other measurement configurations, one JSON line each:
  c3  Goodwin clock network N = 16384 (state 49152), t in [0, 500],
      rtol = atol = 1e-6, coupling stored FP64 / FP32 / BF16 / FP16 / FP8-e4m3.
  c4  ensemble of 512 Kuramoto instances, N log-uniform in [256, 8192],
      K ~ U[0.5, 4), t in [0, 50], rtol = atol = 1e-6, FP32 / BF16 / FP16
      contractions vs FP64 (errors on a stratified 32-instance subset).
  f1  the paper's own pairwise benchmark form: clock / cell-cycle model
      (eq. (CC), arctan pair term, uniform weights) N = 16384, t in [0, 48],
      K = 1, I0 = 1.5, rtol = atol = 1e-6, FP64 vs the paper's recipes (pair
      terms in FP32); bound by the vector ALUs, not by memory.
  f2  synthetic rerun of the paper's accuracy experiments (Sec. 3): normalized
      final error against rtol (LCO N = 1000, Kuramoto N = 2000, clock model
      N = 700) and against N, the BS3(2) estimate against the real local error
      of the linear oscillators (eq. (LCO-Local-Error)), and the beta step-count
      ratios (eq. (Beta-2MP)), for the paper's Single / Mixed1 / Mixed2 / FP64
      solvers plus BF16 and e4m3 coupling storage where a matrix exists.
  f3  parameter sweep on one network: 256 Kuramoto instances sharing one dense
      coupling (N = 8192, A ~ U[0,1) zero diagonal) with their own K ~ U[0.5, 4),
      omega ~ N(0,1) and theta0, t in [0, 10], rtol = atol = 1e-6; every stage is
      one matrix product A [V_1 ... V_256] on the matrix cores (FP64, FP32, BF16,
      FP16 storage, and the BF16 pair: hi + lo BF16 planes), against plain FP64
      single-system solves of the instances.
  c5  learned step-size proposer trained on solver traces of the c1-c3 laws,
      run on Kuramoto N = 32768 (t in [0, 50]) and coupled oscillators
      N = 32768 (t in [0, 10]), FP64 coupling, rtol = atol = 1e-7, against the
      standard controller.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES = {0: 8, 1: 4, 2: 2, 3: 2, 4: 1}
DTYPE = {0: "f64", 1: "f32", 2: "bf16", 3: "f16", 4: "fp8e4m3", 8: "bf16x2"}
METRIC = "pair-interactions/s + time-to-t_end vs plain FP64 GPU at matched final error"
KERNEL_SOURCES = ("bs32_kernels.hip", "bs32_internal.hpp", "bs32_mlp.hpp")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2", choices=["c2", "c3", "c4", "c5", "f1", "f2", "f3"])
    ap.add_argument("--tests", type=int, default=6, help="f2: tests per benchmark and tolerance")
    ap.add_argument("--tests-n", type=int, default=3, help="f2: tests per benchmark and system size")
    ap.add_argument("--parts", default="rtol,size", help="f2: which sweeps to run (rtol, size)")
    ap.add_argument("--n", type=int, default=None, help="agents (single-system configs)")
    ap.add_argument("--rtol", type=float, default=None)
    ap.add_argument("--t1", type=float, default=None)
    ap.add_argument("--modes", default=None, help="comma-separated precision modes to compare with FP64")
    ap.add_argument("--head", type=int, default=None, help="force the headline precision mode")
    ap.add_argument("--ref-rtol", type=float, default=None, help="tolerance of the FP64 reference solve")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-ref", action="store_true", help="skip the reference solution")
    ap.add_argument("--no-attribution", action="store_true",
                    help="skip the storage / arithmetic split of each reduced mode's error")
    ap.add_argument("--sweep", action=argparse.BooleanOptionalAction, default=None,
                    help="tolerance sweep 1e-4 .. 1e-8 (FP64, FP32, BF16; default on for c2)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="MiB of a plain device copy run first (calibrates PMC byte counters)")
    ap.add_argument("--instances", type=int, default=None, help="c4 / f3: ensemble size (512 / 256)")
    ap.add_argument("--no-graph", action="store_true", help="launch attempts directly instead of from HIP graphs")
    ap.add_argument("--label-target", type=float, default=0.9,
                    help="c5: where the training labels aim the next error estimate, as a fraction of the "
                         "tolerance (the library's labels aim at 0.8; 0.9 measured best: 0.95 rejects often)")
    ap.add_argument("--persistent", action="store_true",
                    help="c4: one persistent launch per chunk of attempts (device task queue) instead of one "
                         "grouped launch per stage")
    ap.add_argument("--tile-sweep", action="store_true",
                    help="f3: also time every candidate product of the 16-bit modes (own kernels and the library)")
    ap.add_argument("--method", default="bs32", choices=["bs32", "dp54", "rkf45"],
                    help="single-system configs: the embedded pair (dp54: Dormand-Prince 5(4), rkf45: Fehlberg 4(5); modes 0-4)")
    return ap.parse_args()


def sources_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2605_23727_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def group_kernel(name):
    """The grouped (ensemble) kernel instance of a single-system kernel name: the same
    tile parameters without the last one (the epilogue wave, single systems only)."""
    return name.replace("k_contract_", "k_group_").replace(", false>", ">")


def traffic_lookup(workload, mode_name, kernel):
    """HBM bytes per launch of the contraction kernel from the committed PMC summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), or None when the summary has
    no row for this kernel instance or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel sources sha256: ([0-9a-f]+)", text)
    if not m or m.group(1) != sources_hash():
        return None
    for line in text.splitlines():
        cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
        if len(cells) == 7 and cells[0] == mode_name and cells[1] == kernel:
            try:
                return float(cells[6])
            except ValueError:
                return None
    return None


def calib_copy(torch, dev, mib):
    if mib <= 0:
        return
    src = torch.ones(mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"calibration copy of {mib} MiB done")
    del src, dst


def cpu_baseline(w, seconds):
    """The oracle as it stands, timed on this host's cores on a bounded sample of the
    same workload: the first attempts of the same solve, sized to ~`seconds`."""
    import numpy as np
    import oracle

    def host(x):
        if x is None:
            return None
        return x.cpu().numpy() if hasattr(x, "cpu") else np.asarray(x)

    n = w["n"]
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    threads = min(oracle.threads(), cores)
    kw = dict(A=host(w["A"]), param=host(w["param"]), gain=w["gain"], stimulus=w.get("stimulus", 0.0))
    y0 = host(w["y0"])

    def sample(budget):
        t0 = time.perf_counter()
        _, st, _ = oracle.bs32_solve(w["kind"], n, y0, 0.0, w["t1"], w["rtol"], w["atol"], i_max=2, **kw)
        per_fev = (time.perf_counter() - t0) / max(1, st["n_fev"])
        attempts = max(2, int(budget / per_fev / 3.0))
        t0 = time.perf_counter()
        _, st, _ = oracle.bs32_solve(w["kind"], n, y0, 0.0, w["t1"], w["rtol"], w["atol"], i_max=attempts, **kw)
        return st, time.perf_counter() - t0

    st, dt = sample(seconds)
    pairs = st["n_fev"] * float(n) * n
    # the same oracle on one thread, on a shorter sample
    oracle.set_threads(1)
    try:
        st1, dt1 = sample(seconds / 4.0)
    finally:
        oracle.set_threads(threads)
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": pairs / dt, "unit": "pair-interactions/s", "cores": threads, "kind": "oracle",
            "sample": f"first {st['n_accept'] + st['n_reject']} attempts ({st['n_fev']} RHS evaluations, "
                      f"t reached {st['t_reached']:.3g} of {w['t1']:g}) of the same solve, {dt:.1f} s",
            "seconds": dt, "cpu_model": model, "value_1_thread": st1["n_fev"] * float(n) * n / dt1,
            "sample_1_thread": f"first {st1['n_accept'] + st1['n_reject']} attempts, {dt1:.1f} s"}


def base_line(args, value, ms_per_step, dtype, config):
    return {"metric": METRIC, "value": value, "unit": "pair-interactions/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


# vector-ALU issue peak of MI355X in lane-cycles per second: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz = 39.3e12, one FP64 (or non-packed FP32) instruction per lane per cycle
# (packed FP32 is not used: the published 157.3 TFLOP/s FP32 counts packed FMAs, and
# 78.6 TFLOP/s FP64 an FMA, 2 flops, per lane-cycle).  Transcendental instructions issue
# at a quarter of that rate and count 4 cycles.
VALU_PEAK = 256 * 4 * 16 * 2.4e9


def valu_profile(workload, kernel):
    """(VALU busy %, VALU issue lane-cycles per pair) of a pairwise kernel instance from
    the committed PMC summary, or (None, None).  Lane-cycles per pair: (SQ_INSTS_VALU +
    3 SQ_INSTS_VALU_TRANS_F32 + 3 SQ_INSTS_VALU_TRANS_F64) x 64 / pairs; busy: the
    VALUBusy counter."""
    path = os.path.join(ROOT, "profiles", f"valu_{workload}.md")
    if not os.path.exists(path):
        return None, None
    text = open(path).read()
    m = re.search(r"kernel sources sha256: ([0-9a-f]+)", text)
    if not m or m.group(1) != sources_hash():
        return None, None
    for line in text.splitlines():
        cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
        if len(cells) >= 8 and cells[0] == kernel:
            try:
                return float(cells[-2]), float(cells[-1])
            except ValueError:
                return None, None
    return None, None


def alu_roofline(workload, rh, n):
    """Pairwise kernels are bound by the vector ALUs.  The fraction is the hardware's
    VALU busy share during the kernel (VALUBusy); achieved = that share of the issue
    peak.  The instruction-count estimate (pair evaluations per second x VALU issue
    lane-cycles per pair) is reported beside it: for FP32 it exceeds the 16-lane issue
    rate, because some FP32 instructions take fewer than four cycles per wave."""
    busy, ops = valu_profile(workload, rh["kernel"])
    pairs_per_s = n * n / (rh["contraction_ms"] * 1e-3)
    ach = None if busy is None else busy / 100.0 * VALU_PEAK
    return dict(bound="alu", achieved=None if ach is None else round(ach / 1e12, 3),
                peak=round(VALU_PEAK / 1e12, 2), unit="T VALU lane-cycles/s (busy)",
                frac=None if busy is None else round(busy / 100.0, 4), traffic=None, kernel=rh["kernel"],
                pair_evaluations_per_s=pairs_per_s, valu_issue_lane_cycles_per_pair=ops,
                instruction_estimate_t_per_s=None if ops is None else round(pairs_per_s * ops / 1e12, 3),
                avg_launch_ms=rh["contraction_ms"])


MALL_BYTES = 256 << 20  # Infinity Cache of MI355X


def roofline(kms, bytes_per_launch, kernel, traffic):
    gbs = bytes_per_launch / (kms * 1e-3) / 1e9
    # a matrix that fits the 256 MB Infinity Cache stays there across the launches of a
    # solve: the stream is then served from that cache, and 8 TB/s is the stated HBM
    # ceiling rather than the one that binds
    resident = bytes_per_launch <= MALL_BYTES
    return dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 4),
                traffic=traffic, kernel=kernel, bytes_per_launch=bytes_per_launch, avg_launch_ms=kms,
                residency="infinity-cache" if resident else "hbm")


# ---------------------------------------------------------------------------
# f2: synthetic rerun of the paper's accuracy experiments (Sec. 3)
# ---------------------------------------------------------------------------
PAPER_SOLVERS = [5, 6, 7, 0]  # Single, Mixed1, Mixed2, FP64 (Sec. 2.3, Table MP-Distrib)
STORAGE_SOLVERS = [2, 4]      # BF16 and e4m3 coupling storage (a stored matrix of ones)


def _pct(v, qs):
    import numpy as np
    return [float(x) for x in np.percentile(np.asarray(v, dtype=float), qs)] if len(v) else None


class _Campaign:
    """Runs solves of campaign tests on one library context and keeps the counts."""

    def __init__(self, torch, bs):
        self.torch, self.bs = torch, bs
        self.s = bs.Solver(0)
        self.key = None
        self.pairs = 0.0
        self.seconds = 0.0
        self.solves = 0

    def system(self, w, matrix):
        """Set w's system: pairwise as the paper writes it, or (matrix=True) as a stored
        matrix of ones evaluated by the matrix-vector path (storage formats apply there)."""
        import numpy as np
        key = (w["seed"], w["n"], w["kind"], matrix)
        if key == self.key:
            return
        n = w["n"]
        dev = self.torch.device("cuda:0")
        A = None
        if matrix or w["kind"] == self.bs.LCO_PAPER:
            A = self.torch.ones(n * n, dtype=self.torch.float64, device=dev)
        param = None if w["param"] is None else self.torch.from_numpy(np.asarray(w["param"], float)).to(dev)
        pairwise = (not matrix) and (w["kind"] == self.bs.CLOCK4 or bool(w.get("pairwise", False)))
        self.s.set_system(w["kind"], n, A, param, w["gain"], w.get("stimulus", 0.0), pairwise)
        self.key = key
        self.y0 = self.torch.from_numpy(np.asarray(w["y0"], float)).to(dev)
        self.out = self.torch.empty_like(self.y0)
        self.torch.cuda.synchronize()  # torch's fills are done before the library's stream reads them

    def solve(self, w, mode, rtol, count=True):
        self.s.solve(self.y0, 0.0, w["t1"], rtol, rtol, mode=mode, out=self.out)
        st = self.s.stats()
        if count:
            self.pairs += st["pair_interactions"]
            self.seconds += st["solve_ms"] * 1e-3
            self.solves += 1
        return self.out.cpu().numpy(), st


def bench_accuracy(args, torch, bs):
    import numpy as np
    import workloads

    camp = _Campaign(torch, bs)
    s = camp.s
    s.set_options(i_max=100000, time_limit_s=30.0)  # the paper's attempt limit; a wall-clock bound per solve
    dev = torch.device("cuda:0")
    ref_rtol = args.ref_rtol or 1e-11
    parts = set(args.parts.split(","))
    benches = {
        "lco": dict(make=workloads.lco_campaign, n=1000, seed=7000, rtols=[1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8],
                    sizes=[100, 500, 1000, 2000, 5000], solvers=PAPER_SOLVERS + STORAGE_SOLVERS),
        "kuramoto": dict(make=workloads.kuramoto_campaign, n=2000, seed=8000,
                         rtols=[1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9], sizes=[100, 500, 1000, 2000, 5000],
                         solvers=PAPER_SOLVERS + STORAGE_SOLVERS),
        "clock": dict(make=workloads.clock4_campaign, n=700, seed=9000, rtols=[1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8],
                      sizes=[50, 200, 500, 700, 1000], solvers=PAPER_SOLVERS),
    }
    trace_cap = 1 << 17
    rec_states = 40000
    rec = None

    def reference(name, w):
        """Final state of the exact solution (LCO) or of an FP64 solve at ref_rtol, or None."""
        n = w["n"]
        camp.system(w, False)
        if name == "lco":
            h = torch.from_numpy(np.array([float(w["t1"])])).to(dev)
            return s.lco_flow(n, camp.y0, h).cpu().numpy()
        s.set_options(i_max=2_000_000, time_limit_s=60.0)
        y, st = camp.solve(w, bs.PREC_FP64, ref_rtol, count=False)
        s.set_options(i_max=100000, time_limit_s=30.0)
        return y.copy() if st["status"] == 0 else None

    def run_test(name, cfg, w, rtols, solvers, local=False):
        """Every solver at every tolerance on one test; None if the reference fails."""
        nonlocal rec
        t0 = time.perf_counter()
        ref = reference(name, w)
        if ref is None:
            log(f"  {name} N={w['n']} seed {w['seed']}: reference failed, test skipped")
            return None
        n = w["n"]
        res = {}
        for mode in solvers:
            matrix = mode in STORAGE_SOLVERS and name == "kuramoto"
            camp.system(w, matrix)
            for rtol in rtols:
                lo = local and name == "lco"
                if lo:
                    if rec is None:
                        rec = torch.empty(rec_states * 2 * n, dtype=torch.float64, device=dev)
                    s.set_options(trace=1, trace_cap=trace_cap)
                    s.set_record(rec)
                y, st = camp.solve(w, mode, rtol)
                r = dict(status=int(st["status"]), steps=int(st["n_accept"] + st["n_reject"]),
                         error=float(np.linalg.norm(y - ref) / math.sqrt(n)))
                if lo:
                    s.set_record(None)
                    tr = s.trace(trace_cap)
                    s.set_options(trace=0)
                    na = int(st["n_accept"])
                    if r["status"] == 0 and len(tr) == r["steps"] and na + 1 <= rec_states:
                        acc = tr[tr["accepted"] == 1]
                        h = torch.from_numpy(np.ascontiguousarray(acc["h"])).to(dev)
                        e_real = s.lco_local_error(n, rec, h, 1.0).cpu().numpy()   # delta = Abs / Rel = 1
                        r["local_estimate"] = float(np.mean(acc["err"]))
                        r["local_real"] = float(np.mean(e_real))
                res[(mode, rtol)] = r
        log(f"  {name} N={n} t1={w['t1']:.1f} seed {w['seed']}: {len(res)} solves, "
            f"{time.perf_counter() - t0:.1f} s")
        return res

    out = {}
    if "rtol" in parts:
        for name, cfg in benches.items():
            log(f"f2 error vs rtol: {name} N={cfg['n']}, {args.tests} tests")
            runs = []
            for q in range(args.tests):
                w = cfg["make"](cfg["n"], cfg["seed"] + 10 * q)
                w["seed"] = cfg["seed"] + 10 * q
                r = run_test(name, cfg, w, cfg["rtols"], cfg["solvers"], local=True)
                if r is not None:
                    runs.append(r)
            table, beta, local = {}, {}, {}
            for rtol in cfg["rtols"]:
                done = [r for r in runs if all(r[(m, rtol)]["status"] == 0 for m in cfg["solvers"])]
                for m in cfg["solvers"]:
                    errs = [r[(m, rtol)]["error"] for r in done]
                    table[f"{bs.MODE_NAMES[m]}@{rtol:g}"] = dict(
                        tests=len(done), launched=len(runs), median=_pct(errs, [50])[0] if errs else None,
                        p5=_pct(errs, [5])[0] if errs else None, p95=_pct(errs, [95])[0] if errs else None)
                    if name == "lco":
                        le = [(r[(m, rtol)].get("local_estimate"), r[(m, rtol)].get("local_real")) for r in done
                              if "local_real" in r[(m, rtol)]]
                        if le:
                            local[f"{bs.MODE_NAMES[m]}@{rtol:g}"] = dict(
                                tests=len(le), estimate=_pct([a for a, _ in le], [5, 50, 95]),
                                real=_pct([b for _, b in le], [5, 50, 95]))
            for m in cfg["solvers"]:
                if m == 0:
                    continue
                bv = [r[(0, rt)]["steps"] / r[(m, rt)]["steps"] for r in runs for rt in cfg["rtols"]
                      if all(r[(mm, rt)]["status"] == 0 for mm in cfg["solvers"])]
                if bv:
                    beta[bs.MODE_NAMES[m]] = dict(tests=len(bv), quantiles=_pct(bv, [0, 25, 50, 75, 100]))
            out[name] = dict(n=cfg["n"], error_vs_rtol=table, beta=beta, local_error=local or None)
    if "size" in parts:
        for name, cfg in benches.items():
            rtols = [1e-3, 1e-6, 1e-7, 1e-8]
            log(f"f2 error vs N: {name} sizes {cfg['sizes']}, {args.tests_n} tests each")
            bysize = {}
            for n in cfg["sizes"]:
                runs = []
                for q in range(args.tests_n):
                    w = cfg["make"](n, cfg["seed"] + 500 + 10 * q)
                    w["seed"] = cfg["seed"] + 500 + 10 * q
                    r = run_test(name, cfg, w, rtols, PAPER_SOLVERS)
                    if r is not None:
                        runs.append(r)
                for rtol in rtols:
                    done = [r for r in runs if all(r[(m, rtol)]["status"] == 0 for m in PAPER_SOLVERS)]
                    for m in PAPER_SOLVERS:
                        errs = [r[(m, rtol)]["error"] for r in done]
                        bysize[f"{bs.MODE_NAMES[m]}@{rtol:g}@N={n}"] = dict(
                            tests=len(done), launched=len(runs), quantiles=_pct(errs, [0, 50, 100]) if errs else None)
            out.setdefault(name, {})["error_vs_n"] = bysize
    s.close()
    value = camp.pairs / camp.seconds if camp.seconds > 0 else 0.0
    line = base_line(args, value, 1e3 * camp.seconds / max(1, camp.solves), "mixed",
                     {"workload": f"accuracy campaign (paper Sec. 3, synthetic): LCO / Kuramoto / clock model, "
                                  f"{args.tests} tests per tolerance, {args.tests_n} per size, reference FP64 "
                                  f"rtol {ref_rtol:g} (LCO: analytic)", "global_batch": 1, "seq_len": None})
    line.update({"solves": camp.solves, "solve_seconds": camp.seconds, "accuracy": out,
                 "roofline": None, "cpu_baseline": None})
    return line


# ---------------------------------------------------------------------------
# single-system configurations (c2, c3)
# ---------------------------------------------------------------------------
def bench_single(args, torch, bs, workload, w, modes, ref_rtol):
    import numpy as np

    dev = torch.device("cuda:0")
    n = w["n"]
    t1, rtol = w["t1"], w["rtol"]
    y0 = w["y0"].to(dev) if hasattr(w["y0"], "to") else torch.from_numpy(w["y0"]).to(dev)
    out = torch.empty_like(y0)

    def dev_t(x):
        if x is None:
            return None
        return x.to(dev) if hasattr(x, "to") else torch.from_numpy(x).to(dev)

    pairwise = w["kind"] == bs.CLOCK4 or bool(w.get("pairwise", False))
    s = bs.Solver(0)
    if args.no_graph:
        s.set_options(use_graph=0)
    if args.method != "bs32":
        s.set_options(method=bs.METHOD_DP54 if args.method == "dp54" else bs.METHOD_RKF45)
        modes = [m for m in modes if m < 5]
    A = dev_t(w["A"])
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    s.set_system(w["kind"], n, A, dev_t(w["param"]), w["gain"], w.get("stimulus", 0.0), pairwise)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t_setup) * 1e3
    del A

    ref, ref_info = None, None
    if not args.no_ref:
        log(f"reference solve (GPU FP64 Dormand-Prince 5(4), rtol={ref_rtol:g}) n={n}")
        ref_gpu, rst = reference_solve(bs, torch, w, dev_t(w["A"]), ref_rtol, pairwise)
        log(f"  reference: {rst['n_accept']} accepted, {rst['solve_ms'] / 1e3:.1f} s, status {rst['status']}")
        ref, ref_info = ref_gpu, {"reference": f"GPU FP64 Dormand-Prince 5(4), rtol=atol={ref_rtol:g}"}
        golden = GOLDEN_REF.get((workload, float(t1), w.get("seed")))
        if golden is not None and os.path.exists(golden):
            ref_o = np.load(golden)
            ref = ref_o
            ref_info = {"reference": "oracle FP64 Dormand-Prince 5(4), rtol=atol=1e-12 (" +
                                     os.path.relpath(golden, ROOT) + ")",
                        "gpu_reference": ref_info["reference"],
                        "gpu_reference_rel_l2_vs_oracle": float(np.linalg.norm(ref_gpu - ref_o) / np.linalg.norm(ref_o))}
            log(f"  oracle reference: GPU reference differs by {ref_info['gpu_reference_rel_l2_vs_oracle']:.3e}")

    def final_err(y):
        return None if ref is None else float(np.linalg.norm(y - ref) / math.sqrt(n))

    results, ys = {}, {}
    for mode in sorted(set([0] + modes)):
        log(f"mode {bs.MODE_NAMES[mode]}: {args.warmup} warm-up + {args.steps} timed solves")
        fmt_bytes = BYTES[1] if mode >= 5 else BYTES[mode]
        if pairwise and w["A"] is None:
            fmt_bytes = 0  # uniform pair weights: no matrix is read
        for _ in range(args.warmup):
            s.solve(y0, 0.0, t1, rtol, mode=mode, out=out)
        torch.cuda.synchronize()
        times, pairs, stats = [], 0.0, None
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, stats = s.solve(y0, 0.0, t1, rtol, mode=mode, out=out)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            pairs += stats["pair_interactions"]
        y = out.cpu().numpy()
        ys[mode] = y
        kms = s.time_contraction(mode, repeat=100)
        gbs = n * n * fmt_bytes / (kms * 1e-3) / 1e9
        results[mode] = dict(
            name=bs.MODE_NAMES[mode], time_to_t_end_s=float(np.median(times)), ms_per_step=1e3 * sum(times) / len(times),
            pairs_per_s=pairs / sum(times), accepted=int(stats["n_accept"]), rejected=int(stats["n_reject"]),
            n_fev=int(stats["n_fev"]), accepted_steps_per_s=stats["n_accept"] / float(np.median(times)),
            final_error=final_err(y), status=int(stats["status"]), contraction_ms=kms, contraction_gbs=gbs,
            kernel_ms=stats["kernel_ms"], tile=int(stats["tile"]),
            kernel=s.kernel_name(1 if mode >= 5 else mode, stats["tile"]), fmt_bytes=fmt_bytes)
        log(f"  {results[mode]['time_to_t_end_s'] * 1e3:.2f} ms, error {results[mode]['final_error']}, "
            f"contraction {kms * 1e3:.2f} us ({gbs:.0f} GB/s), tile {stats['tile']}")

    r0 = results[0]
    # headline: the fastest mode whose final error stays within 2x plain FP64's
    # (FP64 itself always qualifies); --head forces one
    if args.head is not None:
        head = args.head
    else:
        ok = [m for m, r in results.items() if r["status"] == 0 and (
            r0["final_error"] is None or r["final_error"] is None or r["final_error"] <= 2.0 * r0["final_error"])]
        head = min(ok, key=lambda m: results[m]["time_to_t_end_s"]) if ok else 0
    rh = results[head]
    if pairwise:
        roof = alu_roofline(workload, rh, n)
    else:
        traffic = traffic_lookup(workload, "rhs_fp32" if head >= 5 else rh["name"], rh["kernel"])
        roof = roofline(rh["contraction_ms"], n * n * rh["fmt_bytes"], rh["kernel"], traffic)

    # storage versus arithmetic (eq. (Metric) errors): each reduced mode against the same
    # reference integrator run on the dequantized stored matrix (A_hat = s Q(A/s))
    attribution = None
    if ref is not None and not pairwise and n <= 8192 and not args.no_attribution:
        attribution = {}
        refs_hat = {}
        for mode in sorted(results):
            if mode == 0 or mode == 8:
                continue
            sm = 1 if mode >= 5 else mode  # the recipes store A in FP32
            if sm not in refs_hat:
                bits, scale = s.packed_coupling(sm)
                A_hat = torch.from_numpy(dequantize(np, bits, sm) * scale).to(dev)
                log(f"reference solve on the dequantized {bs.MODE_NAMES[sm]} matrix")
                refs_hat[sm], _ = reference_solve(bs, torch, w, A_hat, ref_rtol, pairwise)
                del A_hat
            r_hat = refs_hat[sm]
            attribution[results[mode]["name"]] = {
                "final_error": results[mode]["final_error"],
                "storage_error": float(np.linalg.norm(r_hat - ref) / math.sqrt(n)),
                "arithmetic_error": float(np.linalg.norm(ys[mode] - r_hat) / math.sqrt(n))}
        attribution["fp64"] = {"final_error": r0["final_error"], "storage_error": 0.0,
                               "arithmetic_error": r0["final_error"]}

    # work-precision: time to t_end and final error over the tolerance sweep
    sweep = None
    if ref is not None and args.sweep:
        sweep = []
        for rt in (1e-4, 1e-5, 1e-6, 1e-7, 1e-8):
            for mode in [m for m in (0, 1, 2) if m in results]:
                s.solve(y0, 0.0, t1, rt, mode=mode, out=out)
                times = []
                for _ in range(3):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, st = s.solve(y0, 0.0, t1, rt, mode=mode, out=out)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                e = float(np.linalg.norm(out.cpu().numpy() - ref) / math.sqrt(n))
                sweep.append({"rtol": rt, "mode": bs.MODE_NAMES[mode], "time_to_t_end_s": float(np.median(times)),
                              "final_error": e, "accepted": int(st["n_accept"]), "rejected": int(st["n_reject"]),
                              "status": int(st["status"])})
                log(f"  sweep rtol {rt:g} {bs.MODE_NAMES[mode]}: {np.median(times) * 1e3:.2f} ms, error {e:.3e}")

    cpu = None
    if not args.no_cpu:
        log(f"CPU oracle baseline (~{args.cpu_seconds:g} s)")
        cpu = cpu_baseline(w, args.cpu_seconds)

    line = base_line(args, rh["pairs_per_s"], rh["ms_per_step"],
                     ("f32-recipe" if head >= 5 else DTYPE[head] + "+f64-update"),
                     {"workload": workload_desc(workload, w) + {"bs32": "", "dp54": " pair=dormand-prince-5(4)",
                                                                  "rkf45": " pair=fehlberg-4(5)"}[args.method],
                      "precision_mode": rh["name"], "global_batch": 1,
                      "seq_len": None})
    line.update({
        "time_to_t_end_s": rh["time_to_t_end_s"],
        "fp64_time_to_t_end_s": r0["time_to_t_end_s"],
        "speedup_vs_fp64": r0["time_to_t_end_s"] / rh["time_to_t_end_s"],
        "final_error": rh["final_error"],
        "fp64_final_error": r0["final_error"],
        "reference_rtol": None if ref is None else ref_rtol,
        "reference": ref_info,
        "matched_error": (None if rh["final_error"] is None else rh["final_error"] <= 2.0 * r0["final_error"]),
        "accepted_steps_per_s": rh["accepted_steps_per_s"],
        "beta": (r0["accepted"] + r0["rejected"]) / max(1, rh["accepted"] + rh["rejected"]),
        "setup_ms": setup_ms,
        "modes": {v["name"]: {k: v[k] for k in ("time_to_t_end_s", "pairs_per_s", "accepted", "rejected", "n_fev",
                                                 "final_error", "contraction_ms", "contraction_gbs", "tile", "kernel",
                                                 "status")}
                  for v in results.values()},
        "roofline": roof,
        "cpu_baseline": cpu,
    })
    if attribution is not None:
        line["error_attribution"] = attribution
    if sweep is not None:
        line["rtol_sweep"] = sweep
    s.close()
    return line


# oracle references written by tests/golden/make_kuramoto_reference.py, by (workload, t1, seed)
GOLDEN_REF = {("kuramoto_n4096", 50.0, 2000): os.path.join(ROOT, "tests", "golden", "kuramoto_n4096_ref.npy")}


def reference_solve(bs, torch, w, A, rtol, pairwise):
    """FP64 Dormand-Prince 5(4) solve of w with coupling A (a device tensor) at rtol = atol
    on a context of its own; returns (y at t1 as numpy, stats)."""
    dev = torch.device("cuda:0")

    def dev_t(x):
        if x is None:
            return None
        return x.to(dev) if hasattr(x, "to") else torch.from_numpy(x).to(dev)

    r = bs.Solver(0)
    try:
        r.set_options(i_max=10_000_000, method=bs.METHOD_DP54)
        r.set_system(w["kind"], w["n"], A, dev_t(w["param"]), w["gain"], w.get("stimulus", 0.0), pairwise)
        y0 = dev_t(w["y0"])
        out = torch.empty_like(y0)
        _, st = r.solve(y0, 0.0, w["t1"], rtol, rtol, mode=bs.PREC_FP64, out=out)
        return out.cpu().numpy(), st
    finally:
        r.close()


def dequantize(np, bits, mode):
    """Stored values of a packed matrix (bs32_get_packed_coupling) as FP64, before the scale."""
    if mode == 1:
        return bits.astype(np.float64)
    if mode == 2:
        return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    if mode == 3:
        return bits.view(np.float16).astype(np.float64)
    # OCP e4m3fn: sign, 4 exponent bits (bias 7), 3 fraction bits; S.1111.111 is NaN
    b = np.arange(256)
    e, f = (b >> 3) & 15, b & 7
    val = np.where(e == 0, f * 2.0**-9, (8 + f) * np.exp2(e - 10.0))
    val = np.where((e == 15) & (f == 7), np.nan, val) * np.where(b >> 7, -1.0, 1.0)
    return val[bits]


def workload_desc(workload, w):
    if w["kind"] == 5:
        return (f"clock4-pairwise N={w['n']} K={w['gain']:g} I0={w['stimulus']:g} weights="
                f"{'dense' if w['A'] is not None else 'uniform'} t=[0,{w['t1']:g}] rtol=atol={w['rtol']:g} "
                f"seed={w['seed']}")
    if w["kind"] == 3 and w.get("pairwise"):
        return (f"kuramoto-pairwise N={w['n']} K={w['gain']:g} weights={'dense' if w['A'] is not None else 'uniform'} "
                f"t=[0,{w['t1']:g}] rtol=atol={w['rtol']:g} seed={w['seed']}")
    if w["kind"] == 3:
        return f"kuramoto-dense N={w['n']} K={w['gain']:g} t=[0,{w['t1']:g}] rtol=atol={w['rtol']:g} seed={w['seed']}"
    if w["kind"] == 4:
        return (f"goodwin3-dense N={w['n']} kappa={w['gain']:g} t=[0,{w['t1']:g}] rtol=atol={w['rtol']:g} "
                f"seed={w['seed']}")
    return f"{workload} N={w['n']} t=[0,{w['t1']:g}] rtol=atol={w['rtol']:g} seed={w['seed']}"


# ---------------------------------------------------------------------------
# c4: batched ensemble
# ---------------------------------------------------------------------------
def bench_ensemble(args, torch, bs, modes, ref_rtol):
    import numpy as np
    import workloads

    B = args.instances or 512
    rtol = args.rtol or 1e-6
    t1 = args.t1 or 50.0
    ns, ks = workloads.ensemble_sizes(B, seed=4000)
    pairs_total = float(np.sum(ns.astype(np.float64) ** 2))
    log(f"ensemble: {B} instances, sum N^2 = {pairs_total:.3e}, drawing on the device")
    members = [workloads.kuramoto_device(int(n), seed=4001 + b, K=float(k), t1=t1, rtol=rtol)
               for b, (n, k) in enumerate(zip(ns, ks))]
    # stratified subset (by N) checked against a tight-tolerance FP64 reference
    order = np.argsort(ns, kind="stable")
    subset = sorted(int(order[q]) for q in np.linspace(0, B - 1, min(B, 32)).round().astype(int))
    y0 = torch.cat([m["y0"] for m in members]).contiguous()
    offs = np.concatenate([[0], np.cumsum(ns)])
    s = bs.Solver(0)
    if args.persistent:
        s.set_options(ensemble_launch=1)
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    s.set_ensemble(members)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t_setup) * 1e3
    keep = {b: members[b] for b in subset}
    for b, m in enumerate(members):
        if b not in keep:
            m["A"] = None
    del members
    torch.cuda.empty_cache()
    out = torch.empty_like(y0)

    results, ys = {}, {}
    for mode in sorted(set([0] + modes)):
        log(f"mode {bs.MODE_NAMES[mode]}: {args.warmup} warm-up + {args.steps} timed batch solves")
        for _ in range(args.warmup):
            s.solve_batch(y0, 0.0, t1, rtol, mode=mode, out=out)
        times, pairs, tot = [], 0.0, None
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st, tot = s.solve_batch(y0, 0.0, t1, rtol, mode=mode, out=out)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            pairs += tot["pair_interactions"]
        kms = s.time_contraction(mode, repeat=10)
        y = out.cpu().numpy()
        results[mode] = dict(name=bs.MODE_NAMES[mode], time_to_t_end_s=float(np.median(times)),
                             ms_per_step=1e3 * sum(times) / len(times), pairs_per_s=pairs / sum(times),
                             accepted=int(tot["n_accept"]), rejected=int(tot["n_reject"]), n_fev=int(tot["n_fev"]),
                             failed=int(np.sum(st != 0)), contraction_ms=kms,
                             contraction_gbs=pairs_total * BYTES[min(mode, 4)] / (kms * 1e-3) / 1e9,
                             tile=int(tot["tile"]), kernel=s.kernel_name(mode, tot["tile"]), y=y)
        log(f"  {results[mode]['time_to_t_end_s']:.3f} s, {results[mode]['pairs_per_s']:.3e} pairs/s, "
            f"grouped contraction {kms:.3f} ms ({results[mode]['contraction_gbs']:.0f} GB/s)")

    errs = None
    if not args.no_ref:
        log(f"reference: FP64 batch of the {len(subset)}-instance subset at rtol {ref_rtol:g}")
        r = bs.Solver(0)
        r.set_options(i_max=10_000_000)
        r.set_ensemble([keep[b] for b in subset])
        ysub = torch.cat([keep[b]["y0"] for b in subset]).contiguous()
        yr, st, _ = r.solve_batch(ysub, 0.0, t1, ref_rtol, mode=bs.PREC_FP64)
        r.close()
        errs = {}
        for mode, res in results.items():
            e, off = [], 0
            for q, b in enumerate(subset):
                n = int(ns[b])
                e.append(float(np.linalg.norm(res["y"][offs[b]:offs[b] + n] - yr[off:off + n]) / math.sqrt(n)))
                off += n
            errs[mode] = np.array(e)
    # headline: the fastest mode whose median error ratio to FP64 over the checked
    # subset is at most 2 (FP64 itself always qualifies); --head forces one
    def med_ratio(m):
        return float(np.median(errs[m] / np.maximum(errs[0], 1e-300)))
    if args.head is not None:
        head = args.head
    else:
        ok = [m for m, r in results.items() if r["failed"] == 0 and (errs is None or med_ratio(m) <= 2.0)]
        head = min(ok, key=lambda m: results[m]["time_to_t_end_s"]) if ok else 0
    rh, r0 = results[head], results[0]
    ratio = None if errs is None else errs[head] / np.maximum(errs[0], 1e-300)
    for m in results:
        results[m]["error_ratio_vs_fp64_median"] = None if errs is None else med_ratio(m)
    roof = roofline(rh["contraction_ms"], pairs_total * BYTES[min(head, 4)],
                    group_kernel(rh["kernel"]) + f" over {B} instances",
                    traffic_lookup(f"kuramoto_ensemble{B}", rh["name"], group_kernel(rh["kernel"])))
    line = base_line(args, rh["pairs_per_s"], rh["ms_per_step"], DTYPE[min(head, 4)] + "+f64-update",
                     {"workload": f"kuramoto-ensemble B={B} N=logU[256,8192] K=U[0.5,4) t=[0,{t1:g}] "
                                  f"rtol=atol={rtol:g} seed=4000", "precision_mode": rh["name"],
                      "ensemble_launch": "persistent" if args.persistent else "grouped",
                      "global_batch": B, "seq_len": None})
    line.update({
        "time_to_t_end_s": rh["time_to_t_end_s"],
        "fp64_time_to_t_end_s": r0["time_to_t_end_s"],
        "speedup_vs_fp64": r0["time_to_t_end_s"] / rh["time_to_t_end_s"],
        "sum_N2": pairs_total,
        "failed_instances": rh["failed"],
        "error_subset": subset if errs is not None else None,
        "final_error_median": None if errs is None else float(np.median(errs[head])),
        "fp64_final_error_median": None if errs is None else float(np.median(errs[0])),
        "error_ratio_vs_fp64_median": None if ratio is None else float(np.median(ratio)),
        "error_ratio_vs_fp64_max": None if ratio is None else float(np.max(ratio)),
        "matched_error_fraction": None if ratio is None else float(np.mean(ratio <= 2.0)),
        "reference_rtol": None if errs is None else ref_rtol,
        "setup_ms": setup_ms,
        "modes": {v["name"]: {k: v[k] for k in ("time_to_t_end_s", "pairs_per_s", "accepted", "rejected", "n_fev",
                                                 "failed", "contraction_ms", "contraction_gbs", "tile", "kernel",
                                                 "error_ratio_vs_fp64_median")}
                  for v in results.values()},
        "roofline": roof,
        "cpu_baseline": None,
    })
    s.close()
    return line


# ---------------------------------------------------------------------------
# f3: parameter sweep on one network (shared-coupling product)
# ---------------------------------------------------------------------------
MFMA_PEAK_TFLOPS = {0: 78.6, 1: 157.3, 2: 2500.0, 3: 2500.0, 8: 2500.0}  # dense matrix-core peaks of MI355X
# executed products per algorithmic one: operand terms x planes of A
EXEC_FACTOR = {0: 1, 1: 2, 2: 2, 3: 2, 8: 4}


def bench_shared(args, torch, bs, modes, ref_rtol):
    import numpy as np
    import workloads

    dev = torch.device("cuda:0")
    n = args.n or 8192
    B = args.instances or 256
    t1 = args.t1 or 10.0
    rtol = args.rtol or 1e-6
    base = workloads.kuramoto_device(n, seed=10000, t1=t1, rtol=rtol)
    gen = torch.Generator(device=dev)
    gen.manual_seed(10001)
    omega = torch.randn((B, n), generator=gen, device=dev, dtype=torch.float64)
    theta0 = torch.rand((B, n), generator=gen, device=dev, dtype=torch.float64) * (2.0 * math.pi)
    gains = np.random.default_rng(10002).uniform(0.5, 4.0, B)
    torch.cuda.synchronize()
    s = bs.Solver(0)
    if args.no_graph:
        s.set_options(use_graph=0)
    t0s = time.perf_counter()
    s.set_shared_ensemble(bs.KURAMOTO, n, B, A=base["A"], params=omega, gains=gains)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0s) * 1e3
    y0 = theta0.reshape(-1).contiguous()
    out = torch.empty_like(y0)
    results = {}
    for mode in modes:
        log(f"mode {bs.MODE_NAMES[mode]}: {args.warmup} warm-up + {args.steps} timed batch solves (B={B}, N={n})")
        for _ in range(args.warmup):
            s.solve_batch(y0, 0.0, t1, rtol, mode=mode, out=out)
        times, tot = [], None
        for _ in range(args.steps):
            torch.cuda.synchronize()
            tt = time.perf_counter()
            _, st, tot = s.solve_batch(y0, 0.0, t1, rtol, mode=mode, out=out)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - tt)
        kms = s.time_contraction(mode, repeat=20)
        flops = 2.0 * n * n * B * 2  # the contraction's multiply-adds: N^2 per column, m = 2 columns per instance
        results[mode] = dict(
            name=bs.MODE_NAMES[mode], time_to_t_end_s=float(np.median(times)), ms_per_step=1e3 * float(np.mean(times)),
            pairs_per_s=tot["pair_interactions"] / float(np.median(times)), n_fev=int(tot["n_fev"]),
            accepted=int(tot["n_accept"]), rejected=int(tot["n_reject"]), failed=int(np.sum(st != 0)),
            contraction_ms=kms, contraction_tflops=flops / (kms * 1e-3) / 1e12, tile=int(tot["tile"]),
            kernel=s.kernel_name(mode, tot["tile"]), y=out.clone())
        log(f"  {results[mode]['time_to_t_end_s'] * 1e3:.1f} ms, {tot['n_accept']} accepted in all, product "
            f"{kms * 1e3:.1f} us ({results[mode]['contraction_tflops']:.1f} TFLOP/s), {results[mode]['kernel']}")
    # every candidate product of the 16-bit modes, forced one by one: the project's own
    # kernels beside the library product (HIP events, 10 launches each)
    sweep = {}
    if args.tile_sweep:
        for mode in [m for m in results if m in (2, 3, 8)]:
            rows = []
            for i in range(64):
                try:
                    s.set_options(tile=i)
                    name = s.kernel_name(mode, i)
                    s.time_contraction(mode, 2)
                    us = 1e3 * min(s.time_contraction(mode, 10) for _ in range(2))
                except bs.BS32Error as e:
                    if e.code == bs.EINVAL:
                        break
                    continue
                rows.append({"tile": i, "kernel": name, "product_us": us})
            s.set_options(tile=-1)
            rows.sort(key=lambda r: r["product_us"])
            sweep[bs.MODE_NAMES[mode]] = rows
            own = [r for r in rows if not r["kernel"].startswith("hipBLASLt")]
            lib = [r for r in rows if r["kernel"].startswith("hipBLASLt")]
            if own and lib:
                log(f"  {bs.MODE_NAMES[mode]}: fastest own product {own[0]['product_us']:.1f} us ({own[0]['kernel']}), "
                    f"library {lib[0]['product_us']:.1f} us")
    # errors on the first 16 instances against an FP64 batch at ref_rtol
    errs = None
    if not args.no_ref:
        R = min(B, 16)
        log(f"reference: FP64 shared batch of {R} instances at rtol {ref_rtol:g}")
        r = bs.Solver(0)
        r.set_options(i_max=10_000_000)
        r.set_shared_ensemble(bs.KURAMOTO, n, R, A=base["A"], params=omega[:R].contiguous(), gains=gains[:R])
        yr, st, _ = r.solve_batch(theta0[:R].reshape(-1).contiguous(), 0.0, t1, ref_rtol, mode=bs.PREC_FP64)
        r.close()
        yr = yr.reshape(R, n)
        errs = {}
        for mode, res in results.items():
            Y = res["y"].reshape(B, n)[:R].cpu().numpy()
            errs[mode] = np.linalg.norm(Y - yr, axis=1) / math.sqrt(n)
    # the plain FP64 GPU solver, one instance at a time (a bounded sample, scaled to B)
    log("baseline: plain FP64 single-system solves of 4 instances")
    single = bs.Solver(0)
    single.set_system(bs.KURAMOTO, n, base["A"], omega[0].contiguous(), float(gains[0]))
    tsum, pairs = 0.0, 0.0
    for q in range(4):
        single.set_system(bs.KURAMOTO, n, base["A"], omega[q].contiguous(), float(gains[q]))
        yq = theta0[q].contiguous()
        oq = torch.empty_like(yq)
        # packing A and the autotuner run on the first solve of a system: outside the timing
        single.solve(yq, 0.0, 1e-6 * t1, rtol, mode=bs.PREC_FP64, out=oq)
        torch.cuda.synchronize()
        tt = time.perf_counter()
        _, sst = single.solve(yq, 0.0, t1, rtol, mode=bs.PREC_FP64, out=oq)
        torch.cuda.synchronize()
        tsum += time.perf_counter() - tt
        pairs += sst["pair_interactions"]
    single.close()
    single_s = tsum / 4 * B

    def med_ratio(m):
        return float(np.median(errs[m] / np.maximum(errs[0], 1e-300)))
    if args.head is not None:
        head = args.head
    else:
        ok = [m for m, r in results.items() if r["failed"] == 0 and (errs is None or med_ratio(m) <= 2.0)]
        head = min(ok, key=lambda m: results[m]["time_to_t_end_s"]) if ok else modes[0]
    rh = results[head]
    r0 = results.get(0, rh)
    peak = MFMA_PEAK_TFLOPS[head]
    roof = {"bound": "mfma", "achieved": round(rh["contraction_tflops"], 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(rh["contraction_tflops"] / peak, 4), "traffic": None,
            "kernel": rh["kernel"] + f" over {B} instances",
            "flops_per_launch": 2.0 * n * n * B * 2, "avg_launch_ms": rh["contraction_ms"],
            "executed_flops_per_launch": 2.0 * n * n * B * 2 * EXEC_FACTOR[head]}
    line = base_line(args, rh["pairs_per_s"], rh["ms_per_step"],
                     ("f64" if head == 0 else DTYPE[head]) + "+f64-update",
                     {"workload": f"kuramoto-shared-network B={B} N={n} K=U[0.5,4) omega=N(0,1) t=[0,{t1:g}] "
                                  f"rtol=atol={rtol:g} seed=10000", "precision_mode": rh["name"],
                      "global_batch": B, "seq_len": None})
    line.update({
        "time_to_t_end_s": rh["time_to_t_end_s"],
        "fp64_time_to_t_end_s": r0["time_to_t_end_s"],
        "speedup_vs_fp64": r0["time_to_t_end_s"] / rh["time_to_t_end_s"],
        "plain_fp64_single_solves_s": single_s,
        "speedup_vs_plain_fp64_solves": single_s / rh["time_to_t_end_s"],
        "final_error_median": None if errs is None else float(np.median(errs[head])),
        "fp64_final_error_median": None if errs is None else float(np.median(errs[0])),
        "error_ratio_vs_fp64_median": None if errs is None else med_ratio(head),
        "reference_rtol": None if errs is None else ref_rtol,
        "setup_ms": setup_ms,
        "modes": {v["name"]: {k: v[k] for k in ("time_to_t_end_s", "pairs_per_s", "accepted", "rejected", "n_fev",
                                                 "failed", "contraction_ms", "contraction_tflops", "tile", "kernel")}
                  | {"error_ratio_vs_fp64_median": None if errs is None else med_ratio(m)}
                  for m, v in results.items()},
        "roofline": roof,
        "cpu_baseline": None,
    })
    if sweep:
        line["tile_sweep"] = sweep
    s.close()
    return line


# ---------------------------------------------------------------------------
# c5: learned step-size proposer
# ---------------------------------------------------------------------------
def training_set(bs, workloads, log_fn):
    """Traces of the c1-c3 laws (several seeds, tolerances and controller safety
    factors, so that the features cover steps above and below the classical choice)."""
    import numpy as np

    laws = [("osc2", lambda sd: workloads.osc2(256, seed=sd, t1=10.0)),
            ("kuramoto", lambda sd: workloads.kuramoto(1024, seed=sd, t1=50.0)),
            ("goodwin3", lambda sd: workloads.goodwin3(1024, seed=sd, t1=500.0))]
    s = bs.Solver(0)
    F, Y = [], []
    for name, make in laws:
        for sd in (11, 12, 13):
            w = make(sd)
            s.set_workload(w)
            for rtol in (1e-5, 1e-6, 1e-7, 1e-8):
                for safety in (0.9, 0.75, 0.97):
                    s.set_options(trace=1, trace_cap=1 << 20, safety=safety)
                    s.solve(w["y0"], 0.0, w["t1"], rtol)
                    f, y = bs.mlp_features(s.trace(), rtol)
                    F.append(f)
                    Y.append(y)
        log_fn(f"traces of the {name} law: {sum(len(f) for f in F)} samples so far")
    s.close()
    return np.concatenate(F), np.concatenate(Y)


def bench_learned(args, torch, bs, ref_rtol):
    import numpy as np
    import workloads

    t_train = time.perf_counter()
    F, Y = training_set(bs, workloads, log)
    # the library's labels aim the next estimate at 0.8 Rel; another aim shifts every
    # label by (1/3) log(aim / 0.8) (the estimate grows like h^3)
    if args.label_target != 0.8:
        Y = Y + np.float32(math.log(args.label_target / 0.8) / 3.0)
    s = bs.Solver(0)
    W, losses = s.mlp_train(F, Y, epochs=60, batch=256, lr=1e-3, seed=0)
    train_s = time.perf_counter() - t_train
    log(f"trained on {len(F)} samples: loss {losses[0]:.3g} -> {losses[-1]:.3g} ({train_s:.1f} s with traces)")
    n = args.n or 32768
    rtol = args.rtol or 1e-7
    systems = [("kuramoto", workloads.kuramoto_device(n, seed=5000, t1=50.0, rtol=rtol)),
               ("osc2", workloads.osc2_device(n, seed=5001, t1=10.0, rtol=rtol))]
    per = {}
    for name, w in systems:
        s.set_system(w["kind"], n, w["A"], w["param"], w["gain"])
        w["A"] = None
        torch.cuda.empty_cache()
        y0 = w["y0"]
        out = torch.empty_like(y0)
        ref = None
        if not args.no_ref:
            log(f"{name}: reference FP64 rtol {ref_rtol:g}")
            s.set_controller(0)
            s.set_options(i_max=10_000_000)
            yr, _ = s.solve(y0, 0.0, w["t1"], ref_rtol)
            s.set_options(i_max=100000)
            ref = yr
        res = {}
        for ctl in (0, 1):
            if ctl:
                s.set_controller(1, W)
            else:
                s.set_controller(0)
            for _ in range(args.warmup):
                s.solve(y0, 0.0, w["t1"], rtol, out=out)
            times, pairs, st = [], 0.0, None
            for _ in range(args.steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st = s.solve(y0, 0.0, w["t1"], rtol, out=out)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                pairs += st["pair_interactions"]
            y = out.cpu().numpy()
            res[ctl] = dict(time_to_t_end_s=float(np.median(times)), ms_per_step=1e3 * sum(times) / len(times),
                            pairs_per_s=pairs / sum(times), n_fev=int(st["n_fev"]), accepted=int(st["n_accept"]),
                            rejected=int(st["n_reject"]), learned_steps=int(st["n_learned"]), status=int(st["status"]),
                            final_error=None if ref is None else float(np.linalg.norm(y - ref) / math.sqrt(y.size)))
            log(f"  {name} controller {'learned' if ctl else 'standard'}: {res[ctl]['time_to_t_end_s']:.3f} s, "
                f"{res[ctl]['n_fev']} RHS, {res[ctl]['rejected']} rejected, {res[ctl]['learned_steps']} learned, "
                f"error {res[ctl]['final_error']}")
        s.set_controller(0)
        kms = s.time_contraction(0, repeat=20)
        kname = s.kernel_name(0, st["tile"])
        per[name] = dict(standard=res[0], learned=res[1], contraction_ms=kms, kernel=kname,
                         speedup_vs_standard=res[0]["time_to_t_end_s"] / res[1]["time_to_t_end_s"],
                         rhs_ratio=res[1]["n_fev"] / res[0]["n_fev"])
    s.close()
    k = per["kuramoto"]
    line = base_line(args, k["learned"]["pairs_per_s"], k["learned"]["ms_per_step"], "f64",
                     {"workload": f"kuramoto-dense N={n} K=2 t=[0,50] and osc2 N={n} t=[0,10], rtol=atol={rtol:g}, "
                                  f"learned proposer vs standard controller", "precision_mode": "fp64",
                      "global_batch": 1, "seq_len": None})
    line.update({
        "time_to_t_end_s": k["learned"]["time_to_t_end_s"],
        "standard_time_to_t_end_s": k["standard"]["time_to_t_end_s"],
        "speedup_vs_standard": k["speedup_vs_standard"],
        "systems": per,
        "training": {"samples": int(len(F)), "epochs": 60, "batch": 256, "lr": 1e-3, "label_target": args.label_target,
                     "loss_first": float(losses[0]), "loss_last": float(losses[-1]), "seconds": train_s},
        "reference_rtol": None if args.no_ref else ref_rtol,
        "roofline": roofline(k["contraction_ms"], n * n * 8, k["kernel"],
                             traffic_lookup(f"kuramoto_n{n}", "fp64", k["kernel"])),
        "cpu_baseline": None,
    })
    return line


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path would shard rows of A with one all-gather per stage).", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2605_23727_amd as bs
    import workloads

    dev = torch.device("cuda:0")
    calib_copy(torch, dev, args.calib_copy)
    modes = None if args.modes is None else [int(m) for m in args.modes.split(",") if m != ""]
    if args.sweep is None:
        args.sweep = args.config == "c2"
    if args.config == "c2":
        n = args.n or 4096
        w = workloads.kuramoto(n, seed=2000, K=2.0, t1=args.t1 or 50.0, rtol=args.rtol or 1e-6)
        w["seed"] = 2000
        line = bench_single(args, torch, bs, f"kuramoto_n{n}", w,
                            modes if modes is not None else [0, 1, 2, 3, 4, 5, 6, 7], args.ref_rtol or 1e-12)
    elif args.config == "c3":
        n = args.n or 16384
        w = workloads.goodwin3_device(n, seed=3000, t1=args.t1 or 500.0, rtol=args.rtol or 1e-6)
        w["seed"] = 3000
        line = bench_single(args, torch, bs, f"goodwin3_n{n}", w,
                            modes if modes is not None else [0, 1, 2, 3, 4, 5, 6, 7],
                            args.ref_rtol or 1e-9)
    elif args.config == "f1":
        n = args.n or 16384
        w = workloads.clock4(n, seed=6000, K=1.0, I0=1.5, t1=args.t1 or 48.0, rtol=args.rtol or 1e-6)
        w["seed"] = 6000
        line = bench_single(args, torch, bs, f"clock4_n{n}", w, modes if modes is not None else [0, 5, 6, 7],
                            args.ref_rtol or 1e-9)
    elif args.config == "f2":
        line = bench_accuracy(args, torch, bs)
    elif args.config == "f3":
        line = bench_shared(args, torch, bs, modes if modes is not None else [0, 1, 2, 3, 8], args.ref_rtol or 1e-9)
    elif args.config == "c4":
        line = bench_ensemble(args, torch, bs, modes if modes is not None else [0, 1, 2, 3], args.ref_rtol or 1e-9)
    else:
        line = bench_learned(args, torch, bs, args.ref_rtol or 1e-10)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Seeded synthetic inputs shaped like the paper's benchmark systems.

This module is shared by the tests, the smoke check and the benchmark, and it
feeds both the HIP library and the CPU oracle.  It holds none of the method's
arithmetic: it only draws random numbers in a fixed order.

Host draws use ``numpy.random.Generator(PCG64(seed))``; systems too large to
draw on the host (tens of GB of weights) are drawn on the GPU with torch's
Philox generator (``backend="torch"``), and the few rows an oracle check needs
are copied back from there.

Seeds follow ``seed = 1000 * config + instance``.

Workloads (the paper's three benchmarks, Sec. 2.1, generalised to a dense
weight matrix A in place of the uniform weights M_ij = 1/N):

* ``osc2``      coupled oscillators x'' = -w_i^2 x_i + (1/N) sum_j A_ij (x_j - x_i),
                A symmetric U[0,1) with zero diagonal, w ~ U[0.5,1.5), x0, v0 ~ N(0,1).
* ``lco_paper`` the paper's Benchmark 1 (uniform weights), initial values U[0,2).
* ``kuramoto``  theta_i' = w_i + (K/N) sum_j A_ij sin(theta_j - theta_i), A U[0,1)
                zero diagonal, w ~ N(0,1), theta0 ~ U[0,2pi), K = 2.
* ``goodwin3``  Goodwin clock network, C U[0,1) zero diagonal, b ~ U[0.18,0.22),
                kappa = 0.5, (x,y,z)_0 = (0.062, 0.310, 1.549) * 2 U[0,1)^3
                (uniform up to twice the b = 0.2 steady state).
* ``ensemble``  Kuramoto instances with N log-uniform in [256, 8192], K ~ U[0.5,4).
* ``clock4``    the paper's Benchmark 3 (clock / cell cycle, arctan pair term).
* ``*_campaign`` one test of the paper's accuracy campaign per benchmark.
"""
from __future__ import annotations

import math

import numpy as np

OSC2, LCO_PAPER, KURAMOTO, GOODWIN3, CLOCK4 = 1, 2, 3, 4, 5
DIM = {OSC2: 2, LCO_PAPER: 2, KURAMOTO: 1, GOODWIN3: 3, CLOCK4: 4}


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _zero_diag(A):
    np.fill_diagonal(A, 0.0)
    return A


def osc2(n, seed=1000, t1=10.0, rtol=1e-6, atol=None):
    g = _rng(seed)
    U = g.random((n, n))
    A = np.triu(U, 1)
    A = A + A.T
    w = g.uniform(0.5, 1.5, n)
    x0 = g.standard_normal(n)
    v0 = g.standard_normal(n)
    y0 = np.empty(2 * n)
    y0[0::2] = x0
    y0[1::2] = v0
    return dict(kind=OSC2, n=n, A=A, param=w, gain=1.0, y0=y0, t0=0.0, t1=t1, rtol=rtol,
                atol=rtol if atol is None else atol)


def lco_paper(n, seed=1000, t1=10 * math.pi, rtol=1e-6, atol=None, dense=False):
    g = _rng(seed)
    y0 = g.random(2 * n) * 2.0
    A = np.ones((n, n)) if dense else None
    return dict(kind=LCO_PAPER, n=n, A=A, param=None, gain=1.0, y0=y0, t0=0.0, t1=t1, rtol=rtol,
                atol=rtol if atol is None else atol)


def kuramoto(n, seed=2000, K=2.0, t1=50.0, rtol=1e-6, atol=None):
    g = _rng(seed)
    A = _zero_diag(g.random((n, n)))
    w = g.standard_normal(n)
    th0 = g.random(n) * (2.0 * math.pi)
    return dict(kind=KURAMOTO, n=n, A=A, param=w, gain=K, y0=th0, t0=0.0, t1=t1, rtol=rtol,
                atol=rtol if atol is None else atol)


def goodwin3(n, seed=3000, kappa=0.5, t1=500.0, rtol=1e-6, atol=None):
    g = _rng(seed)
    C = _zero_diag(g.random((n, n)))
    b = g.uniform(0.18, 0.22, n)
    u = g.random((n, 3)) * 2.0
    y0 = (u * np.array([0.062, 0.310, 1.549])).reshape(-1)
    return dict(kind=GOODWIN3, n=n, A=C, param=b, gain=kappa, y0=y0, t0=0.0, t1=t1, rtol=rtol,
                atol=rtol if atol is None else atol)


def clock4(n, seed=6000, K=1.0, I0=1.5, t1=48.0, rtol=1e-6, atol=None, dense=False):
    """Paper Benchmark 3 (clock / cell cycle, arctan coupling) as its appendix sets it
    up: k1 ~ N(0.339278, 0.090909^2) per cell (truncated to (0, k0)), X_i = (1, 1, -1.19, -0.62) +
    0.2 (p1..p4) with p ~ U[-0.5, 0.5], uniform weights M_ij = 1/N (dense=True:
    A ~ U[0,1) with zero diagonal).  K in {0.001, 0.1, 1, 10}, I0 in
    {0.228249, 1.5, 10}, t1 in [48, 72] in the paper's campaign.  Draw order:
    k1, initial values, A."""
    g = _rng(seed)
    k1 = 0.339278 + 0.090909 * g.standard_normal(n)
    # truncated to (0, k0): theta^h = k1 / (k0 - k1) must stay positive, or theta^h +
    # X_i2^4 can vanish (about one cell in 10^4 falls outside, so the paper's
    # N <= 1000 rarely meets it); out-of-range draws are drawn again
    while True:
        bad = (k1 <= 0.0) | (k1 >= 2.0)
        if not bad.any():
            break
        k1[bad] = 0.339278 + 0.090909 * g.standard_normal(int(bad.sum()))
    y0 = (np.array([1.0, 1.0, -1.19, -0.62]) + 0.2 * (g.random((n, 4)) - 0.5)).reshape(-1)
    A = _zero_diag(g.random((n, n))) if dense else None
    return dict(kind=CLOCK4, n=n, A=A, param=k1, gain=float(K), stimulus=float(I0), y0=y0, t0=0.0, t1=t1,
                rtol=rtol, atol=rtol if atol is None else atol)


# ---------------------------------------------------------------------------
# the paper's test campaign (appendix parameter tables), uniform weights.
# The paper draws its explored parameters from a Sobol set and its initial
# values with Matlab's generator; here every draw is PCG64 over the same
# intervals.
# ---------------------------------------------------------------------------
def lco_campaign(n, seed):
    """Benchmark 1 test: T_f from {10 pi, 20 pi, 50 pi}, initial values 2 U(0,1)."""
    g = _rng(seed)
    t1 = float(g.choice([10.0, 20.0, 50.0])) * math.pi
    y0 = g.random(2 * n) * 2.0
    return dict(kind=LCO_PAPER, n=n, A=None, param=None, gain=1.0, y0=y0, t0=0.0, t1=t1, rtol=1e-6, atol=1e-6)


def kuramoto_campaign(n, seed):
    """Benchmark 2 test, pairwise sin with uniform weights: sigma ~ U(0,1], K ~ U[0, 3 sigma],
    omega = sigma N(0,1), theta0 = 2 pi U(0,1), T_f = 4 pi / (median|omega| K + 0.001)."""
    g = _rng(seed)
    sigma = 1.0 - g.random()
    K = 3.0 * sigma * g.random()
    w = sigma * g.standard_normal(n)
    th0 = g.random(n) * (2.0 * math.pi)
    t1 = 4.0 * math.pi / (float(np.median(np.abs(w))) * K + 0.001)
    return dict(kind=KURAMOTO, n=n, A=None, param=w, gain=K, y0=th0, t0=0.0, t1=t1, rtol=1e-6, atol=1e-6,
                pairwise=True, sigma=sigma)


def clock4_campaign(n, seed):
    """Benchmark 3 test: K from {0.001, 0.1, 1, 10}, I0 from {0.228249, 1.5, 10},
    T_f ~ U[48, 72], cells drawn as in ``clock4``."""
    g = _rng(seed)
    K = float(g.choice([0.001, 0.1, 1.0, 10.0]))
    I0 = float(g.choice([0.228249, 1.5, 10.0]))
    t1 = float(g.uniform(48.0, 72.0))
    return clock4(n, seed=seed + 1, K=K, I0=I0, t1=t1)


def ensemble_sizes(count, seed=4000, nmin=256, nmax=8192):
    """Per-instance (N, K) of the batched Kuramoto ensemble: N log-uniform, K ~ U[0.5, 4)."""
    g = _rng(seed)
    ln = g.uniform(math.log(nmin), math.log(nmax), count)
    ns = np.clip(np.rint(np.exp(ln)).astype(np.int64), nmin, nmax)
    ks = g.uniform(0.5, 4.0, count)
    return ns, ks


def ensemble_member(n, K, seed, t1=50.0, rtol=1e-6):
    """One Kuramoto member drawn on the host (same law as ``kuramoto``)."""
    return kuramoto(int(n), seed=seed, K=float(K), t1=t1, rtol=rtol)


# ---------------------------------------------------------------------------
# device-side draws for systems whose weights do not fit a host draw
# ---------------------------------------------------------------------------
def kuramoto_device(n, seed, K=2.0, t1=50.0, rtol=1e-6, device="cuda", dtype=None):
    """Kuramoto system drawn with torch's Philox generator on ``device``.

    Returns torch tensors (A is n x n FP64 on the device).  Draw order: A, w, theta0.
    """
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    A = torch.rand((n, n), generator=gen, device=device, dtype=torch.float64)
    A.fill_diagonal_(0.0)
    w = torch.randn(n, generator=gen, device=device, dtype=torch.float64)
    th0 = torch.rand(n, generator=gen, device=device, dtype=torch.float64) * (2.0 * math.pi)
    return dict(kind=KURAMOTO, n=n, A=A, param=w, gain=float(K), y0=th0, t0=0.0, t1=t1, rtol=rtol, atol=rtol)


def osc2_device(n, seed, t1=10.0, rtol=1e-7, device="cuda"):
    """Coupled oscillators drawn on the device; A symmetric with zero diagonal."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    A = torch.rand((n, n), generator=gen, device=device, dtype=torch.float64)
    A = torch.triu(A, 1)
    A = A + A.T
    w = torch.rand(n, generator=gen, device=device, dtype=torch.float64) + 0.5
    x0 = torch.randn(n, generator=gen, device=device, dtype=torch.float64)
    v0 = torch.randn(n, generator=gen, device=device, dtype=torch.float64)
    y0 = torch.stack([x0, v0], dim=1).reshape(-1).contiguous()
    return dict(kind=OSC2, n=n, A=A, param=w, gain=1.0, y0=y0, t0=0.0, t1=t1, rtol=rtol, atol=rtol)


def goodwin3_device(n, seed, kappa=0.5, t1=500.0, rtol=1e-6, device="cuda"):
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    C = torch.rand((n, n), generator=gen, device=device, dtype=torch.float64)
    C.fill_diagonal_(0.0)
    b = torch.rand(n, generator=gen, device=device, dtype=torch.float64) * 0.04 + 0.18
    u = torch.rand((n, 3), generator=gen, device=device, dtype=torch.float64) * 2.0
    y0 = (u * torch.tensor([0.062, 0.310, 1.549], device=device, dtype=torch.float64)).reshape(-1).contiguous()
    return dict(kind=GOODWIN3, n=n, A=C, param=b, gain=kappa, y0=y0, t0=0.0, t1=t1, rtol=rtol, atol=rtol)


# The five benchmark configurations (sizes as the paper-shaped workloads define them)
CONFIGS = {
    1: dict(name="osc2-n256", make=lambda: osc2(256, seed=1000, t1=10.0, rtol=1e-6)),
    2: dict(name="kuramoto-n4096", make=lambda: kuramoto(4096, seed=2000, K=2.0, t1=50.0, rtol=1e-6)),
    3: dict(name="goodwin3-n16384", make=lambda: goodwin3(16384, seed=3000, kappa=0.5, t1=500.0, rtol=1e-6)),
}

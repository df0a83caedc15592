"""The allocation-free gradient entry point (bs32_mlp_grad_noalloc) against the
allocating one (bs32_mlp_grad): same kernels, same inputs, so the gradient and
the loss must agree bit for bit.  Two calls in a row, the second smaller, so a
stale scratch array from the first call would show; sizes beyond the limit and
host buffers are rejected."""
import sys

import numpy as np
import pytest

from tests import mlp_cases as mc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    w = mc.random_net(seed).astype(np.float32)
    w[mc.OFF_MU:mc.OFF_MU + mc.IN] = rng.normal(0.0, 0.5, mc.IN)
    w[mc.OFF_ISD:mc.OFF_ISD + mc.IN] = rng.uniform(0.5, 2.0, mc.IN)
    X = rng.normal(0.0, 1.5, (n, mc.IN)).astype(np.float32)
    Y = rng.normal(0.0, 0.7, n).astype(np.float32)
    return w, X, Y


def test_noalloc_gradient_equals_allocating_entry_point():
    import torch

    import paper_2605_23727_amd as b
    s = b.Solver(0)
    try:
        for n, seed in ((b.MLP_NOALLOC_MAX, 1), (777, 2)):
            say(f"[no-alloc gradient] n={n} seed={seed}")
            w, X, Y = _inputs(n, seed)
            g_ref, L_ref = s.mlp_grad(w, X, Y)
            W = torch.from_numpy(w).cuda()
            F = torch.from_numpy(X.reshape(-1)).cuda()
            Yd = torch.from_numpy(Y).cuda()
            G = torch.full((b.MLP_PARAMS,), float("nan"), dtype=torch.float64, device="cuda")
            L = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
            s.mlp_grad_noalloc(W, F, Yd, G, L)
            torch.cuda.synchronize()
            g = G.cpu().numpy()
            assert np.array_equal(g, g_ref), np.max(np.abs(g - g_ref))
            assert L.item() == L_ref
        say("[no-alloc gradient] limits")
        big = torch.zeros((b.MLP_NOALLOC_MAX + 1) * mc.IN, dtype=torch.float32, device="cuda")
        Ybig = torch.zeros(b.MLP_NOALLOC_MAX + 1, dtype=torch.float32, device="cuda")
        with pytest.raises(b.BS32Error):
            s.mlp_grad_noalloc(W, big, Ybig, G, L)
        with pytest.raises(b.BS32Error):  # host memory is not accepted
            s.mlp_grad_noalloc(W.cpu(), F, Yd, G, L)
    finally:
        s.close()

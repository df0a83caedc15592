"""Python binding of ``libbs32.so``, the gfx950 mixed-precision BS3(2) solver.

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  Arrays may be numpy arrays (host) or torch tensors (host or device);
torch is used for device memory and streams, nothing else.  The C ABI is
declared in ``include/bs32.h``.

If the shared library has not been built (``python -m
paper_2605_23727_amd.build``) importing the binding's entry points raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbs32.so")

# bs32_status
OK, MAX_STEPS, MAX_REJECTS, H_TOO_SMALL, TIMEOUT, TOO_SLOW, NONFINITE, RANGE = 0, 1, 2, 3, 4, 5, 6, 7
EINVAL, ENOMEM, EDEVICE, ESTATE, EUNSUPPORTED = -1, -2, -3, -4, -5
# bs32_system_kind
OSC2, LCO_PAPER, KURAMOTO, GOODWIN3, CLOCK4 = 1, 2, 3, 4, 5
DIM = {OSC2: 2, LCO_PAPER: 2, KURAMOTO: 1, GOODWIN3: 3, CLOCK4: 4}
# bs32_precision_mode
(PREC_FP64, PREC_RHS_FP32, PREC_RHS_BF16, PREC_RHS_FP16, PREC_RHS_FP8_E4M3,
 PREC_PAPER_SINGLE, PREC_PAPER_MIXED1, PREC_PAPER_MIXED2, PREC_RHS_BF16X2) = range(9)
MLP_PARAMS = 4883  # BS32_MLP_PARAMS
MLP_NOALLOC_MAX = 16384  # BS32_MLP_NOALLOC_MAX
METHOD_BS32, METHOD_DP54, METHOD_RKF45 = 0, 1, 2  # bs32_method
MLP_IN = 9
MODE_NAMES = {0: "fp64", 1: "rhs_fp32", 2: "rhs_bf16", 3: "rhs_fp16", 4: "rhs_fp8_e4m3", 5: "paper_single",
              6: "paper_mixed1", 7: "paper_mixed2", 8: "rhs_bf16x2"}


class SystemDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("coupling_on_device", C.c_int32), ("n", C.c_int64),
                ("coupling", C.c_void_p), ("agent_param", C.c_void_p), ("gain", C.c_double),
                ("stimulus", C.c_double), ("pairwise", C.c_int32), ("reserved", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_accept", C.c_int64), ("n_reject", C.c_int64), ("n_fev", C.c_int64),
                ("pair_interactions", C.c_double), ("t_reached", C.c_double), ("h_last", C.c_double),
                ("h_min_seen", C.c_double), ("err_last", C.c_double), ("solve_ms", C.c_double),
                ("kernel_ms", C.c_double), ("status", C.c_int32), ("mode", C.c_int32),
                ("n_learned", C.c_int64), ("tile", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Options(C.Structure):
    _fields_ = [("i_max", C.c_int64), ("time_limit_s", C.c_double), ("slow_limit_s", C.c_double),
                ("h_max", C.c_double), ("h0", C.c_double), ("safety", C.c_double), ("facmin", C.c_double),
                ("facmax", C.c_double), ("fixed_step", C.c_int32), ("use_graph", C.c_int32),
                ("trace", C.c_int32), ("trace_cap", C.c_int32), ("controller", C.c_int32),
                ("tile", C.c_int32), ("method", C.c_int32), ("ensemble_launch", C.c_int32)]


class TraceRec(C.Structure):
    _fields_ = [("t", C.c_double), ("h", C.c_double), ("err", C.c_double), ("fnorm", C.c_double),
                ("accepted", C.c_int32), ("proposer", C.c_int32)]


class BS32Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bs32 error {code}: {msg}")
        self.code = code


_lib = None

# every entry point of include/bs32.h with its ctypes signature
_SIGS = {
    "bs32_create": ([C.c_void_p, C.c_int, C.c_void_p], C.c_int),
    "bs32_default_options": ([C.c_void_p], C.c_int),
    "bs32_set_options": ([C.c_void_p, C.c_void_p], C.c_int),
    "bs32_set_system": ([C.c_void_p, C.c_void_p], C.c_int),
    "bs32_solve": ([C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, C.c_void_p],
                   C.c_int),
    "bs32_stats": ([C.c_void_p, C.c_void_p], C.c_int),
    "bs32_rhs": ([C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p], C.c_int),
    "bs32_get_trace": ([C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "bs32_time_contraction": ([C.c_void_p, C.c_int, C.c_int, C.c_void_p], C.c_int),
    "bs32_kernel_name": ([C.c_void_p, C.c_int, C.c_int, C.c_char_p, C.c_size_t], C.c_int),
    "bs32_get_packed_coupling": ([C.c_void_p, C.c_int, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "bs32_set_ensemble": ([C.c_void_p, C.c_int32, C.c_void_p], C.c_int),
    "bs32_set_shared_ensemble": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p], C.c_int),
    "bs32_solve_batch": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_int,
                          C.c_void_p, C.c_void_p], C.c_int),
    "bs32_batch_stats": ([C.c_void_p, C.c_int32, C.c_void_p], C.c_int),
    "bs32_set_record": ([C.c_void_p, C.c_void_p, C.c_int64], C.c_int),
    "bs32_lco_flow": ([C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "bs32_lco_local_error": ([C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p],
                             C.c_int),
    "bs32_mlp_features": ([C.c_void_p, C.c_size_t, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "bs32_mlp_train": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_int, C.c_float, C.c_uint64,
                        C.c_void_p, C.c_void_p], C.c_int),
    "bs32_mlp_grad": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p], C.c_int),
    "bs32_mlp_grad_noalloc": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p],
                              C.c_int),
    "bs32_set_controller": ([C.c_void_p, C.c_int, C.c_void_p, C.c_size_t], C.c_int),
    "bs32_recipe_row": ([C.c_int, C.c_int, C.c_void_p], C.c_int),
    "bs32_last_error": ([C.c_void_p], C.c_char_p),
    "bs32_destroy": ([C.c_void_p], None),
}


def lib():
    """Load libbs32.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: torch ships its own libamdhip64 under the same
        # soname as ROCm's.  Loaded first, it satisfies the library's dependency, so
        # device pointers and streams are shared with torch; loaded after the library,
        # it would bring a second HIP/HSA runtime that then finds no GPU.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_23727_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


_TRACE_DTYPE = np.dtype([("t", "f8"), ("h", "f8"), ("err", "f8"), ("fnorm", "f8"), ("accepted", "i4"),
                         ("proposer", "i4")])


def _f32(x, n=None):
    a = np.ascontiguousarray(x, dtype=np.float32)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def mlp_features(trace, rtol):
    """(features [n, 9] float32, labels [n] float32) of the learned proposer from a trace."""
    tr = np.ascontiguousarray(trace, dtype=_TRACE_DTYPE)
    cap = max(len(tr) - 4, 0)
    F = np.zeros((cap, MLP_IN), dtype=np.float32)
    Y = np.zeros(cap, dtype=np.float32)
    n = C.c_size_t(0)
    rc = lib().bs32_mlp_features(tr.ctypes.data if len(tr) else None, len(tr), float(rtol),
                                 F.ctypes.data if cap else None, Y.ctypes.data if cap else None, C.byref(n))
    if rc != 0:
        raise BS32Error(rc, "bs32_mlp_features failed")
    return F[: n.value].copy(), Y[: n.value].copy()


def recipe_row(mode, stage_row):
    """(F, Sigma, G) single flags the library evaluates for a recipe mode and stage row (0 k2, 1 k3, 2 k4)."""
    out = np.zeros(3, dtype=np.int32)
    rc = lib().bs32_recipe_row(int(mode), int(stage_row), out.ctypes.data)
    if rc != 0:
        raise BS32Error(rc, "bs32_recipe_row failed")
    return tuple(int(v) for v in out)


class _Buf:
    """A pointer to float64 data: numpy array (host) or torch tensor (host/device)."""

    def __init__(self, x, n=None, writable=False):
        self.keep = None
        if x is None:
            self.ptr = None
            return
        try:
            import torch
            is_t = isinstance(x, torch.Tensor)
        except ImportError:  # pragma: no cover
            is_t = False
        if is_t:
            if x.dtype != torch.float64 or not x.is_contiguous():
                if writable:
                    raise ValueError("output tensor must be contiguous float64")
                x = x.to(torch.float64).contiguous()
            if n is not None and x.numel() != n:
                raise ValueError(f"expected {n} values, got {x.numel()}")
            self.keep = x
            self.ptr = x.data_ptr()
        else:
            if writable:
                if not (isinstance(x, np.ndarray) and x.dtype == np.float64 and x.flags.c_contiguous):
                    raise ValueError("output array must be contiguous float64")
                arr = x
            else:
                arr = np.ascontiguousarray(x, dtype=np.float64)
            if n is not None and arr.size != n:
                raise ValueError(f"expected {n} values, got {arr.size}")
            self.keep = arr
            self.ptr = arr.ctypes.data


class Solver:
    """One library context (device buffers, stream, packed system)."""

    def __init__(self, device: int = 0, stream=None):
        L = lib()
        self._ctx = C.c_void_p()
        sp = None
        if stream is not None:
            sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        rc = L.bs32_create(C.byref(self._ctx), device, sp)
        if rc != 0:
            raise BS32Error(rc, "bs32_create failed")
        self.kind = None
        self.n = None
        self._opt = Options()
        L.bs32_default_options(C.byref(self._opt))

    def _check(self, rc, allow_positive=False):
        if rc < 0 or (rc > 0 and not allow_positive):
            msg = lib().bs32_last_error(self._ctx)
            raise BS32Error(rc, msg.decode() if msg else "")
        return rc

    def close(self):
        if self._ctx:
            lib().bs32_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- options
    @property
    def options(self):
        return {f: getattr(self._opt, f) for f, _ in Options._fields_}

    def set_options(self, **kw):
        o = Options()
        C.memmove(C.byref(o), C.byref(self._opt), C.sizeof(Options))
        for k, v in kw.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        self._check(lib().bs32_set_options(self._ctx, C.byref(o)))
        self._opt = o

    # -- system
    def set_system(self, kind, n, A=None, param=None, gain=1.0, stimulus=0.0, pairwise=False):
        Ab = _Buf(A, n * n)
        pb = _Buf(param, n)
        d = SystemDesc(kind, 0, n, Ab.ptr, pb.ptr, float(gain), float(stimulus), int(bool(pairwise)), 0)
        self._check(lib().bs32_set_system(self._ctx, C.byref(d)))
        self.kind, self.n = kind, n

    def set_workload(self, w):
        self.set_system(w["kind"], w["n"], w["A"], w["param"], w["gain"], w.get("stimulus", 0.0),
                        w.get("pairwise", False))

    # -- solve
    def solve(self, y0, t0, t1, rtol, atol=None, mode=PREC_FP64, out=None):
        """Integrate; returns (y_out, stats dict).  Solver terminations (status > 0)
        are reported in stats['status'], not raised."""
        m = DIM[self.kind] * self.n
        yb = _Buf(y0, m)
        if out is None:
            out = np.empty(m)
        ob = _Buf(out, m, writable=True)
        rc = lib().bs32_solve(self._ctx, yb.ptr, float(t0), float(t1), float(rtol),
                              float(rtol if atol is None else atol), int(mode), ob.ptr)
        self._check(rc, allow_positive=True)
        return out, self.stats()

    def stats(self):
        s = Stats()
        self._check(lib().bs32_stats(self._ctx, C.byref(s)))
        return s.as_dict()

    def rhs(self, y, mode=PREC_FP64, repeat=1, out=None):
        m = DIM[self.kind] * self.n
        yb = _Buf(y, m)
        if out is None:
            out = np.empty(m)
        ob = _Buf(out, m, writable=True)
        self._check(lib().bs32_rhs(self._ctx, yb.ptr, int(mode), int(repeat), ob.ptr))
        return out

    def time_contraction(self, mode=PREC_FP64, repeat=50):
        """Mean duration (ms) of one launch of the N^2 contraction kernel (HIP events)."""
        ms = C.c_double(0)
        self._check(lib().bs32_time_contraction(self._ctx, int(mode), int(repeat), C.byref(ms)))
        return ms.value

    # -- ensembles
    def set_ensemble(self, systems):
        """systems: list of dicts with kind, n, A, param, gain (same kind for all)."""
        keep = []
        descs = (SystemDesc * len(systems))()
        for q, w in enumerate(systems):
            Ab = _Buf(w.get("A"), w["n"] * w["n"])
            pb = _Buf(w.get("param"), w["n"])
            keep += [Ab, pb]
            descs[q] = SystemDesc(w["kind"], 0, w["n"], Ab.ptr, pb.ptr, float(w.get("gain", 1.0)),
                                  float(w.get("stimulus", 0.0)), int(bool(w.get("pairwise", False))), 0)
        self._check(lib().bs32_set_ensemble(self._ctx, len(systems), descs))
        self.kind = systems[0]["kind"]
        self.ens_n = [int(w["n"]) for w in systems]
        self.n = None

    def set_shared_ensemble(self, kind, n, count, A=None, params=None, gains=None):
        """`count` instances sharing one coupling A (n x n); params: count x n agent
        parameters (or None), gains: count values (or None = 1)."""
        Ab = _Buf(A, n * n)
        pb = _Buf(params, count * n) if params is not None else _Buf(None)
        g = None if gains is None else np.ascontiguousarray(np.broadcast_to(np.asarray(gains, np.float64), (count,)))
        d = SystemDesc(kind, 0, n, Ab.ptr, None, 1.0, 0.0, 0, 0)
        self._check(lib().bs32_set_shared_ensemble(self._ctx, C.byref(d), int(count), pb.ptr,
                                                   None if g is None else g.ctypes.data))
        self.kind = kind
        self.ens_n = [int(n)] * int(count)
        self.n = None

    def solve_batch(self, y0_concat, t0, t1, rtol, atol=None, mode=PREC_FP64, out=None):
        """Returns (y_out concatenated, per-instance status array, totals dict)."""
        B = len(self.ens_n)
        m = DIM[self.kind] * sum(self.ens_n)
        yb = _Buf(y0_concat, m)
        if out is None:
            out = np.empty(m)
        ob = _Buf(out, m, writable=True)
        t0a = np.ascontiguousarray(np.broadcast_to(np.asarray(t0, dtype=np.float64), (B,)))
        t1a = np.ascontiguousarray(np.broadcast_to(np.asarray(t1, dtype=np.float64), (B,)))
        st = np.zeros(B, dtype=np.int32)
        rc = lib().bs32_solve_batch(self._ctx, yb.ptr, t0a.ctypes.data, t1a.ctypes.data, float(rtol),
                                    float(rtol if atol is None else atol), int(mode), ob.ptr, st.ctypes.data)
        self._check(rc, allow_positive=True)
        return out, st, self.stats()

    def batch_stats(self, instance):
        s = Stats()
        self._check(lib().bs32_batch_stats(self._ctx, int(instance), C.byref(s)))
        return s.as_dict()

    def kernel_name(self, mode, tile):
        """Contraction kernel instance of a precision mode and candidate tile (profiler naming)."""
        buf = C.create_string_buffer(256)
        self._check(lib().bs32_kernel_name(self._ctx, int(mode), int(tile), buf, 256))
        return buf.value.decode()

    def packed_coupling(self, mode):
        """(stored N x N matrix as raw format values, power-of-two scale) for a precision mode."""
        if int(mode) == PREC_RHS_BF16X2:   # hi plane, then lo plane
            buf = np.empty((2, self.n, self.n), dtype=np.uint16)
        else:
            dt = {0: np.float64, 1: np.float32, 2: np.uint16, 3: np.uint16, 4: np.uint8}[min(int(mode), 4)]
            buf = np.empty((self.n, self.n), dtype=dt)
        sc = C.c_double(0)
        self._check(lib().bs32_get_packed_coupling(self._ctx, int(mode), buf.ctypes.data, buf.nbytes, C.byref(sc)))
        return buf, sc.value

    def trace(self, cap=1 << 20):
        buf = np.zeros(cap, dtype=_TRACE_DTYPE)
        n = C.c_size_t(0)
        self._check(lib().bs32_get_trace(self._ctx, buf.ctypes.data, cap, C.byref(n)))
        return buf[: n.value].copy()

    # -- accuracy diagnostics
    def set_record(self, states):
        """Record later solves into `states` (a float64 CUDA tensor of cap x d*N values, or
        None to stop): slot 0 the initial value, slot k the state after k accepted steps."""
        if states is None:
            self._check(lib().bs32_set_record(self._ctx, None, 0))
            self._rec = None
            return
        m = DIM[self.kind] * self.n
        if states.numel() % m != 0:
            raise ValueError(f"record size {states.numel()} is not a multiple of the state size {m}")
        b = _Buf(states, writable=True)
        self._check(lib().bs32_set_record(self._ctx, b.ptr, states.numel() // m))
        self._rec = states  # the library writes into it; keep it alive

    def lco_flow(self, n, X, h, out=None):
        """Analytic flow of eq. (LCO) (uniform weights): out[k] = exp(h[k] L) X[k] (CUDA tensors)."""
        import torch
        count = h.numel()
        if out is None:
            out = torch.empty(count * 2 * n, dtype=torch.float64, device=X.device)
        xb, hb, ob = _Buf(X, count * 2 * n), _Buf(h, count), _Buf(out, count * 2 * n, writable=True)
        self._check(lib().bs32_lco_flow(self._ctx, int(n), int(count), xb.ptr, hb.ptr, ob.ptr))
        return out

    def lco_local_error(self, n, states, h, delta, out=None):
        """eq. (LCO-Local-Error) of consecutive recorded states (CUDA tensors); returns err [steps]."""
        import torch
        steps = h.numel()
        if out is None:
            out = torch.empty(steps, dtype=torch.float64, device=h.device)
        sb, hb, ob = _Buf(states, None), _Buf(h, steps), _Buf(out, steps, writable=True)
        if states.numel() < (steps + 1) * 2 * n:
            raise ValueError("states must hold steps + 1 states")
        self._check(lib().bs32_lco_local_error(self._ctx, int(n), int(steps), sb.ptr, hb.ptr, float(delta), ob.ptr))
        return out

    # -- learned step-size proposer
    def set_controller(self, kind, weights=None):
        """kind 0: standard controller; kind 1: learned proposer with MLP_PARAMS weights."""
        w = None if weights is None else _f32(weights, MLP_PARAMS)
        self._check(lib().bs32_set_controller(self._ctx, int(kind), None if w is None else w.ctypes.data,
                                              0 if w is None else w.size))
        self._opt.controller = int(kind)

    def mlp_train(self, features, labels, epochs=50, batch=256, lr=1e-3, seed=0):
        """Train on the GPU; returns (weights [MLP_PARAMS] float32, loss per epoch [epochs])."""
        F = _f32(features)
        n = F.size // MLP_IN
        Y = _f32(labels, n)
        W = np.zeros(MLP_PARAMS, dtype=np.float32)
        L = np.zeros(int(epochs), dtype=np.float32)
        self._check(lib().bs32_mlp_train(self._ctx, F.ctypes.data, Y.ctypes.data, n, int(epochs), int(batch),
                                         float(lr), int(seed), W.ctypes.data, L.ctypes.data))
        return W, L

    def mlp_grad_noalloc(self, weights, features, labels, grad_out, loss_out=None):
        """bs32_mlp_grad_noalloc on device buffers (torch tensors or raw device pointers):
        weights / features / labels FP32, grad_out (MLP_PARAMS) and loss_out (1) FP64.
        Enqueued on the context's stream; returns without waiting."""
        def ptr(x):
            return None if x is None else (x if isinstance(x, int) else x.data_ptr())
        n = (features.numel() if hasattr(features, "numel") else 0) // MLP_IN
        self._check(lib().bs32_mlp_grad_noalloc(self._ctx, ptr(weights), ptr(features), ptr(labels), n,
                                                ptr(grad_out), ptr(loss_out)))

    def mlp_grad(self, weights, features, labels):
        """(gradient [MLP_PARAMS] float64, loss) of the training loss at BF16-rounded weights."""
        W = _f32(weights, MLP_PARAMS)
        F = _f32(features)
        n = F.size // MLP_IN
        Y = _f32(labels, n)
        g = np.zeros(MLP_PARAMS, dtype=np.float64)
        loss = C.c_double(0)
        self._check(lib().bs32_mlp_grad(self._ctx, W.ctypes.data, F.ctypes.data, Y.ctypes.data, n, g.ctypes.data,
                                        C.byref(loss)))
        return g, loss.value

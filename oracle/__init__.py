"""Plain CPU reference ("oracle") of the mixed-precision BS3(2) solver.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this package; the product library
never does, and this package never imports the product library.

The numerics live in ``bs32_oracle.c`` (FP64, pairwise definitions of the
paper's right-hand sides, Sec. 2.1; the BS3(2) pair with FSAL, Sec. 2.2; the
recipes of Sec. 2.3) and ``mlp.py`` (FP64 forward/backward of the step-size
proposer).  This module only marshals numpy arrays into the C library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liborc_bs32.so")
SRC_PATH = os.path.join(_HERE, "bs32_oracle.c")

OSC2, LCO_PAPER, KURAMOTO, GOODWIN3, CLOCK4 = 1, 2, 3, 4, 5
FMT_F64, FMT_F32, FMT_BF16, FMT_F16, FMT_E4M3, FMT_BF16X2 = 0, 1, 2, 3, 4, 5
(PREC_FP64, PREC_RHS_FP32, PREC_RHS_BF16, PREC_RHS_FP16, PREC_RHS_FP8,
 PREC_PAPER_SINGLE, PREC_PAPER_MIXED1, PREC_PAPER_MIXED2, PREC_RHS_BF16X2) = range(9)
OK, MAX_STEPS, MAX_REJECTS, H_TOO_SMALL, NONFINITE = 0, 1, 2, 3, 6
DIM = {OSC2: 2, LCO_PAPER: 2, KURAMOTO: 1, GOODWIN3: 3, CLOCK4: 4}
MLP_IN, MLP_HID, MLP_PARAMS = 9, 64, 4883


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11 + OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                        SRC_PATH, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class System(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int64), ("A", C.c_void_p), ("param", C.c_void_p),
                ("gain", C.c_double), ("stimulus", C.c_double)]


class Options(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("h_max", C.c_double), ("h0", C.c_double),
                ("i_max", C.c_int64), ("fixed_step", C.c_int32), ("safety", C.c_double),
                ("facmin", C.c_double), ("facmax", C.c_double), ("split_terms", C.c_int32),
                ("split_fmt", C.c_int32), ("split_shift", C.c_int32), ("mlp_w", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("n_accept", C.c_int64), ("n_reject", C.c_int64), ("n_fev", C.c_int64),
                ("t_reached", C.c_double), ("h_last", C.c_double), ("h_next", C.c_double),
                ("err_last", C.c_double), ("h_min_seen", C.c_double), ("status", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TraceRec(C.Structure):
    _fields_ = [("t", C.c_double), ("h", C.c_double), ("err", C.c_double), ("fnorm", C.c_double),
                ("accepted", C.c_int32), ("proposer", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.orc_rhs.argtypes = [P, C.c_double, P, P]
        L.orc_rhs_rows.argtypes = [P, P, C.c_int64, P, C.c_double, P, P]
        L.orc_rhs_lowp.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, P, P]
        L.orc_rhs_lowp_rows.argtypes = [P, C.c_int, C.c_double, P, C.c_int64, P, C.c_double, P, P]
        L.orc_rhs_recipe.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_double, P, P]
        L.orc_round_fmt.argtypes = [C.c_double, C.c_int]
        L.orc_round_fmt.restype = C.c_double
        L.orc_encode_fmt.argtypes = [C.c_double, C.c_int]
        L.orc_encode_fmt.restype = C.c_uint32
        L.orc_decode_fmt.argtypes = [C.c_uint32, C.c_int]
        L.orc_decode_fmt.restype = C.c_double
        L.orc_matrix_scale.argtypes = [P, C.c_int64, C.c_int]
        L.orc_matrix_scale.restype = C.c_double
        L.orc_split.argtypes = [C.c_double, C.c_int, C.c_int, C.c_int, P]
        L.orc_bs32_solve.argtypes = [P, P, C.c_int, P, C.c_double, C.c_double, P, P, P, C.c_int64, P]
        L.orc_dp54_solve.argtypes = [P, P, P, C.c_double, C.c_double, P, P]
        L.orc_rkf45_solve.argtypes = [P, P, P, C.c_double, C.c_double, P, P]
        L.orc_rkf45_tableau.argtypes = [P, P, P, P]
        L.orc_bs32_attempt.argtypes = [P, C.c_double, C.c_double, P, P, C.c_double, C.c_double, P, P, P]
        L.orc_bs32_tableau.argtypes = [P, P, P, P]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        L.orc_mlp_forward.argtypes = [P, P]
        L.orc_mlp_forward.restype = C.c_double
        L.orc_dp54_tableau.argtypes = [P, P, P, P]
        L.orc_recipe_table.argtypes = [P]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data


class _Sys:
    """Keeps the numpy buffers alive while the C struct points at them."""

    def __init__(self, kind, n, A=None, param=None, gain=1.0, stimulus=0.0):
        self.A = None if A is None else _f64(A).reshape(-1)
        self.param = None if param is None else _f64(param)
        if self.A is not None:
            assert self.A.size == n * n
        if self.param is not None:
            assert self.param.size == n
        self.s = System(kind, n, _ptr(self.A), _ptr(self.param), float(gain), float(stimulus))

    @property
    def ref(self):
        return C.byref(self.s)


def rhs(kind, n, y, A=None, param=None, gain=1.0, stimulus=0.0, t=0.0):
    s = _Sys(kind, n, A, param, gain, stimulus)
    y = _f64(y)
    f = np.empty_like(y)
    assert lib().orc_rhs(s.ref, t, _ptr(y), _ptr(f)) == 0
    return f


def rhs_rows(kind, n, rows, y, A_rows=None, param=None, gain=1.0, stimulus=0.0, t=0.0):
    s = _Sys(kind, n, None, param, gain, stimulus)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    y = _f64(y)
    Ar = None if A_rows is None else _f64(A_rows).reshape(-1)
    if Ar is not None:
        assert Ar.size == rows.size * n
    f = np.empty(rows.size * DIM[kind])
    assert lib().orc_rhs_rows(s.ref, _ptr(rows), rows.size, _ptr(Ar), t, _ptr(y), _ptr(f)) == 0
    return f


def rhs_lowp(kind, n, y, fmt, A=None, param=None, gain=1.0, stimulus=0.0, split_fmt=-1, split_terms=0, split_shift=0, t=0.0):
    s = _Sys(kind, n, A, param, gain, stimulus)
    y = _f64(y)
    f = np.empty_like(y)
    assert lib().orc_rhs_lowp(s.ref, fmt, split_fmt, split_terms, split_shift, t, _ptr(y), _ptr(f)) == 0
    return f


def rhs_lowp_rows(kind, n, rows, y, fmt, scale, A_rows=None, param=None, gain=1.0, stimulus=0.0, t=0.0):
    """Reduced-precision right-hand side of the listed rows; scale = matrix_scale of the
    whole matrix (of its largest magnitude)."""
    s = _Sys(kind, n, None, param, gain, stimulus)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    y = _f64(y)
    Ar = None if A_rows is None else _f64(A_rows).reshape(-1)
    if Ar is not None:
        assert Ar.size == rows.size * n
    f = np.empty(rows.size * DIM[kind])
    rc = lib().orc_rhs_lowp_rows(s.ref, fmt, float(scale), _ptr(rows), rows.size, _ptr(Ar), t, _ptr(y), _ptr(f))
    assert rc == 0
    return f


def rhs_recipe(kind, n, y, pF, pS, pG, A=None, param=None, gain=1.0, stimulus=0.0, t=0.0):
    s = _Sys(kind, n, A, param, gain, stimulus)
    y = _f64(y)
    f = np.empty_like(y)
    assert lib().orc_rhs_recipe(s.ref, pF, pS, pG, t, _ptr(y), _ptr(f)) == 0
    return f


def round_fmt(x, fmt):
    L = lib()
    return np.array([L.orc_round_fmt(float(v), fmt) for v in np.ravel(x)]).reshape(np.shape(x))


def encode_fmt(x, fmt):
    L = lib()
    return np.array([L.orc_encode_fmt(float(v), fmt) for v in np.ravel(x)], dtype=np.uint32).reshape(np.shape(x))


def decode_fmt(bits, fmt):
    L = lib()
    return np.array([L.orc_decode_fmt(int(b), fmt) for b in np.ravel(bits)]).reshape(np.shape(bits))


def matrix_scale(A, fmt):
    A = _f64(A).reshape(-1)
    return lib().orc_matrix_scale(_ptr(A), A.size, fmt)


def split(v, fmt, terms, shift):
    out = np.empty(terms)
    lib().orc_split(float(v), fmt, terms, shift, _ptr(out))
    return out


def options(rtol, atol=None, h_max=0.0, h0=0.0, i_max=0, fixed_step=False, safety=0.0, facmin=0.0,
            facmax=0.0, split_terms=0, split_fmt=-1, split_shift=0):
    return Options(rtol, rtol if atol is None else atol, h_max, h0, i_max, int(fixed_step), safety, facmin,
                   facmax, split_terms, split_fmt, split_shift)


def bs32_solve(kind, n, y0, t0, t1, rtol, atol=None, A=None, param=None, gain=1.0, stimulus=0.0, mode=PREC_FP64,
               trace_cap=0, mlp_w=None, **opt):
    """Adaptive BS3(2)+FSAL solve.  Returns (y, stats dict, trace array or None).

    mlp_w: MLP_PARAMS weights of the learned step-size proposer (None: standard controller)."""
    s = _Sys(kind, n, A, param, gain, stimulus)
    o = options(rtol, atol, **opt)
    w = None
    if mlp_w is not None:
        w = _f64(mlp_w)
        assert w.size == MLP_PARAMS
        o.mlp_w = w.ctypes.data
    y0 = _f64(y0)
    y = np.empty_like(y0)
    st = Stats()
    tr = (TraceRec * trace_cap)() if trace_cap else None
    tl = C.c_int64(0)
    rc = lib().orc_bs32_solve(s.ref, C.byref(o), mode, _ptr(y0), t0, t1, _ptr(y), C.byref(st),
                              C.cast(tr, C.c_void_p) if tr is not None else None, trace_cap, C.byref(tl))
    if rc < 0:
        raise ValueError(f"oracle solve rejected its arguments (kind {kind}, mode {mode})")
    trace = None
    if tr is not None:
        trace = np.array([(r.t, r.h, r.err, r.fnorm, r.accepted, r.proposer) for r in tr[: tl.value]],
                         dtype=[("t", "f8"), ("h", "f8"), ("err", "f8"), ("fnorm", "f8"), ("accepted", "i4"),
                                ("proposer", "i4")])
    return y, st.as_dict(), trace


def set_threads(n):
    """OpenMP threads of the oracle's row loops (n <= 0 keeps the current setting)."""
    lib().orc_set_threads(int(n))


def threads():
    return int(lib().orc_get_threads())


def mlp_forward(w, f):
    """FP64 network output for one feature vector (the C oracle's evaluation)."""
    w = _f64(w)
    f = _f64(f)
    assert w.size == MLP_PARAMS and f.size == MLP_IN
    return lib().orc_mlp_forward(_ptr(w), _ptr(f))


def dp54_solve(kind, n, y0, t0, t1, rtol, atol=None, A=None, param=None, gain=1.0, stimulus=0.0, **opt):
    s = _Sys(kind, n, A, param, gain, stimulus)
    o = options(rtol, atol, **opt)
    y0 = _f64(y0)
    y = np.empty_like(y0)
    st = Stats()
    lib().orc_dp54_solve(s.ref, C.byref(o), _ptr(y0), t0, t1, _ptr(y), C.byref(st))
    return y, st.as_dict()


def rkf45_solve(kind, n, y0, t0, t1, rtol, atol=None, A=None, param=None, gain=1.0, stimulus=0.0, **opt):
    s = _Sys(kind, n, A, param, gain, stimulus)
    o = options(rtol, atol, **opt)
    y0 = _f64(y0)
    y = np.empty_like(y0)
    st = Stats()
    lib().orc_rkf45_solve(s.ref, C.byref(o), _ptr(y0), t0, t1, _ptr(y), C.byref(st))
    return y, st.as_dict()


def rkf45_tableau():
    c, a, b, bh = np.empty(6), np.empty(36), np.empty(6), np.empty(6)
    lib().orc_rkf45_tableau(_ptr(c), _ptr(a), _ptr(b), _ptr(bh))
    return c, a.reshape(6, 6), b, bh


def bs32_attempt(kind, n, t, h, X, K1, rtol, atol=None, A=None, param=None, gain=1.0, stimulus=0.0):
    s = _Sys(kind, n, A, param, gain, stimulus)
    X = _f64(X)
    K1 = _f64(K1)
    Xn = np.empty_like(X)
    K4 = np.empty_like(X)
    err = C.c_double(0)
    lib().orc_bs32_attempt(s.ref, t, h, _ptr(X), _ptr(K1), rtol, rtol if atol is None else atol, _ptr(Xn),
                           _ptr(K4), C.byref(err))
    return Xn, K4, err.value


def bs32_tableau():
    c, a, b, bt = np.empty(4), np.empty(16), np.empty(4), np.empty(4)
    lib().orc_bs32_tableau(_ptr(c), _ptr(a), _ptr(b), _ptr(bt))
    return c, a.reshape(4, 4), b, bt


def dp54_tableau():
    c, a, b, bt = np.empty(7), np.empty(49), np.empty(7), np.empty(7)
    lib().orc_dp54_tableau(_ptr(c), _ptr(a), _ptr(b), _ptr(bt))
    return c, a.reshape(7, 7), b, bt


def recipe_table():
    """{(solver, stage): (F, Sigma, G)} with 1 = single, as the integrator uses it."""
    out = np.zeros(27, dtype=np.int32)
    lib().orc_recipe_table(_ptr(out))
    t = {}
    for r, solver in enumerate(("Single", "Mixed1", "Mixed2")):
        for k, stage in enumerate(("k2", "k3", "k4")):
            t[(solver, stage)] = tuple(int(v) for v in out[9 * r + 3 * k: 9 * r + 3 * k + 3])
    return t

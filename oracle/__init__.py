"""FP64 CPU oracle for order-statistics directional filters (arXiv:1009.0958).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check
and the benchmark's CPU-baseline leg may import this package.  It never
imports the GPU package and the GPU package never imports it.

The arithmetic lives in ``odf_oracle.c`` (plain C, IEEE double, direct
per-window definitions of eqs. 1-3, 4-7 and 10); this module only marshals
numpy arrays.  Images are ``(B, M, N, 3)`` or ``(M, N, 3)`` arrays of any
real dtype; they are promoted to float64 exactly (uint8 and float32 values
are representable in double).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "odf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BVDF, DDF = 0, 1
EXACT, MINIMAX, RGB = 0, 1, 2

_lib = None


def build(force: bool = False) -> str:
    """Compile ``odf_oracle.c`` into ``liboracle.so`` (gcc, -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        # ODF_ORACLE_LIB: a prebuilt copy of the same source (the sanitizer
        # test's instrumented build); otherwise build in place when stale
        path = os.environ.get("ODF_ORACLE_LIB")
        if not path:
            path = build()
        lib = ctypes.CDLL(path)
        P, I, D, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
        lib.oracle_threads.restype = I
        lib.oracle_pair_terms.argtypes = [P, P, I64, I, I, I, P, P]
        lib.oracle_filter.argtypes = [P, I, I, I, I, I, D, I, I, P, P, P, P, P, I]
        lib.oracle_filter_at.argtypes = [P, I, I, I, I, I, D, I, I, P, I64, P, P, P, P, P, I]
        lib.oracle_backward_hard.argtypes = [P, P, I, I, I, I, P]
        lib.oracle_softmin_fwd.argtypes = [P, I, I, I, I, I, D, D, P, P, I]
        lib.oracle_softmin_bwd.argtypes = [P, P, I, I, I, I, I, D, D, P, I]
        lib.oracle_acwddf.argtypes = [P, I, I, I, I, I, I, I, D, P, P, P, P, I]
        lib.oracle_acwddf_at.argtypes = [P, I, I, I, I, I, I, I, D, P, I64, P, P, P, P, I]
        lib.oracle_cwfilter.argtypes = [P, I, I, I, I, I, I, I, I, P, P, P, I]
        for f in (lib.oracle_pair_terms, lib.oracle_filter, lib.oracle_filter_at,
                  lib.oracle_backward_hard, lib.oracle_softmin_fwd, lib.oracle_softmin_bwd,
                  lib.oracle_acwddf, lib.oracle_acwddf_at, lib.oracle_cwfilter):
            f.restype = I
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _batch(img):
    x = np.ascontiguousarray(np.asarray(img), dtype=np.float64)
    squeeze = x.ndim == 3
    if squeeze:
        x = x[None]
    if x.ndim != 4 or x.shape[-1] != 3:
        raise ValueError("image must be (M, N, 3) or (B, M, N, 3)")
    return x, squeeze


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s rejected its arguments" % what)


def threads() -> int:
    """Number of OpenMP threads the oracle uses by default."""
    return _load().oracle_threads()


def pair_terms(a, b, kind=BVDF, dist=EXACT, q=4):
    """Pair terms theta(a_i, b_i) of the chosen variant and L2(a_i, b_i), float64 arrays."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, 3))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(-1, 3))
    if a.shape != b.shape:
        raise ValueError("a and b must have the same number of vectors")
    th = np.empty(a.shape[0])
    l2 = np.empty(a.shape[0])
    _check(_load().oracle_pair_terms(_ptr(a), _ptr(b), a.shape[0], kind, dist, q, _ptr(th),
                                     _ptr(l2)), "pair_terms")
    return th, l2


def filter(img, window=3, kind=BVDF, p=0.5, dist=EXACT, q=4, aggregates=False, nthreads=0):
    """Full filter.  Returns (out, idx) or (out, idx, A, D, Omega) when ``aggregates``.

    out is float64 with the shape of ``img`` (an exact copy of the selected
    member), idx uint8 (row-major window index), A/D/Omega float64 (..., n).
    """
    x, squeeze = _batch(img)
    B, M, N, _ = x.shape
    n = window * window
    out = np.empty_like(x)
    idx = np.empty((B, M, N), np.uint8)
    A = D = O = None
    if aggregates:
        A = np.empty((B, M, N, n))
        D = np.empty((B, M, N, n))
        O = np.empty((B, M, N, n))
    _check(_load().oracle_filter(_ptr(x), B, M, N, window, kind, float(p), dist, q, _ptr(out),
                                 _ptr(idx), _ptr(A), _ptr(D), _ptr(O), nthreads), "filter")
    res = [out, idx] + ([A, D, O] if aggregates else [])
    if squeeze:
        res = [r[0] for r in res]
    return tuple(res)


def filter_at(img, pix, window=3, kind=BVDF, p=0.5, dist=EXACT, q=4, nthreads=0):
    """Filter evaluated only at flat pixel positions ``pix`` ((b*M + r)*N + c).

    Returns (out (k,3), idx (k,), A (k,n), D (k,n), Omega (k,n)).
    """
    x, _ = _batch(img)
    B, M, N, _ = x.shape
    n = window * window
    pix = np.ascontiguousarray(np.asarray(pix, dtype=np.int64).ravel())
    k = pix.shape[0]
    out = np.empty((k, 3))
    idx = np.empty(k, np.uint8)
    A, D, O = np.empty((k, n)), np.empty((k, n)), np.empty((k, n))
    _check(_load().oracle_filter_at(_ptr(x), B, M, N, window, kind, float(p), dist, q, _ptr(pix),
                                    k, _ptr(out), _ptr(idx), _ptr(A), _ptr(D), _ptr(O), nthreads),
           "filter_at")
    return out, idx, A, D, O


def backward_hard(idx, dy, window=3):
    """Gradient of the hard filter: dy routed to the selected source pixels."""
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint8))
    dyb, squeeze = _batch(dy)
    B, M, N, _ = dyb.shape
    idx = idx.reshape(B, M, N)
    dx = np.empty_like(dyb)
    _check(_load().oracle_backward_hard(_ptr(idx), _ptr(dyb), B, M, N, window, _ptr(dx)),
           "backward_hard")
    return dx[0] if squeeze else dx


def softmin_fwd(img, window=5, kind=DDF, p=0.25, tau=0.1, weights=False, nthreads=0):
    """Softmin relaxation y = sum_u pi_u x_u; returns y (and pi (..., n) if ``weights``)."""
    x, squeeze = _batch(img)
    B, M, N, _ = x.shape
    y = np.empty_like(x)
    pi = np.empty((B, M, N, window * window)) if weights else None
    _check(_load().oracle_softmin_fwd(_ptr(x), B, M, N, window, kind, float(p), float(tau),
                                      _ptr(y), _ptr(pi), nthreads), "softmin_fwd")
    if squeeze:
        y = y[0]
        pi = None if pi is None else pi[0]
    return (y, pi) if weights else y


def softmin_bwd(img, dy, window=5, kind=DDF, p=0.25, tau=0.1, nthreads=0):
    """Analytic gradient of sum(dy * softmin_fwd(img)) with respect to img."""
    x, squeeze = _batch(img)
    g, _ = _batch(dy)
    B, M, N, _ = x.shape
    if g.shape != x.shape:
        raise ValueError("dy must have the shape of img")
    dx = np.empty_like(x)
    _check(_load().oracle_softmin_bwd(_ptr(x), _ptr(g), B, M, N, window, kind, float(p),
                                      float(tau), _ptr(dx), nthreads), "softmin_bwd")
    return dx[0] if squeeze else dx


def acwddf(img, window=3, dist=EXACT, q=4, lam=2, T=10.8, diag=False, nthreads=0):
    """Adaptive centre-weighted DDF (Section III, Experiment 2; eq. 9).

    Returns (out, idx, S) or (out, idx, S, diag) when ``diag``: out float64
    with the shape of ``img``, idx uint8 (the DDF selection where S > T, else
    the centre (n - 1) / 2), S float64 (the switching statistic), diag
    float64 (..., 5n): the eq. (3) objective, the three centre-weighted
    objectives (k = lam, lam + 1, lam + 2) and A(x_u, x_d) * L2(x_u, x_d).
    """
    x, squeeze = _batch(img)
    B, M, N, _ = x.shape
    n = window * window
    out = np.empty_like(x)
    idx = np.empty((B, M, N), np.uint8)
    S = np.empty((B, M, N))
    dg = np.empty((B, M, N, 5 * n)) if diag else None
    _check(_load().oracle_acwddf(_ptr(x), B, M, N, window, dist, q, int(lam), float(T), _ptr(out),
                                 _ptr(idx), _ptr(S), _ptr(dg), nthreads), "acwddf")
    res = [out, idx, S] + ([dg] if diag else [])
    if squeeze:
        res = [r[0] for r in res]
    return tuple(res)


def acwddf_at(img, pix, window=3, dist=EXACT, q=4, lam=2, T=10.8, nthreads=0):
    """ACWDDF at flat pixel positions ``pix``: (out (k,3), idx (k,), S (k,), diag (k, 5n))."""
    x, _ = _batch(img)
    B, M, N, _ = x.shape
    n = window * window
    pix = np.ascontiguousarray(np.asarray(pix, dtype=np.int64).ravel())
    k = pix.shape[0]
    out, idx, S, dg = np.empty((k, 3)), np.empty(k, np.uint8), np.empty(k), np.empty((k, 5 * n))
    _check(_load().oracle_acwddf_at(_ptr(x), B, M, N, window, dist, q, int(lam), float(T),
                                    _ptr(pix), k, _ptr(out), _ptr(idx), _ptr(S), _ptr(dg),
                                    nthreads), "acwddf_at")
    return out, idx, S, dg


def cwfilter(img, window=3, vmf=True, dist=EXACT, q=4, level=1, nthreads=0):
    """Centre-weighted filters (Section III, eq. 9): CWVMF^k (vmf) minimises
    sum_v w_v(k) L2(x_u, x_v) with w_d(k) = n - 2k + 2 on the centre member and
    1 elsewhere; CWDDF^k (not vmf) minimises the product of the weighted angle
    and L2 sums (the pair term of `dist`, eq. 10 for chromaticity).
    Returns (out, idx, obj): obj (..., n) the objective of every member."""
    x, squeeze = _batch(img)
    B, M, N, _ = x.shape
    n = window * window
    out = np.empty_like(x)
    idx = np.empty((B, M, N), np.uint8)
    obj = np.empty((B, M, N, n))
    _check(_load().oracle_cwfilter(_ptr(x), B, M, N, window, int(bool(vmf)), dist, q, int(level),
                                   _ptr(out), _ptr(idx), _ptr(obj), nthreads), "cwfilter")
    res = (out, idx, obj)
    return tuple(r[0] for r in res) if squeeze else res

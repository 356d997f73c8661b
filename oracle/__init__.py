"""FastFCA reference oracle (FP64, CPU) -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The GPU library never does, and shares
no code with it: the oracle is a plain C99 file (``fastfca_oracle.c``) built
with gcc, following Algorithm 1 / Algorithm 2 (Sec. IV-E), the negative
log-likelihood of Sec. IV-D (eq:negll) and the multichannel Wiener filter of
Sec. IV-F (eq:Doclo) step by step in double precision.

Arrays use the paper's roles with the library's layouts:
    x   [F,T,M] complex    P [F,M,M] complex (column m is w_m)
    lam [F,N,M] real       v [F,T,N] real      y [N,F,T,M] complex

The ``mnmf_*`` functions are FastMNMF (Sec. V and its appendix): h_{ijn} =
sum_k t_{ikn} v_{jkn} with tp [I,K,N] and va [J,K,N].

The ``*_blocks`` functions are the piecewise stationary extension (Sec. VI):
blocks of B consecutive frames share h, the input of the algorithms is the
block covariance Xhat_j, and v is [F,J,N] with J = T / B.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fastfca_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK = 0
E_SINGULAR = -4


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP over frequencies)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        c_int, c_double, vp = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        lib.ofc_weighted_cov.argtypes = [c_int, c_int, c_int, vp, vp, vp, vp]
        lib.ofc_ip_column.argtypes = [c_int, vp, vp, c_int]
        lib.ofc_ip_column.restype = c_int
        lib.ofc_decorrelated_power.argtypes = [c_int, c_int, vp, vp, vp]
        lib.ofc_em_source.argtypes = [c_int, c_int, c_int, vp, vp, vp, c_int, vp]
        lib.ofc_mm_update.argtypes = [c_int, c_int, c_int, vp, vp, vp, vp]
        lib.ofc_logabsdet2.argtypes = [c_int, vp]
        lib.ofc_logabsdet2.restype = c_double
        lib.ofc_loglik_freq.argtypes = [c_int, c_int, c_int, vp, vp, vp, vp]
        lib.ofc_loglik_freq.restype = c_double
        lib.ofc_iterate_freq.argtypes = [c_int, c_int, c_int, vp, vp, vp, vp, c_int, c_int, vp, vp]
        lib.ofc_iterate_freq.restype = c_int
        lib.ofc_fit.argtypes = [c_int, c_int, c_int, c_int, vp, vp, vp, vp, c_int, c_int, vp, c_int]
        lib.ofc_fit.restype = c_int
        lib.ofc_loglik.argtypes = [c_int, c_int, c_int, c_int, vp, vp, vp, vp, vp]
        lib.ofc_loglik.restype = c_double
        lib.ofc_mwf.argtypes = [c_int, c_int, c_int, c_int, vp, vp, vp, vp, vp]
        lib.ofc_mwf.restype = c_int
        lib.ofc_num_threads.restype = c_int
        lib.ofc_block_cov.argtypes = [c_int, c_int, c_int, vp, vp]
        lib.ofc_weighted_cov_blocks.argtypes = [c_int, c_int, c_int, vp, vp, vp, vp]
        lib.ofc_block_power.argtypes = [c_int, c_int, vp, vp, vp]
        lib.ofc_loglik_blocks_freq.argtypes = [c_int, c_int, c_int, vp, vp, vp, vp]
        lib.ofc_loglik_blocks_freq.restype = c_double
        lib.ofc_fit_blocks.argtypes = [c_int, c_int, c_int, c_int, c_int, vp, vp, vp, vp, c_int, c_int, vp,
                                       c_int]
        lib.ofc_fit_blocks.restype = c_int
        lib.ofc_loglik_blocks.argtypes = [c_int, c_int, c_int, c_int, c_int, vp, vp, vp, vp, vp]
        lib.ofc_loglik_blocks.restype = c_double
        lib.ofc_mwf_blocks.argtypes = [c_int, c_int, c_int, c_int, c_int, vp, vp, vp, vp, vp]
        lib.ofc_mwf_blocks.restype = c_int
        lib.ofc_mnmf_h.argtypes = [c_int, c_int, c_int, c_int, vp, vp, vp]
        lib.ofc_mnmf_loglik.argtypes = [c_int, c_int, c_int, c_int, c_int, vp, vp, vp, vp, vp, vp]
        lib.ofc_mnmf_loglik.restype = c_double
        lib.ofc_mnmf_iterate.argtypes = [c_int, c_int, c_int, c_int, c_int, vp, vp, vp, vp, vp, c_int]
        lib.ofc_mnmf_iterate.restype = c_int
        lib.ofc_mnmf_fit.argtypes = [c_int, c_int, c_int, c_int, c_int, vp, vp, vp, vp, vp, c_int, vp]
        lib.ofc_mnmf_fit.restype = c_int
        _lib = lib
    return _lib


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().ofc_num_threads())


# ---------------------------------------------------------------- per frequency
def weighted_cov(x, lam, v):
    """Q[m] = (1/T) sum_t x_t x_t^H / sigma^2_{mt} for one frequency (eq:wsampcov).
    x [T,M], lam [N,M], v [T,N] -> Q [M,M,M]."""
    x, lam, v = _c128(x), _f64(lam), _f64(v)
    T, M = x.shape
    N = lam.shape[0]
    Q = np.zeros((M, M, M), np.complex128)
    _load().ofc_weighted_cov(T, M, N, _p(x), _p(lam), _p(v), _p(Q))
    return Q


def ip_column(P, Qm, m):
    """IP update of column m (eq:ip1, eq:ip2). Returns the new P (copy)."""
    P = _c128(P).copy()
    Qm = _c128(Qm)
    st = _load().ofc_ip_column(P.shape[0], _p(P), _p(Qm), int(m))
    if st != OK:
        raise FloatingPointError("ofc_ip_column status %d" % st)
    return P


def decorrelated_power(P, x):
    """U [M,T] = |P^H x_t|^2 (eq:Udef)."""
    P, x = _c128(P), _c128(x)
    T, M = x.shape
    U = np.zeros((M, T), np.float64)
    _load().ofc_decorrelated_power(T, M, _p(P), _p(x), _p(U))
    return U


def em_source(U, lam, v, n):
    """EM update of source n (Algorithm 1, loop body over n). Returns (lam, v) copies."""
    U, lam, v = _f64(U), _f64(lam).copy(), _f64(v).copy()
    M, T = U.shape
    N = lam.shape[0]
    phi = np.zeros(M * T, np.float64)
    _load().ofc_em_source(T, M, N, _p(U), _p(lam), _p(v), int(n), _p(phi))
    return lam, v


def mm_update(U, lam, v):
    """MM update of L then H (Algorithm 2). Returns (lam, v) copies."""
    U, lam, v = _f64(U), _f64(lam).copy(), _f64(v).copy()
    M, T = U.shape
    N = lam.shape[0]
    scratch = np.zeros(2 * M * T, np.float64)
    _load().ofc_mm_update(T, M, N, _p(U), _p(lam), _p(v), _p(scratch))
    return lam, v


def logabsdet2(P):
    P = _c128(P)
    return float(_load().ofc_logabsdet2(P.shape[0], _p(P)))


def loglik_freq(x, P, lam, v):
    """LL per bin of one frequency (eq:negll, sign flipped, /T, M ln pi restored)."""
    x, P, lam, v = _c128(x), _c128(P), _f64(lam), _f64(v)
    T, M = x.shape
    N = lam.shape[0]
    return float(_load().ofc_loglik_freq(T, M, N, _p(x), _p(P), _p(lam), _p(v)))


def iterate_freq(x, P, lam, v, what=3, algo=0):
    """One iteration on one frequency; what bit0 = IP sweep, bit1 = L/H update;
    algo 0 = EM (Algorithm 1), 1 = MM (Algorithm 2). Returns (P, lam, v) copies."""
    x = _c128(x)
    P, lam, v = _c128(P).copy(), _f64(lam).copy(), _f64(v).copy()
    T, M = x.shape
    N = lam.shape[0]
    Qw = np.zeros(M * M * M, np.complex128)
    dw = np.zeros(3 * M * T, np.float64)
    st = _load().ofc_iterate_freq(T, M, N, _p(x), _p(P), _p(lam), _p(v), int(what), int(algo),
                                  _p(Qw), _p(dw))
    if st != OK:
        raise FloatingPointError("ofc_iterate_freq status %d" % st)
    return P, lam, v


# ---------------------------------------------------------------- all frequencies
def fit(x, P, lam, v, n_iter, algo=0, trace=False, nthreads=0):
    """Run n_iter iterations on every frequency. Inputs are not modified.
    Returns (P, lam, v, ll_trace) with ll_trace [n_iter] = LL/bin after each
    iteration (mean over f of the per-frequency LL) or None."""
    x = _c128(x)
    P, lam, v = _c128(P).copy(), _f64(lam).copy(), _f64(v).copy()
    F, T, M = x.shape
    N = lam.shape[1]
    tr = np.zeros((F, max(n_iter, 1)), np.float64) if trace else None
    st = _load().ofc_fit(F, T, M, N, _p(x), _p(P), _p(lam), _p(v), int(n_iter), int(algo),
                         _p(tr) if trace else None, int(nthreads))
    if st != OK:
        raise FloatingPointError("ofc_fit status %d" % st)
    return P, lam, v, (tr[:, :n_iter].mean(axis=0) if trace else None)


def loglik(x, P, lam, v):
    """(LL per bin, per-frequency LL [F])."""
    x, P, lam, v = _c128(x), _c128(P), _f64(lam), _f64(v)
    F, T, M = x.shape
    N = lam.shape[1]
    llf = np.zeros(F, np.float64)
    ll = _load().ofc_loglik(F, T, M, N, _p(x), _p(P), _p(lam), _p(v), _p(llf))
    return float(ll), llf


def mwf(x, P, lam, v):
    """Source images y [N,F,T,M] by eq:Doclo."""
    x, P, lam, v = _c128(x), _c128(P), _f64(lam), _f64(v)
    F, T, M = x.shape
    N = lam.shape[1]
    y = np.zeros((N, F, T, M), np.complex128)
    st = _load().ofc_mwf(F, T, M, N, _p(x), _p(P), _p(lam), _p(v), _p(y))
    if st != OK:
        raise FloatingPointError("ofc_mwf status %d" % st)
    return y


# ---------------------------------------------------------------- piecewise stationary (Sec. VI)
def block_cov(x, B):
    """Xhat [J,M,M] = (1/B) sum_b x x^H over blocks of B frames of one frequency x [T,M]."""
    x = _c128(x)
    T, M = x.shape
    J = T // B
    Xh = np.zeros((J, M, M), np.complex128)
    _load().ofc_block_cov(J, int(B), M, _p(x), _p(Xh))
    return Xh


def weighted_cov_blocks(Xh, lam, v):
    """Q [M,M,M] = (1/J) sum_j Xhat_j / sigma^2_{mj} for one frequency."""
    Xh, lam, v = _c128(Xh), _f64(lam), _f64(v)
    J, M, _ = Xh.shape
    N = lam.shape[0]
    Q = np.zeros((M, M, M), np.complex128)
    _load().ofc_weighted_cov_blocks(J, M, N, _p(Xh), _p(lam), _p(v), _p(Q))
    return Q


def block_power(P, Xh):
    """U [M,J] = w_m^H Xhat_j w_m."""
    P, Xh = _c128(P), _c128(Xh)
    J, M, _ = Xh.shape
    U = np.zeros((M, J), np.float64)
    _load().ofc_block_power(J, M, _p(P), _p(Xh), _p(U))
    return U


def loglik_blocks_freq(Xh, P, lam, v):
    """Block-model LL per frame of one frequency (eq:negllpws, sign flipped, /J, M ln pi restored)."""
    Xh, P, lam, v = _c128(Xh), _c128(P), _f64(lam), _f64(v)
    J, M, _ = Xh.shape
    N = lam.shape[0]
    return float(_load().ofc_loglik_blocks_freq(J, M, N, _p(Xh), _p(P), _p(lam), _p(v)))


def fit_blocks(x, B, P, lam, v, n_iter, algo=0, trace=False, nthreads=0):
    """fit() for the block model: v [F,J,N]. Returns (P, lam, v, ll_trace)."""
    x = _c128(x)
    P, lam, v = _c128(P).copy(), _f64(lam).copy(), _f64(v).copy()
    F, T, M = x.shape
    N = lam.shape[1]
    tr = np.zeros((F, max(n_iter, 1)), np.float64) if trace else None
    st = _load().ofc_fit_blocks(F, T, M, N, int(B), _p(x), _p(P), _p(lam), _p(v), int(n_iter), int(algo),
                                _p(tr) if trace else None, int(nthreads))
    if st != OK:
        raise FloatingPointError("ofc_fit_blocks status %d" % st)
    return P, lam, v, (tr[:, :n_iter].mean(axis=0) if trace else None)


def loglik_blocks(x, B, P, lam, v):
    """(LL per frame, per-frequency LL [F]) of the block model."""
    x, P, lam, v = _c128(x), _c128(P), _f64(lam), _f64(v)
    F, T, M = x.shape
    N = lam.shape[1]
    llf = np.zeros(F, np.float64)
    ll = _load().ofc_loglik_blocks(F, T, M, N, int(B), _p(x), _p(P), _p(lam), _p(v), _p(llf))
    return float(ll), llf


def mwf_blocks(x, B, P, lam, v):
    """Source images y [N,F,T,M] of the block model (each frame uses its block's h)."""
    x, P, lam, v = _c128(x), _c128(P), _f64(lam), _f64(v)
    F, T, M = x.shape
    N = lam.shape[1]
    y = np.zeros((N, F, T, M), np.complex128)
    st = _load().ofc_mwf_blocks(F, T, M, N, int(B), _p(x), _p(P), _p(lam), _p(v), _p(y))
    if st != OK:
        raise FloatingPointError("ofc_mwf_blocks status %d" % st)
    return y


# ---------------------------------------------------------------- FastMNMF (Sec. V, appendix)
def mnmf_h(tp, va):
    """h [I,J,N] = sum_k t_{ikn} v_{jkn}."""
    tp, va = _f64(tp), _f64(va)
    I, K, N = tp.shape
    J = va.shape[0]
    h = np.zeros((I, J, N), np.float64)
    _load().ofc_mnmf_h(I, J, N, K, _p(tp), _p(va), _p(h))
    return h


def mnmf_loglik(x, P, lam, tp, va):
    """(LL per bin, per-frequency LL [I]) of FastMNMF (eq:FastMNMFcost)."""
    x, P, lam, tp, va = _c128(x), _c128(P), _f64(lam), _f64(tp), _f64(va)
    I, J, M = x.shape
    N = lam.shape[1]
    K = tp.shape[1]
    llf = np.zeros(I, np.float64)
    ll = _load().ofc_mnmf_loglik(I, J, M, N, K, _p(x), _p(P), _p(lam), _p(tp), _p(va), _p(llf))
    return float(ll), llf


def mnmf_iterate(x, P, lam, tp, va, what=15):
    """One FastMNMF iteration (bit 0 IP, 1 Lambda, 2 T, 3 V). Returns copies (P, lam, tp, va)."""
    x = _c128(x)
    P, lam, tp, va = _c128(P).copy(), _f64(lam).copy(), _f64(tp).copy(), _f64(va).copy()
    I, J, M = x.shape
    N = lam.shape[1]
    K = tp.shape[1]
    st = _load().ofc_mnmf_iterate(I, J, M, N, K, _p(x), _p(P), _p(lam), _p(tp), _p(va), int(what))
    if st != OK:
        raise FloatingPointError("ofc_mnmf_iterate status %d" % st)
    return P, lam, tp, va


def mnmf_fit(x, P, lam, tp, va, n_iter, trace=False):
    """n_iter FastMNMF iterations. Returns (P, lam, tp, va, ll_trace or None)."""
    x = _c128(x)
    P, lam, tp, va = _c128(P).copy(), _f64(lam).copy(), _f64(tp).copy(), _f64(va).copy()
    I, J, M = x.shape
    N = lam.shape[1]
    K = tp.shape[1]
    tr = np.zeros(max(n_iter, 1), np.float64) if trace else None
    st = _load().ofc_mnmf_fit(I, J, M, N, K, _p(x), _p(P), _p(lam), _p(tp), _p(va), int(n_iter),
                              _p(tr) if trace else None)
    if st != OK:
        raise FloatingPointError("ofc_mnmf_fit status %d" % st)
    return P, lam, tp, va, (tr[:n_iter] if trace else None)

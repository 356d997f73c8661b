"""Python binding of the FastFCA HIP library (libfastfca.so, include/fastfca.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels. PyTorch supplies device memory and the HIP stream. There is no
CPU code path: if the library or a GPU is missing, construction raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfastfca.so")

OK = 0
E_ARG, E_NOMEM, E_HIP, E_SINGULAR, E_NONFINITE, E_STATE, E_UNSUPPORTED, E_DECREASE = -1, -2, -3, -4, -5, -6, -7, -8
_NAMES = {E_ARG: "E_ARG", E_NOMEM: "E_NOMEM", E_HIP: "E_HIP", E_SINGULAR: "E_SINGULAR",
          E_NONFINITE: "E_NONFINITE", E_STATE: "E_STATE", E_UNSUPPORTED: "E_UNSUPPORTED", E_DECREASE: "E_DECREASE"}

# Every entry point of include/fastfca.h with its ctypes signature.
_vp, _i, _u64, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_double
_pi = ctypes.POINTER(ctypes.c_int)
SIGNATURES = {
    "fastfca_init": (_i, [ctypes.POINTER(_vp), _vp, _i, _i, _i, _i, _vp, _vp, _vp, _u64, _vp]),
    "fastfca_init_batch": (_i, [ctypes.POINTER(_vp), _i, _vp, _u64, _vp]),
    "fastfca_em_step": (_i, [_vp, _i]),
    "fastfca_sync": (_i, [_vp]),
    "fastfca_loglik": (_i, [_vp, _i, ctypes.POINTER(_d), _vp]),
    "fastfca_ll_trace": (_i, [_vp, _i, ctypes.POINTER(_d), _i]),
    "fastfca_mwf": (_i, [_vp, _i, _vp]),
    "fastfca_get_params": (_i, [_vp, _i, _vp, _vp, _vp]),
    "fastfca_set_params": (_i, [_vp, _i, _vp, _vp, _vp]),
    "fastfca_shape": (_i, [_vp, _i, _pi, _pi, _pi, _pi]),
    "fastfca_num_problems": (_i, [_vp]),
    "fastfca_set_config": (_i, [_vp, _i, _i]),
    "fastfca_autotune": (_i, [_vp, _i, ctypes.c_char_p]),
    "fastfca_get_config": (_i, [_vp, _i, _pi, _pi]),
    "fastfca_set_algorithm": (_i, [_vp, _i]),
    "fastfca_set_ll_alarm": (_i, [_vp, _d]),
    "fastfca_set_tail_split": (_i, [_vp, _i]),
    "fastfca_set_schedule": (_i, [_vp, _i]),
    "fastfca_init_blocks": (_i, [ctypes.POINTER(_vp), _vp, _i, _i, _i, _i, _i, _vp, _vp, _vp, _u64, _vp]),
    "fastfca_block_length": (_i, [_vp, _i]),
    "fastfca_mnmf_init": (_i, [ctypes.POINTER(_vp), _vp, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _vp]),
    "fastfca_mnmf_get_params": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "fastfca_mnmf_set_params": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "fastfca_synth_mixture": (_i, [_vp, _i, _i, _i, _i, _i, ctypes.c_float, _u64, _vp]),
    "fastfca_last_error": (ctypes.c_char_p, [_vp]),
    "fastfca_destroy": (None, [_vp]),
    # learned warm start
    "fastfca_net_last_error": (ctypes.c_char_p, []),
    "fastfca_net_pack_weights": (_i, [_vp, _i, _i, _i, _i, _i, _i, _vp, _vp]),
    "fastfca_net_conv_fwd": (_i, [_vp, _i, _i, _i, _vp, _i, _i, _vp, _i, _vp, _i, _vp, _vp, _vp]),
    "fastfca_net_conv_bwd_weight": (_i, [_vp, _i, _i, _vp, _i, _i, _i, _i, _vp, _vp, _vp]),
    "fastfca_net_relu_grad": (_i, [_vp, _vp, _vp, _u64, _vp]),
    "fastfca_net_mean_t": (_i, [_vp, _i, _i, _vp, _vp]),
    "fastfca_net_mean_t_bwd": (_i, [_vp, _i, _i, _vp, _vp]),
    "fastfca_net_linear_fwd": (_i, [_vp, _i, _i, _vp, _vp, _i, _vp, _vp]),
    "fastfca_net_forward_fused": (_i, [_vp, _i, _i, _i, _i, _i, _i, _vp, _vp, _i, _vp, _i, _vp, _vp, _vp, _vp,
                                       _vp]),
    "fastfca_net_linear_bwd": (_i, [_vp, _i, _i, _vp, _i, _vp, _vp, _vp, _vp, _vp]),
    "fastfca_net_pit_loss": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _i, ctypes.c_float, _vp, _vp, _vp, _vp, _vp]),
    "fastfca_net_adamw": (_i, [_vp, _vp, _vp, _vp, _u64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, ctypes.c_float, _i, ctypes.c_float, _vp]),
    "fastfca_ws_features": (_i, [_vp, _i, _i, _i, ctypes.c_float, _vp, _vp, _vp]),
    "fastfca_ws_targets": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _i, _vp, _vp, _vp]),
    "fastfca_ws_apply": (_i, [_vp, _vp, _i, _i, _i, _i, _vp, _vp, _vp]),
    "fastfca_warmstart": (_i, [_vp, _i, _vp, _pi]),
    "fastfca_warmstart_race": (_i, [_vp, _i, _vp, _i, _pi]),
    "fastfca_fit_noalloc": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _vp, _i, _vp, _vp, _vp]),
}


class Problem(ctypes.Structure):
    """fastfca_problem (one mixture of a batch)."""
    _fields_ = [("x", _vp), ("F", _i), ("T", _i), ("M", _i), ("N", _i),
                ("P0", _vp), ("lambda0", _vp), ("v0", _vp)]


class NetDesc(ctypes.Structure):
    """fastfca_net (the trained warm-start network as fastfca_warmstart reads it)."""
    _fields_ = [("M", _i), ("N", _i), ("C", _i), ("L", _i), ("Wb", _vp), ("b", _vp), ("Kp0", _i),
                ("Wv", _vp), ("ldv", _i), ("bv", _vp), ("Wl", _vp), ("bl", _vp)]


class FastFCAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_NAMES.get(code, "?"), code, msg))
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfastfca.so (no GPU call is made). Raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError("libfastfca.so is not built (run __graft_entry__.build()): %s" % path)
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_dev(t, dtype, shape, name):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError("%s must be a contiguous CUDA %s tensor of shape %s, got %s %s %s"
                         % (name, dtype, tuple(shape), t.device, t.dtype, tuple(t.shape)))
    return t


def synth_mixture(F, T, M, N, rank=8, diffuse=0.05, seed=0, stream=None, out=None):
    """Seeded synthetic mixture x [F,T,M] (CUDA complex64) drawn on the GPU."""
    lib = load_library()
    x = out if out is not None else torch.empty((F, T, M), dtype=torch.complex64, device="cuda")
    _check_dev(x, torch.complex64, (F, T, M), "x")
    rc = lib.fastfca_synth_mixture(_ptr(x), F, T, M, N, rank, float(diffuse), int(seed), _stream(stream))
    if rc != OK:
        raise FastFCAError(rc, lib.fastfca_last_error(None).decode())
    return x


def fit_noalloc(x, P, lam, v, n_iter, status, ll_trace=None, stream=None):
    """fastfca_fit_noalloc: n_iter IP+EM iterations on caller buffers with no
    device allocation (x [F,T,M] complex64; P [F,M,M] complex128, lam [F,N,M]
    and v [F,T,N] float32 updated in place; status [F] int32 and ll_trace
    [F,n_iter] float64 (optional) written). Asynchronous on the stream."""
    lib = load_library()
    F, T, M = x.shape
    N = lam.shape[1]
    _check_dev(x, torch.complex64, (F, T, M), "x")
    _check_dev(P, torch.complex128, (F, M, M), "P")
    _check_dev(lam, torch.float32, (F, N, M), "lam")
    _check_dev(v, torch.float32, (F, T, N), "v")
    _check_dev(status, torch.int32, (F,), "status")
    _check_dev(ll_trace, torch.float64, (F, n_iter), "ll_trace")
    rc = lib.fastfca_fit_noalloc(_ptr(x), F, T, M, N, _ptr(P), _ptr(lam), _ptr(v), int(n_iter), _ptr(status),
                                 _ptr(ll_trace), _stream(stream))
    if rc != OK:
        raise FastFCAError(rc, lib.fastfca_last_error(None).decode())


class FastFCA:
    """A library context holding one mixture (or a batch, see from_batch).

    x: CUDA complex64 [F,T,M]; P0: complex128 [F,M,M]; lam0: float32 [F,N,M];
    v0: float32 [F,T,N]. Missing initial values use the library's seeded init.
    """

    def __init__(self, x=None, N=None, P0=None, lam0=None, v0=None, seed=0, stream=None, _ctx=None):
        self._lib = load_library()
        self._stream_obj = stream if stream is not None else torch.cuda.current_stream()
        if _ctx is not None:
            self._ctx = _ctx
            return
        F, T, M = x.shape
        _check_dev(x, torch.complex64, (F, T, M), "x")
        _check_dev(P0, torch.complex128, (F, M, M), "P0")
        _check_dev(lam0, torch.float32, (F, N, M), "lam0")
        _check_dev(v0, torch.float32, (F, T, N), "v0")
        ctx = ctypes.c_void_p()
        rc = self._lib.fastfca_init(ctypes.byref(ctx), _ptr(x), F, T, M, int(N), _ptr(P0), _ptr(lam0),
                                    _ptr(v0), int(seed), _stream(self._stream_obj))
        if rc != OK:
            raise FastFCAError(rc, self._lib.fastfca_last_error(None).decode())
        self._ctx = ctx

    @classmethod
    def from_blocks(cls, x, N, block_len, P0=None, lam0=None, v0=None, seed=0, stream=None):
        """Piecewise stationary model (Sec. VI): blocks of block_len frames of
        x [F,T,M] share h, so v0 (and get_params' v) is [F, T // block_len, N];
        mwf() still returns every frame."""
        lib = load_library()
        stream = stream if stream is not None else torch.cuda.current_stream()
        F, T, M = x.shape
        J = T // block_len
        _check_dev(x, torch.complex64, (F, T, M), "x")
        _check_dev(P0, torch.complex128, (F, M, M), "P0")
        _check_dev(lam0, torch.float32, (F, N, M), "lam0")
        _check_dev(v0, torch.float32, (F, J, N), "v0")
        ctx = ctypes.c_void_p()
        rc = lib.fastfca_init_blocks(ctypes.byref(ctx), _ptr(x), F, T, M, int(N), int(block_len), _ptr(P0),
                                     _ptr(lam0), _ptr(v0), int(seed), _stream(stream))
        if rc != OK:
            raise FastFCAError(rc, lib.fastfca_last_error(None).decode())
        return cls(stream=stream, _ctx=ctx)

    @classmethod
    def mnmf(cls, x, N, K, lam0, t0, v0, P0=None, stream=None):
        """FastMNMF (NMF source powers h = sum_k t_{ikn} v_{jkn}): lam0 [F,N,M],
        t0 [F,K,N], v0 [T,K,N] float32, P0 [F,M,M] complex128 or None."""
        lib = load_library()
        stream = stream if stream is not None else torch.cuda.current_stream()
        F, T, M = x.shape
        _check_dev(x, torch.complex64, (F, T, M), "x")
        _check_dev(P0, torch.complex128, (F, M, M), "P0")
        _check_dev(lam0, torch.float32, (F, N, M), "lam0")
        _check_dev(t0, torch.float32, (F, K, N), "t0")
        _check_dev(v0, torch.float32, (T, K, N), "v0")
        ctx = ctypes.c_void_p()
        rc = lib.fastfca_mnmf_init(ctypes.byref(ctx), _ptr(x), F, T, M, int(N), int(K), _ptr(P0), _ptr(lam0),
                                   _ptr(t0), _ptr(v0), _stream(stream))
        if rc != OK:
            raise FastFCAError(rc, lib.fastfca_last_error(None).decode())
        obj = cls(stream=stream, _ctx=ctx)
        obj._mnmf_K = int(K)
        return obj

    def mnmf_get_params(self):
        """(P [F,M,M], lam [F,N,M], t [F,K,N], v [T,K,N]) of a FastMNMF context."""
        F, T, M, N = self.shape()
        K = self._mnmf_K
        P = torch.empty((F, M, M), dtype=torch.complex128, device="cuda")
        lam = torch.empty((F, N, M), dtype=torch.float32, device="cuda")
        t = torch.empty((F, K, N), dtype=torch.float32, device="cuda")
        v = torch.empty((T, K, N), dtype=torch.float32, device="cuda")
        self._chk(self._lib.fastfca_mnmf_get_params(self._ctx, _ptr(P), _ptr(lam), _ptr(t), _ptr(v)))
        return P, lam, t, v

    def mnmf_set_params(self, P=None, lam=None, t=None, v=None):
        F, T, M, N = self.shape()
        K = self._mnmf_K
        _check_dev(P, torch.complex128, (F, M, M), "P")
        _check_dev(lam, torch.float32, (F, N, M), "lam")
        _check_dev(t, torch.float32, (F, K, N), "t")
        _check_dev(v, torch.float32, (T, K, N), "v")
        self._chk(self._lib.fastfca_mnmf_set_params(self._ctx, _ptr(P), _ptr(lam), _ptr(t), _ptr(v)))

    @classmethod
    def from_batch(cls, problems, seed=0, stream=None):
        """problems: list of dicts with x [F,T,M] and N, optional P0, lam0, v0."""
        lib = load_library()
        stream = stream if stream is not None else torch.cuda.current_stream()
        arr = (Problem * len(problems))()
        for i, p in enumerate(problems):
            x = p["x"]
            F, T, M = x.shape
            N = int(p["N"])
            _check_dev(x, torch.complex64, (F, T, M), "x")
            arr[i] = Problem(x.data_ptr(), F, T, M, N,
                             _check_dev(p.get("P0"), torch.complex128, (F, M, M), "P0").data_ptr() if p.get("P0") is not None else None,
                             _check_dev(p.get("lam0"), torch.float32, (F, N, M), "lam0").data_ptr() if p.get("lam0") is not None else None,
                             _check_dev(p.get("v0"), torch.float32, (F, T, N), "v0").data_ptr() if p.get("v0") is not None else None)
        ctx = ctypes.c_void_p()
        rc = lib.fastfca_init_batch(ctypes.byref(ctx), len(problems), ctypes.cast(arr, ctypes.c_void_p),
                                    int(seed), _stream(stream))
        if rc != OK:
            raise FastFCAError(rc, lib.fastfca_last_error(None).decode())
        return cls(stream=stream, _ctx=ctx)

    # -------------------------------------------------------------- helpers
    def _chk(self, rc):
        if rc < 0:
            raise FastFCAError(rc, self._lib.fastfca_last_error(self._ctx).decode())
        return rc

    @property
    def num_problems(self):
        return self._chk(self._lib.fastfca_num_problems(self._ctx))

    def shape(self, b=0):
        F, T, M, N = (ctypes.c_int() for _ in range(4))
        self._chk(self._lib.fastfca_shape(self._ctx, b, ctypes.byref(F), ctypes.byref(T),
                                          ctypes.byref(M), ctypes.byref(N)))
        return F.value, T.value, M.value, N.value

    # -------------------------------------------------------------- method
    def em_step(self, n_iter=1):
        self._chk(self._lib.fastfca_em_step(self._ctx, int(n_iter)))

    def sync(self):
        self._chk(self._lib.fastfca_sync(self._ctx))

    def loglik(self, b=0, per_f=False):
        ll = ctypes.c_double()
        F = self.shape(b)[0]
        llf = torch.empty(F, dtype=torch.float64, device="cuda") if per_f else None
        self._chk(self._lib.fastfca_loglik(self._ctx, b, ctypes.byref(ll), _ptr(llf)))
        return (ll.value, llf) if per_f else ll.value

    def ll_trace(self, b=0, max_n=1 << 20):
        buf = np.zeros(max_n if max_n < 65536 else 65536, np.float64)
        n = self._chk(self._lib.fastfca_ll_trace(self._ctx, b, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(buf)))
        return buf[:n].copy()

    def block_length(self, b=0):
        """Frames per block of the piecewise stationary model, 0 for the frame model."""
        return self._chk(self._lib.fastfca_block_length(self._ctx, b))

    def mwf(self, b=0, out=None):
        F, T, M, N = self.shape(b)
        T *= max(1, self.block_length(b))
        y = out if out is not None else torch.empty((N, F, T, M), dtype=torch.complex64, device="cuda")
        _check_dev(y, torch.complex64, (N, F, T, M), "y")
        self._chk(self._lib.fastfca_mwf(self._ctx, b, _ptr(y)))
        return y

    def get_params(self, b=0):
        F, T, M, N = self.shape(b)
        P = torch.empty((F, M, M), dtype=torch.complex128, device="cuda")
        lam = torch.empty((F, N, M), dtype=torch.float32, device="cuda")
        v = torch.empty((F, T, N), dtype=torch.float32, device="cuda")
        self._chk(self._lib.fastfca_get_params(self._ctx, b, _ptr(P), _ptr(lam), _ptr(v)))
        return P, lam, v

    def set_params(self, P=None, lam=None, v=None, b=0):
        """Overwrite (P, lambda, v) of mixture b from CUDA tensors (None keeps)."""
        F, T, M, N = self.shape(b)
        _check_dev(P, torch.complex128, (F, M, M), "P")
        _check_dev(lam, torch.float32, (F, N, M), "lam")
        _check_dev(v, torch.float32, (F, T, N), "v")
        self._chk(self._lib.fastfca_set_params(self._ctx, b, _ptr(P), _ptr(lam), _ptr(v)))

    def warmstart(self, net=None, b=0, count=False):
        """fastfca_warmstart: replace mixture b's start by the network's warm
        start (net: a warmstart.ConvNet) or, with net=None, by the
        whitening-only start; the library keeps the new start only in the
        frequencies where its log-likelihood is not below the old one's.
        count=True synchronizes and returns how many frequencies kept it."""
        desc = net.descriptor() if net is not None else None
        n = ctypes.c_int(0)
        self._chk(self._lib.fastfca_warmstart(self._ctx, b, ctypes.byref(desc) if desc is not None else None,
                                              ctypes.byref(n) if count else None))
        return n.value if count else None

    def warmstart_race(self, net=None, race_iters=100, b=0, count=False):
        """fastfca_warmstart_race: run the current start and the new one (the
        network's, or the whitening-only start with net=None) race_iters
        iterations side by side and keep per frequency the better; count=True
        synchronizes and returns how many frequencies kept the new start."""
        desc = net.descriptor() if net is not None else None
        n = ctypes.c_int(0)
        self._chk(self._lib.fastfca_warmstart_race(self._ctx, b, ctypes.byref(desc) if desc is not None else None,
                                                   int(race_iters), ctypes.byref(n) if count else None))
        return n.value if count else None

    def set_tail_split(self, blocks=-1):
        """fastfca_set_tail_split: -1 automatic, 0 off, k > 0 blocks."""
        self._chk(self._lib.fastfca_set_tail_split(self._ctx, int(blocks)))

    def set_ll_alarm(self, tol):
        """fastfca_set_ll_alarm (float('inf') disables the alarm)."""
        self._chk(self._lib.fastfca_set_ll_alarm(self._ctx, float(tol)))

    def set_config(self, threads=0, bins_per_thread=0):
        self._chk(self._lib.fastfca_set_config(self._ctx, int(threads), int(bins_per_thread)))

    def set_algorithm(self, algo):
        """'em' (Algorithm 1, default) or 'mm' (Algorithm 2)."""
        code = {"em": 0, "mm": 1}[algo] if isinstance(algo, str) else int(algo)
        self._chk(self._lib.fastfca_set_algorithm(self._ctx, code))

    def set_schedule(self, schedule):
        """Batches: 'classes' (one launch per (M, N, T-bucket) class) or 'persistent'."""
        code = {"classes": 0, "persistent": 1}[schedule] if isinstance(schedule, str) else int(schedule)
        self._chk(self._lib.fastfca_set_schedule(self._ctx, code))

    def get_config(self, b=0):
        th, bpt = ctypes.c_int(), ctypes.c_int()
        self._chk(self._lib.fastfca_get_config(self._ctx, b, ctypes.byref(th), ctypes.byref(bpt)))
        return th.value, bpt.value

    def autotune(self, n_iter=10, cache_path=None):
        self._chk(self._lib.fastfca_autotune(self._ctx, int(n_iter),
                                             cache_path.encode() if cache_path else None))

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.fastfca_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

"""Seeded synthetic mixtures and initial parameters.

This module holds no FastFCA arithmetic: it only draws inputs. Both the GPU
library's tests/benchmark and the FP64 oracle consume what it produces.

The paper evaluates on real-room recordings (Sec. VII) that are not
available; these draws stand in for them with the paper's STFT shape
(F = 513 bins from 1024-point frames, Table 1) and the FCA generative model
of Sec. III-A: each source image c_n(t,f) ~ N_c(0, v_n(t,f) R_n(f)),
x = sum_n c_n (eq:summodel).

Recipe (all draws from numpy's PCG64 seeded by SeedSequence):
  * v_n = W_n H_n, a rank-K non-negative factorization with Gamma(1,1) (=Exp(1))
    factors W_n [F,K], H_n [K,T]   (a low-rank, speech-like power spectrogram)
  * R_n(f) = a a^H + delta I with a_m = exp(i theta), theta ~ U[0, 2 pi)
    drawn independently per (n, f, m)  (unit-modulus random-phase steering)
  * c_n = sqrt(v_n) chol(R_n) z with z ~ N_c(0, I) (real, imag ~ N(0, 1/2))
  * initial parameters: P = I; lam_nm = 0.5 + u; v_tn = (|x_t|^2/(M N) + d_f)(0.5 + u')
    with d_f = 1e-6 mean_t |x_t|^2/(M N), u, u' ~ U[0, 1)
"""
from __future__ import annotations

import numpy as np

# Shapes of the evaluated workloads. Each entry: name -> dict of generator args.
CONFIGS = {
    # small case: M=2 mics, N=3 sources, F=257, T=200, rank 4, diffuse 0.1
    "c0": dict(F=257, T=200, M=2, N=3, rank=4, diffuse=0.1, n_iter=50, config_id=0),
    # headline case: M=2, N=3, F=513, T=1000, rank 8, diffuse 0.05
    "c1": dict(F=513, T=1000, M=2, N=3, rank=8, diffuse=0.05, n_iter=100, config_id=1),
    # large array: M=8, N=10, F=1025, T=4000, rank 8, diffuse 0.05
    "c3": dict(F=1025, T=4000, M=8, N=10, rank=8, diffuse=0.05, n_iter=100, config_id=3),
}


def _rng(*key):
    return np.random.default_rng(np.random.SeedSequence([int(k) for k in key]))


def mixture(F, T, M, N, rank=8, diffuse=0.05, config_id=0, mixture_id=0, return_truth=False,
            dtype=np.complex64):
    """Draw one mixture x [F,T,M] (complex64 by default).

    With return_truth, also return the true (v [F,T,N], R [F,N,M,M], c [N,F,T,M])."""
    rng = _rng(config_id, mixture_id, 0)
    Wf = rng.gamma(1.0, 1.0, size=(N, F, rank))
    Ht = rng.gamma(1.0, 1.0, size=(N, rank, T))
    v = np.einsum("nfk,nkt->nft", Wf, Ht)                       # [N,F,T]
    theta = rng.uniform(0.0, 2.0 * np.pi, size=(N, F, M))
    a = np.exp(1j * theta)                                      # [N,F,M]
    R = a[..., :, None] * np.conj(a[..., None, :]) + diffuse * np.eye(M)[None, None]
    C = np.linalg.cholesky(R)                                   # [N,F,M,M]
    x = np.zeros((F, T, M), np.complex128)
    cs = [] if return_truth else None
    for n in range(N):
        z = (rng.standard_normal((F, T, M)) + 1j * rng.standard_normal((F, T, M))) * np.sqrt(0.5)
        c = np.sqrt(v[n])[..., None] * np.einsum("fij,ftj->fti", C[n], z)
        x += c
        if return_truth:
            cs.append(c.astype(dtype))
    x = x.astype(dtype)
    if return_truth:
        return x, np.ascontiguousarray(v.transpose(1, 2, 0)), R.transpose(1, 0, 2, 3), np.stack(cs)
    return x


def init_params(x, N, config_id=0, mixture_id=0):
    """Initial (P [F,M,M] complex128, lam [F,N,M] float32, v [F,T,N] float32)."""
    F, T, M = x.shape
    rng = _rng(config_id, mixture_id, 1)
    p = (np.abs(x.astype(np.complex128)) ** 2).sum(axis=2) / (M * N)   # [F,T]
    d = 1e-6 * p.mean(axis=1, keepdims=True)
    lam = (0.5 + rng.random((F, N, M))).astype(np.float32)
    v = ((p + d)[..., None] * (0.5 + rng.random((F, T, N)))).astype(np.float32)
    P = np.broadcast_to(np.eye(M, dtype=np.complex128), (F, M, M)).copy()
    return P, lam, v


def init_params_blocks(x, N, B, config_id=0, mixture_id=0):
    """Initial state of the piecewise stationary model (blocks of B frames):
    as init_params with the frame power replaced by the block's mean power;
    v is [F, T//B, N]."""
    F, T, M = x.shape
    J = T // B
    rng = _rng(config_id, mixture_id, 4)
    p = (np.abs(x[:, :J * B].astype(np.complex128)) ** 2).sum(axis=2).reshape(F, J, B).mean(axis=2) / (M * N)
    d = 1e-6 * p.mean(axis=1, keepdims=True)
    lam = (0.5 + rng.random((F, N, M))).astype(np.float32)
    v = ((p + d)[..., None] * (0.5 + rng.random((F, J, N)))).astype(np.float32)
    P = np.broadcast_to(np.eye(M, dtype=np.complex128), (F, M, M)).copy()
    return P, lam, v


def init_params_mnmf(x, N, K, config_id=0, mixture_id=0):
    """Initial FastMNMF state: P = I, lam [F,N,M] = 0.5 + u, spectral patterns
    tp [F,K,N] = a_f (0.5 + u'), activations va [T,K,N] = b_t (0.5 + u''),
    with a_f b_t the rank-one fit of the mixture power |x_ft|^2 / (M N K)."""
    F, T, M = x.shape
    rng = _rng(config_id, mixture_id, 5)
    p = (np.abs(x.astype(np.complex128)) ** 2).sum(axis=2)              # [F,T]
    a = p.mean(axis=1) / (M * N * K) + 1e-12
    b = p.mean(axis=0) / p.mean() + 1e-6
    lam = (0.5 + rng.random((F, N, M))).astype(np.float32)
    tp = (a[:, None, None] * (0.5 + rng.random((F, K, N)))).astype(np.float32)
    va = (b[:, None, None] * (0.5 + rng.random((T, K, N)))).astype(np.float32)
    P = np.broadcast_to(np.eye(M, dtype=np.complex128), (F, M, M)).copy()
    return P, lam, tp, va


def batch_specs(B=256, F=513, config_id=2, seed=0):
    """Shapes of the mixed batch: T ~ U{200..2000}, M in {2,3,4}, N in {M+1, M+2}."""
    rng = _rng(config_id, 10**6 + seed, 2)
    specs = []
    for b in range(B):
        M = int(rng.integers(2, 5))
        N = int(M + rng.integers(1, 3))
        T = int(rng.integers(200, 2001))
        specs.append(dict(F=F, T=T, M=M, N=N, rank=8, diffuse=0.05, config_id=config_id, mixture_id=b))
    return specs


def random_params(F, T, M, N, seed=0, cond=3.0):
    """Random well-conditioned state (P, lam, v) for identity tests on tiny inputs."""
    rng = _rng(99, seed, 3)
    P = (rng.standard_normal((F, M, M)) + 1j * rng.standard_normal((F, M, M))) / np.sqrt(2 * M)
    P += cond * np.eye(M)[None] / np.sqrt(M)
    lam = 0.2 + rng.random((F, N, M))
    v = 0.1 + rng.gamma(1.0, 1.0, size=(F, T, N))
    return P, lam, v

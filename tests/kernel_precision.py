"""Numpy emulation of the precision of the GPU kernels' Algorithm 1 iteration
(test infrastructure; shares nothing with the HIP sources).

It runs IP+EM (Algorithm 1, Sec. IV-E) with the arithmetic of each stage in a
chosen precision, so that a CPU test can attribute a difference between the
GPU and the FP64 oracle to one stage:

  q_mode  'f64'    every Q_m term and sum in double precision
          'tree32' each lane sums its bins' single precision terms
                   x x^H / sigma^2 (bins t = lane + k * threads), then the
                   lane partials are added in a balanced single precision tree
          'tree64' the same lane partials, added in a double precision tree
  f32_rest        U = |P^H x|^2 with P rounded to single precision, and the
                   source updates (G_n, Phi_n, L, H) in single precision

The IP update (eq:ip1, eq:ip2) is always double precision, as in the kernels.
"""
from __future__ import annotations

import numpy as np


def _tree(a, dtype):
    """Balanced pairwise sum along axis 0, every partial rounded to dtype."""
    a = a.astype(dtype)
    while a.shape[0] > 1:
        if a.shape[0] % 2:
            a = np.concatenate([a, np.zeros_like(a[:1])])
        a = (a[0::2] + a[1::2]).astype(dtype)
    return a[0]


def weighted_covs(xf, lam, v, q_mode, threads, bpt):
    """The M weighted covariances Q_m (eq:wsampcov) of one frequency."""
    T, M = xf.shape
    if q_mode == "f64":
        w = 1.0 / (v.astype(np.float64) @ lam.astype(np.float64))
        xx = xf.astype(np.complex128)[:, :, None] * np.conj(xf.astype(np.complex128))[:, None, :]
        return np.stack([(w[:, m, None, None] * xx).sum(axis=0) / T for m in range(M)])
    assert threads * bpt >= T
    w = (np.float32(1.0) / (v.astype(np.float32) @ lam.astype(np.float32))).astype(np.float32)
    xx = (xf[:, :, None] * np.conj(xf)[:, None, :]).astype(np.complex64)
    Q = np.zeros((M, M, M), np.complex128)
    for m in range(M):
        terms = np.zeros((bpt * threads, M, M), np.complex64)
        terms[:T] = (w[:, m, None, None] * xx).astype(np.complex64)
        terms = terms.reshape(bpt, threads, M, M)        # bin t = lane + k * threads
        lane = np.zeros((threads, M, M), np.complex64)
        for k in range(bpt):
            lane = (lane + terms[k]).astype(np.complex64)
        tot = _tree(lane, np.complex64 if q_mode == "tree32" else np.complex128)
        Q[m] = tot.astype(np.complex128) / T
    return Q


def fit(x, P, lam, v, n_iter, q_mode="f64", f32_rest=False, threads=128, bpt=4):
    """n_iter IP+EM iterations on every frequency; returns (P, lam, v) in FP64."""
    F, T, M = x.shape
    N = lam.shape[1]
    P = np.array(P, np.complex128)
    lam = np.array(lam, np.float64)
    v = np.array(v, np.float64)
    rt = np.float32 if f32_rest else np.float64
    for _ in range(n_iter):
        for f in range(F):
            Q = weighted_covs(x[f], lam[f], v[f], q_mode, threads, bpt)
            Pf = P[f]
            for m in range(M):                               # eq:ip1, eq:ip2
                w = np.linalg.solve(Pf.conj().T @ Q[m], np.eye(M)[m])
                Pf[:, m] = w / np.sqrt(np.real(w.conj() @ Q[m] @ w))
            if f32_rest:
                U = np.abs(x[f].astype(np.complex64) @ np.conj(Pf.astype(np.complex64))) ** 2
            else:
                U = np.abs(x[f].astype(np.complex128) @ np.conj(Pf)) ** 2
            U = U.astype(rt)
            L, H = lam[f].astype(rt), v[f].astype(rt)
            for n in range(N):                               # Algorithm 1, sources in order
                a = H[:, n, None] * L[None, n]
                g = a / (H @ L)
                phi = g * g * U + (1 - g) * a
                L[n] = (_tree(phi / H[:, n, None], rt) / T).astype(rt)
                H[:, n] = (phi / L[None, n]).mean(axis=1)
            lam[f], v[f] = L, H
    return P, lam, v

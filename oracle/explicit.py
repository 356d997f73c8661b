"""Explicit full-matrix forms of the FCA model -- TEST INFRASTRUCTURE.

These are the definitions of Sec. III written out with M x M matrices and
numpy linear algebra, with no use of the joint-diagonalization shortcut. They
pin the oracle's diagonal-domain formulas on tiny inputs:

* R_n = P^{-H} diag(lam_n) P^{-1}              (eq:parametrizationFastFCA)
* X_t = sum_n v_tn R_n                           (eq:obsden)
* ln N_c(x | 0, X) = -M ln pi - ln det X - x^H X^{-1} x   (density of Sec. III-A)
* F_tn = v_tn R_n X_t^{-1},  c_hat = F_tn x_t    (eq:mwf2)
"""
from __future__ import annotations

import numpy as np


def scm(P, lam):
    """R [N,M,M] for one frequency: R_n = P^{-H} diag(lam_n) P^{-1}."""
    Pinv = np.linalg.inv(P)
    return np.stack([Pinv.conj().T @ np.diag(l.astype(np.complex128)) @ Pinv for l in lam])


def loglik_freq(x, P, lam, v):
    """Mean over t of ln N_c(x_t | 0, X_t) with X_t = sum_n v_tn R_n."""
    R = scm(P, lam)
    T, M = x.shape
    acc = 0.0
    for t in range(T):
        X = np.tensordot(v[t].astype(np.complex128), R, axes=(0, 0))
        sign, logdet = np.linalg.slogdet(X)
        quad = np.real(np.conj(x[t]) @ np.linalg.solve(X, x[t]))
        acc += -M * np.log(np.pi) - logdet - quad
    return acc / T


def mwf_freq(x, P, lam, v):
    """c_hat [N,T,M] for one frequency by the general MWF of eq:mwf2."""
    R = scm(P, lam)
    T, M = x.shape
    N = lam.shape[0]
    y = np.zeros((N, T, M), np.complex128)
    for t in range(T):
        X = np.tensordot(v[t].astype(np.complex128), R, axes=(0, 0))
        Xinv = np.linalg.inv(X)
        for n in range(N):
            y[n, t] = v[t, n] * R[n] @ Xinv @ x[t]
    return y

"""Pins of the oracle's piecewise stationary extension (Sec. VI): blocks of B
frames share h, and Algorithms 1 and 2 run on the block covariances.

Each identity is written here independently of the oracle's C code: full
matrix Gaussian densities, the decomposition eq:ldpytha into an AJD term and
an Itakura-Saito term, the B = 1 reduction to the frame model, einsum forms,
and monotonicity of the iterations.
"""
import numpy as np
import pytest

import oracle
from oracle import explicit
from paper_2101_08563_amd import synth


def _cn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def _state(F, J, M, N, seed):
    P, lam, _ = synth.random_params(F, 2, M, N, seed=seed)
    rng = np.random.default_rng(seed + 1000)
    v = 0.1 + rng.gamma(1.0, 1.0, size=(F, J, N))
    return P, lam, v


def test_block_covariance_definition():
    rng = np.random.default_rng(0)
    x = _cn(rng, 12, 3)
    Xh = oracle.block_cov(x, 4)
    ref = np.einsum("jbr,jbc->jrc", x.reshape(3, 4, 3), x.reshape(3, 4, 3).conj()) / 4
    np.testing.assert_allclose(Xh, ref, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("M,N,B", [(2, 3, 4), (3, 4, 5), (4, 6, 8), (2, 2, 2)])
def test_block_loglik_equals_full_matrix_density(M, N, B):
    """Block LL per frame == mean over frames of ln N_c(x_t | 0, sum_n h_{j(t)n} R_n)
    with full matrices (the density behind eq:negllpws)."""
    rng = np.random.default_rng(10 * M + N + B)
    J = 5
    x = _cn(rng, 2, J * B, M) * 1.5
    P, lam, v = _state(2, J, M, N, seed=M + N)
    ll, llf = oracle.loglik_blocks(x, B, P, lam, v)
    ref = np.array([explicit.loglik_freq(x[f], P[f], lam[f], np.repeat(v[f], B, axis=0)) for f in range(2)])
    np.testing.assert_allclose(llf, ref, rtol=1e-12, atol=1e-12)
    assert abs(ll - ref.mean()) < 1e-12


@pytest.mark.parametrize("M,N,B", [(2, 3, 4), (3, 5, 6), (4, 4, 9)])
def test_ldpytha_decomposition(M, N, B):
    """eq:ldpytha: eq:negllpws = sum_j D_LD(P^H X_j P | ddiag(P^H X_j P))
    + sum_{m,j} D_IS(<|y_mj|^2> | sigma^2_mj), up to the constant
    sum_j ln det X_j + M J that the paper's equality leaves out (B >= M so every
    block covariance is positive definite)."""
    rng = np.random.default_rng(M * N * B)
    J = 6
    x = _cn(rng, J * B, M) * 2.0
    P, lam, v = _state(1, J, M, N, seed=3 * M)
    P, lam, v = P[0], lam[0], v[0]
    Xh = oracle.block_cov(x, B)
    nll = -J * oracle.loglik_blocks_freq(Xh, P, lam, v) - J * M * np.log(np.pi)
    s2 = v @ lam                                            # [J, M]
    ajd = 0.0
    dis = 0.0
    lndet = 0.0
    for j in range(J):
        A = P.conj().T @ Xh[j] @ P
        d = np.real(np.diag(A))
        ajd += np.sum(np.log(d)) - np.linalg.slogdet(A)[1]  # D_LD(A | ddiag A)
        r = d / s2[j]
        dis += np.sum(r - np.log(r) - 1.0)
        lndet += np.linalg.slogdet(Xh[j])[1]
    assert abs(nll - (ajd + dis + lndet + M * J)) < 1e-9 * max(1.0, abs(nll))


def test_block_power_and_weighted_cov_by_einsum():
    rng = np.random.default_rng(4)
    M, N, B, J = 3, 4, 3, 7
    x = _cn(rng, J * B, M)
    P, lam, v = _state(1, J, M, N, seed=8)
    P, lam, v = P[0], lam[0], v[0]
    Xh = oracle.block_cov(x, B)
    U = oracle.block_power(P, Xh)
    np.testing.assert_allclose(U, np.real(np.einsum("rm,jrc,cm->mj", P.conj(), Xh, P)), rtol=1e-13)
    s2 = v @ lam
    Q = oracle.weighted_cov_blocks(Xh, lam, v)
    np.testing.assert_allclose(Q, np.einsum("jrc,jm->mrc", Xh, 1.0 / s2) / J, rtol=1e-13)


@pytest.mark.parametrize("algo", [0, 1])
def test_block_size_one_is_the_frame_model(algo):
    """eq:negllpws reduces to the frame model's cost when B = 1, and so do the
    iterations."""
    x = synth.mixture(F=4, T=60, M=2, N=3, rank=3, config_id=70)
    P0, lam0, v0 = synth.init_params(x, 3, config_id=70)
    a = oracle.fit(x, P0, lam0, v0, 6, algo=algo, trace=True)
    b = oracle.fit_blocks(x, 1, P0, lam0, v0, 6, algo=algo, trace=True)
    for u, w in zip(a, b):
        np.testing.assert_allclose(w, u, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("M,N,B,algo", [(2, 3, 4, 0), (3, 4, 5, 0), (2, 3, 8, 1), (4, 5, 4, 0)])
def test_block_iterations_are_monotone(M, N, B, algo):
    x = synth.mixture(F=3, T=40 * B, M=M, N=N, rank=4, config_id=71, mixture_id=B)
    P0, lam0, v0 = synth.init_params_blocks(x, N, B, config_id=71, mixture_id=B)
    _, _, _, tr = oracle.fit_blocks(x, B, P0, lam0, v0, 40, algo=algo, trace=True)
    ll0, _ = oracle.loglik_blocks(x, B, P0, lam0, v0)
    tr = np.concatenate([[ll0], tr])
    assert np.diff(tr).min() > -1e-10 * np.abs(tr).max(), np.diff(tr).min()
    assert tr[-1] > tr[0] + 0.1


def test_block_mwf_is_frame_mwf_with_block_h_and_sums_to_mixture():
    rng = np.random.default_rng(9)
    M, N, B, J = 3, 4, 5, 4
    x = _cn(rng, 2, J * B, M)
    P, lam, v = _state(2, J, M, N, seed=11)
    y = oracle.mwf_blocks(x, B, P, lam, v)
    ref = np.stack([explicit.mwf_freq(x[f], P[f], lam[f], np.repeat(v[f], B, axis=0)) for f in range(2)], axis=1)
    np.testing.assert_allclose(y, ref, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(y.sum(axis=0), x, rtol=1e-10, atol=1e-12)

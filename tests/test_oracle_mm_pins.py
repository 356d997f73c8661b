"""Pins of the oracle's multiplicative (MM) rules by brute-force minimization
of their auxiliary function.

Algorithm 2 updates L, then H, by the MM algorithm for IS-NMF (Sec. IV-E;
the MM principle of Sec. III-C): each rule must equal the minimizer of an
auxiliary function that majorizes the cost
    D(theta) = sum_{m,t} [ U_mt / s_mt + ln s_mt ],   s = A theta,
where A holds the (non-negative) coefficient of every updated parameter in
sigma^2 (eq:sigmadef). The auxiliary function used here is built from the two
inequalities that majorize an IS cost: Jensen's inequality for the convex
1/s, with the weights psi_c = a_c theta'_c / s' of the current iterate, and
the tangent line of the concave ln s at s':
    D+(theta; theta') = sum_{m,t} [ U sum_c psi_c^2 / (a_c theta_c)
                                    + ln s' + (s - s') / s' ].
The tests first check that D+ really majorizes D and touches it at theta'
(so a wrong auxiliary function in this file would fail), then minimize D+
numerically, coordinate by coordinate over log theta, and compare with the
oracle's closed-form rules: Algorithm 2's L rule with H fixed, its H rule
with the NEW L, and FastMNMF's Lambda, T and V rules (Sec. V, its appendix).
Mutated rules (exponent 1 instead of 1/2, H from the old L) are shown to
fail the same checks, in Python and as a mutated build of the oracle's C
source.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest
from scipy import optimize

import oracle
from paper_2101_08563_amd import synth


# ----------------------------------------------------------------- the generic pin
def is_cost(theta, A, U):
    s = A @ theta
    return float(np.sum(U / s + np.log(s)))


def aux_cost(theta, theta0, A, U):
    """D+(theta; theta0): Jensen on 1/s, tangent line on ln s (see the module text)."""
    s0 = A @ theta0
    psi = A * theta0[None, :] / s0[:, None]          # [rows, params], rows sum to 1
    jensen = np.sum(U[:, None] * psi ** 2 / (A * theta[None, :] + (A == 0)) * (A != 0))
    s = A @ theta
    return float(jensen + np.sum(np.log(s0) + (s - s0) / s0))


def brute_force_minimizer(theta0, A, U, sweeps=2):
    """Coordinate-wise minimization of D+ over log theta: a bounded 1-D search
    brackets each coordinate's minimum, then a root of the central-difference
    derivative of D+ pins it down (a function value search alone stalls near
    1e-7 in the argument, where D+ is flat). A second sweep must not move any
    coordinate, so the function is minimized jointly."""
    th = theta0.copy()
    h = 1e-5
    for sw in range(sweeps):
        prev = th.copy()
        for c in range(th.size):
            def f(z, c=c):
                t = th.copy()
                t[c] = np.exp(z)
                return aux_cost(t, theta0, A, U)

            def g(z):
                return (f(z + h) - f(z - h)) / (2 * h)
            z0 = np.log(th[c])
            r = optimize.minimize_scalar(f, bounds=(z0 - 12.0, z0 + 12.0), method="bounded",
                                         options=dict(xatol=1e-10))
            a = b = r.x
            step = 1e-4
            while g(a) > 0:
                a -= step
                step *= 2
            step = 1e-4
            while g(b) < 0:
                b += step
                step *= 2
            th[c] = np.exp(optimize.brentq(g, a, b, xtol=1e-14, rtol=1e-14) if a < b else a)
        if sw > 0:
            np.testing.assert_allclose(th, prev, rtol=1e-8)
    return th


def check_majorizes(theta0, A, U, rng):
    """D+ >= D everywhere (random points) and D+ = D at theta0."""
    assert abs(aux_cost(theta0, theta0, A, U) - is_cost(theta0, A, U)) <= 1e-11 * abs(is_cost(theta0, A, U))
    for _ in range(20):
        th = theta0 * np.exp(rng.normal(scale=1.0, size=theta0.shape))
        assert aux_cost(th, theta0, A, U) >= is_cost(th, A, U) - 1e-10 * abs(is_cost(th, A, U))


# ----------------------------------------------------------------- Algorithm 2 (one frequency)
def coef_L(H, M):
    """s_{mt} = sum_n L_{mn} H_{nt}: rows (m, t), parameters (m, n) with value lam[n][m]."""
    N, T = H.shape
    A = np.zeros((M * T, N * M))
    for m in range(M):
        for t in range(T):
            for n in range(N):
                A[m * T + t, n * M + m] = H[n, t]
    return A


def coef_H(L, T):
    """Rows (m, t), parameters (t, n) with value v[t][n] (coefficient L_{mn})."""
    M, N = L.shape
    A = np.zeros((M * T, T * N))
    for m in range(M):
        for t in range(T):
            for n in range(N):
                A[m * T + t, t * N + n] = L[m, n]
    return A


def _small_case(M=2, N=3, T=7, seed=0):
    rng = np.random.default_rng(seed)
    lam = 0.3 + rng.random((N, M)) * 2.0            # [N][M]
    v = 0.2 + rng.exponential(size=(T, N))          # [T][N]
    U = rng.exponential(size=(M, T)) * 3.0          # [M][T]
    return U, lam, v, rng


def reference_mm(U, lam, v):
    """(L, H) of one MM step, each the brute-force minimizer of its own D+."""
    M, T = U.shape
    N = lam.shape[0]
    Uf = U.reshape(-1)
    A_L = coef_L(v.T, M)
    lam1 = brute_force_minimizer(lam.reshape(-1), A_L, Uf).reshape(N, M)
    A_H = coef_H(lam1.T, T)                         # H's auxiliary function at the NEW L
    v1 = brute_force_minimizer(v.reshape(-1), A_H, Uf).reshape(T, N)
    return lam1, v1


@pytest.mark.parametrize("M,N,T,seed", [(2, 3, 7, 0), (3, 2, 6, 1), (4, 5, 5, 2)])
def test_auxiliary_functions_majorize_the_is_cost(M, N, T, seed):
    U, lam, v, rng = _small_case(M, N, T, seed)
    check_majorizes(lam.reshape(-1), coef_L(v.T, M), U.reshape(-1), rng)
    check_majorizes(v.reshape(-1), coef_H(lam.T, T), U.reshape(-1), rng)


@pytest.mark.parametrize("M,N,T,seed", [(2, 3, 7, 0), (3, 2, 6, 1), (4, 5, 5, 2)])
def test_mm_update_is_the_auxiliary_minimizer(M, N, T, seed):
    """Algorithm 2: L <- argmin D+_L(.; L, H); then H <- argmin D+_H(.; L_new, H)."""
    U, lam, v, _ = _small_case(M, N, T, seed)
    lam_ref, v_ref = reference_mm(U, lam, v)
    lam1, v1 = oracle.mm_update(U, lam, v)
    np.testing.assert_allclose(lam1, lam_ref, rtol=1e-7)
    np.testing.assert_allclose(v1, v_ref, rtol=1e-7)


def _mm_exponent_one(U, lam, v):
    """Mutant: the multiplicative rule without its square root."""
    s = v @ lam
    lam = lam * (((U.T / s ** 2).T @ v) / ((1 / s).T @ v)).T
    s = v @ lam
    v = v * ((U.T / s ** 2) @ lam.T) / ((1 / s) @ lam.T)
    return lam, v


def _mm_old_L(U, lam, v):
    """Mutant: H updated from the OLD L (both rules from the same sigma^2)."""
    s = v @ lam
    a, b = U.T / s ** 2, 1 / s
    lam_new = lam * np.sqrt(((a.T @ v) / (b.T @ v)).T)
    v_new = v * np.sqrt((a @ lam.T) / (b @ lam.T))
    return lam_new, v_new


def _mm_correct(U, lam, v):
    """The rules written from the minimizer in closed form (for the mutants' baseline)."""
    s = v @ lam
    lam = lam * np.sqrt((((U.T / s ** 2).T @ v) / ((1 / s).T @ v)).T)
    s = v @ lam
    v = v * np.sqrt(((U.T / s ** 2) @ lam.T) / ((1 / s) @ lam.T))
    return lam, v


@pytest.mark.parametrize("rule,should_pass", [(_mm_correct, True), (_mm_exponent_one, False), (_mm_old_L, False)])
def test_pin_rejects_mutated_rules(rule, should_pass):
    U, lam, v, _ = _small_case(3, 4, 6, 3)
    lam_ref, v_ref = reference_mm(U, lam, v)
    lam1, v1 = rule(U, lam, v)
    ok = np.allclose(lam1, lam_ref, rtol=1e-7, atol=0) and np.allclose(v1, v_ref, rtol=1e-7, atol=0)
    assert ok == should_pass


def _mutant_oracle(tmp_path, old, new):
    """The oracle's C source with one textual change, built with gcc."""
    src_path = os.path.join(os.path.dirname(oracle.__file__), "fastfca_oracle.c")
    with open(src_path) as fh:
        src = fh.read()
    assert src.count(old) >= 1
    mut = tmp_path / "oracle_mutant.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", str(so), str(mut), "-lm"])
    lib = ctypes.CDLL(str(so))
    vp, ci = ctypes.c_void_p, ctypes.c_int
    lib.ofc_mm_update.argtypes = [ci, ci, ci, vp, vp, vp, vp]
    return lib


def test_mutated_oracle_build_fails_the_pin(tmp_path):
    """The oracle with the square root of Algorithm 2's rules dropped: the
    unmutated build passes the pin (above), this one does not."""
    lib = _mutant_oracle(tmp_path, "sqrt(num / den)", "(num / den)")
    U, lam, v, _ = _small_case(2, 3, 7, 0)
    lam1, v1 = lam.copy(), v.copy()
    scratch = np.zeros(2 * U.size)
    M, T = U.shape
    lib.ofc_mm_update(T, M, lam.shape[0], U.ctypes.data, lam1.ctypes.data, v1.ctypes.data, scratch.ctypes.data)
    lam_ref, v_ref = reference_mm(U, lam, v)
    assert not np.allclose(lam1, lam_ref, rtol=1e-7)
    # and the unmutated rule, through the same call convention, does match
    lam2, v2 = oracle.mm_update(U, lam, v)
    np.testing.assert_allclose(lam2, lam_ref, rtol=1e-7)


# ----------------------------------------------------------------- FastMNMF (Sec. V)
def _mnmf_case(F=2, T=5, M=2, N=2, K=2, cid=84):
    x = synth.mixture(F=F, T=T, M=M, N=N, rank=2, diffuse=0.1, config_id=cid)
    P, lam, tp, va = synth.init_params_mnmf(x, N, K, config_id=cid)
    P = P + 0.2 * np.random.default_rng(cid).standard_normal(P.shape)
    U = np.stack([oracle.decorrelated_power(P[i], x[i]) for i in range(F)])   # [F][M][T]
    return x, P, lam.astype(np.float64), tp.astype(np.float64), va.astype(np.float64), U


def _rows_mnmf(U):
    """Rows (i, m, t) of the cost, flattened in that order."""
    return U.reshape(-1)


def coef_mnmf(which, lam, tp, va, M):
    """Coefficients of sigma^2_{imt} = sum_n lam[i][n][m] sum_k tp[i][k][n] va[t][k][n] in the
    parameters of one factor (which = 'lam' | 'tp' | 'va'), rows (i, m, t)."""
    F, N, _ = lam.shape
    K = tp.shape[1]
    T = va.shape[0]
    shape = {"lam": lam.shape, "tp": tp.shape, "va": va.shape}[which]
    A = np.zeros((F * M * T, int(np.prod(shape))))
    for i in range(F):
        for m in range(M):
            for t in range(T):
                r = (i * M + m) * T + t
                for n in range(N):
                    for k in range(K):
                        c = lam[i, n, m] * tp[i, k, n] * va[t, k, n]
                        if which == "lam":
                            A[r, np.ravel_multi_index((i, n, m), shape)] += c / lam[i, n, m]
                        elif which == "tp":
                            A[r, np.ravel_multi_index((i, k, n), shape)] += c / tp[i, k, n]
                        else:
                            A[r, np.ravel_multi_index((t, k, n), shape)] += c / va[t, k, n]
    return A


@pytest.mark.parametrize("which,bit", [("lam", 2), ("tp", 4), ("va", 8)])
def test_mnmf_rules_are_auxiliary_minimizers(which, bit):
    """Each FastMNMF factor rule equals the brute-force minimizer of its own D+
    (the other factors held at their current values), the auxiliary function
    checked to majorize the cost first."""
    x, P, lam, tp, va, U = _mnmf_case()
    M = x.shape[2]
    A = coef_mnmf(which, lam, tp, va, M)
    theta0 = {"lam": lam, "tp": tp, "va": va}[which].reshape(-1)
    check_majorizes(theta0, A, _rows_mnmf(U), np.random.default_rng(bit))
    ref = brute_force_minimizer(theta0, A, _rows_mnmf(U))
    _, lam2, tp2, va2 = oracle.mnmf_iterate(x, P, lam, tp, va, bit)
    got = {"lam": lam2, "tp": tp2, "va": va2}[which].reshape(-1)
    np.testing.assert_allclose(got, ref, rtol=1e-7)

"""The algebraic forms the kernels use for the IP sweep (eq:ip1, eq:ip2), restated
in numpy and checked against the oracle's column-by-column solve on the CPU.

- M = 2: the adjugate closed form in which the second column is computed from
  the first column's u, before the first column's normalization, and the
  determinant of the new P from the same quantities.
- M = 3, 4: w_m = u / sqrt(b^H u), u = Q_m^{-1} b, b = P^{-H} e_m, with P^{-1}
  kept current by Sherman-Morrison updates and det P by the matrix determinant
  lemma.
These check the derivations; the GPU parity tests check the kernels.
"""
import numpy as np
import pytest

import oracle


def hpd(rng, M, k=3):
    A = rng.standard_normal((M, k * M)) + 1j * rng.standard_normal((M, k * M))
    return A @ A.conj().T / (k * M)


def general(rng, M):
    return np.eye(M) + 0.5 * (rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M)))


def oracle_sweep(P, Q):
    for m in range(P.shape[0]):
        P = oracle.ip_column(P, Q[m], m)
    return P, oracle.logabsdet2(P)


def closed_form_2(P, Qs, qscale):
    """Qs: T times the Q_m; qscale = sqrt(T)."""
    (P00, P01), (P10, P11) = P

    def adj(Q, b0, b1):
        return Q[1, 1] * b0 - Q[0, 1] * b1, Q[0, 0] * b1 - Q[1, 0] * b0

    dq = [np.linalg.det(Q).real for Q in Qs]
    a0, a1 = adj(Qs[0], np.conj(P11), np.conj(-P01))
    sb = (P11 * a0 - P01 * a1).real
    d = P00 * P11 - P01 * P10
    t = sb * dq[0] * abs(d) ** 2
    be0, be1 = np.conj(-a1), np.conj(a0)
    n0, n1 = adj(Qs[1], be0, be1)
    sg = (np.conj(be0) * n0 + np.conj(be1) * n1).real
    de = a0 * P11 - P01 * a1
    t2 = sg * dq[1] * abs(de) ** 2
    c = qscale / np.sqrt(t) * d
    r2 = qscale / np.sqrt(t2)
    W = np.array([[a0 * c, r2 * n0 * de], [a1 * c, r2 * n1 * de]])
    return W, np.log(abs(np.linalg.det(W)) ** 2)


def inverse_form(P, Q):
    M = P.shape[0]
    P = P.copy()
    Qi = [np.linalg.inv(Q[m]) for m in range(M)]
    G = np.linalg.inv(P)
    ldet = np.log(abs(np.linalg.det(P)) ** 2)
    for m in range(M):
        b = np.conj(G[m, :])
        u = Qi[m] @ b
        s = (b.conj() @ u).real
        w = u / np.sqrt(s)
        a = w - P[:, m]
        Ga = G @ a
        den = 1.0 + Ga[m]
        G = G - np.outer(Ga, G[m, :]) / den
        ldet += np.log(abs(den) ** 2)
        P[:, m] = w
    return P, ldet, G


@pytest.mark.parametrize("seed", range(6))
def test_m2_closed_form_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    T = 1000.0
    Q = np.stack([hpd(rng, 2) for _ in range(2)])
    P0 = np.eye(2, dtype=complex) if seed == 0 else general(rng, 2)
    Po, lo = oracle_sweep(P0, Q)
    W, lw = closed_form_2(P0, T * Q, np.sqrt(T))
    assert np.abs(W - Po).max() <= 1e-12 * np.abs(Po).max()
    assert abs(lw - lo) <= 1e-11


@pytest.mark.parametrize("M", [3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("seed", range(4))
def test_inverse_form_matches_oracle(M, seed):
    """The form of the resident kernels' sweep for M = 3, 4 and of the wide
    kernels' sweep for M up to 8."""
    rng = np.random.default_rng(100 + 10 * M + seed)
    Q = np.stack([hpd(rng, M) for _ in range(M)])
    P0 = np.eye(M, dtype=complex) if seed == 0 else general(rng, M)
    Po, lo = oracle_sweep(P0, Q)
    Pi, li, G = inverse_form(P0, Q)
    assert np.abs(Pi - Po).max() <= 1e-11 * np.abs(Po).max()
    assert abs(li - lo) <= 1e-10
    # the updated inverse is the inverse of the new P
    assert np.abs(G @ Pi - np.eye(M)).max() <= 1e-10

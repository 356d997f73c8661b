"""Pins of the oracle's FastMNMF (Sec. V and its appendix): h_{ijn} =
sum_k t_{ikn} v_{jkn}, IP for every W_i, majorization-minimization for
Lambda, T and V.

Checked against: the full-matrix Gaussian density with that h, monotonicity
of every sub-update, two special cases in which the T and the V rules reduce
to the (separately pinned) multiplicative rule of Algorithm 2 for H, the
Lambda rule against Algorithm 2's L rule, and stationarity of the cost at a
fixed point by finite differences.
"""
import numpy as np
import pytest

import oracle
from oracle import explicit
from paper_2101_08563_amd import synth


def _case(F=3, T=40, M=2, N=3, K=4, cid=80):
    x = synth.mixture(F=F, T=T, M=M, N=N, rank=3, diffuse=0.1, config_id=cid)
    P, lam, tp, va = synth.init_params_mnmf(x, N, K, config_id=cid)
    return x, P, lam.astype(np.float64), tp.astype(np.float64), va.astype(np.float64)


def test_h_is_the_nmf_product():
    rng = np.random.default_rng(0)
    tp = rng.random((4, 3, 2))
    va = rng.random((7, 3, 2))
    np.testing.assert_allclose(oracle.mnmf_h(tp, va), np.einsum("ikn,jkn->ijn", tp, va), rtol=1e-14)


def test_loglik_equals_full_matrix_density():
    x, P, lam, tp, va = _case(F=2, T=9, M=3, N=4, K=2, cid=81)
    P = P + 0.3 * np.random.default_rng(1).standard_normal(P.shape)
    ll, llf = oracle.mnmf_loglik(x, P, lam, tp, va)
    h = np.einsum("ikn,jkn->ijn", tp, va)
    ref = [explicit.loglik_freq(x[i], P[i], lam[i], h[i]) for i in range(2)]
    np.testing.assert_allclose(llf, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("what", [1, 2, 4, 8])
def test_every_sub_update_is_monotone(what):
    x, P, lam, tp, va = _case()
    for _ in range(3):  # from a few different iterates
        before, _ = oracle.mnmf_loglik(x, P, lam, tp, va)
        P2, lam2, tp2, va2 = oracle.mnmf_iterate(x, P, lam, tp, va, what)
        after, _ = oracle.mnmf_loglik(x, P2, lam2, tp2, va2)
        assert after >= before - 1e-12 * abs(before), (what, before, after)
        P, lam, tp, va = oracle.mnmf_iterate(x, P, lam, tp, va, 15)


def test_lambda_rule_is_algorithm2_l_rule():
    x, P, lam, tp, va = _case(cid=82)
    _, lam2, _, _ = oracle.mnmf_iterate(x, P, lam, tp, va, 2)
    h = np.einsum("ikn,jkn->ijn", tp, va)
    for i in range(x.shape[0]):
        U = oracle.decorrelated_power(P[i], x[i])
        l_ref, _ = oracle.mm_update(U, lam[i], h[i])
        np.testing.assert_allclose(lam2[i], l_ref, rtol=1e-12)


def test_t_rule_with_identity_activations_is_algorithm2_h_rule():
    """K = T and v_{jkn} = delta_{jk}: h_{ijn} = t_{ijn} is a free per-bin
    power and the Lambda-then-T update is Algorithm 2's L-then-H update."""
    F, T, M, N = 2, 12, 2, 3
    x, P, lam, _, _ = _case(F=F, T=T, M=M, N=N, K=T, cid=83)
    rng = np.random.default_rng(3)
    tp = 0.2 + rng.random((F, T, N))
    va = np.broadcast_to(np.eye(T)[:, :, None], (T, T, N)).copy()
    _, lam2, tp2, va2 = oracle.mnmf_iterate(x, P, lam, tp, va, 2 | 4)
    for i in range(F):
        U = oracle.decorrelated_power(P[i], x[i])
        l_ref, v_ref = oracle.mm_update(U, lam[i], tp[i])
        np.testing.assert_allclose(lam2[i], l_ref, rtol=1e-12)
        np.testing.assert_allclose(tp2[i], v_ref, rtol=1e-12)


def test_v_rule_with_identity_patterns_is_algorithm2_h_rule():
    """K = F and t_{ikn} = delta_{ik}: h_{ijn} = v_{jin} and the Lambda-then-V
    update is Algorithm 2's L-then-H update of every frequency."""
    F, T, M, N = 3, 10, 2, 3
    x, P, lam, _, _ = _case(F=F, T=T, M=M, N=N, K=F, cid=84)
    rng = np.random.default_rng(4)
    tp = np.broadcast_to(np.eye(F)[:, :, None], (F, F, N)).copy()
    va = 0.2 + rng.random((T, F, N))
    _, lam2, _, va2 = oracle.mnmf_iterate(x, P, lam, tp, va, 2 | 8)
    for i in range(F):
        U = oracle.decorrelated_power(P[i], x[i])
        l_ref, v_ref = oracle.mm_update(U, lam[i], va[:, i, :])
        np.testing.assert_allclose(lam2[i], l_ref, rtol=1e-12)
        np.testing.assert_allclose(va2[:, i, :], v_ref, rtol=1e-12)


def test_tensor_decomposition_fixed_point_is_stationary():
    """With W fixed (no IP), the Lambda/T/V updates are MM on the bounded
    Itakura-Saito part of eq:FastMNMFcost; after many iterations the
    log-likelihood is stationary in log lambda, log t and log v (central
    differences of the oracle's own LL)."""
    x, P, lam, tp, va = _case(F=6, T=40, M=2, N=3, K=2, cid=85)
    P = P + 0.2 * np.random.default_rng(6).standard_normal(P.shape)
    prev = -np.inf
    for it in range(4000):
        P, lam, tp, va = oracle.mnmf_iterate(x, P, lam, tp, va, 2 | 4 | 8)
        if it % 500 == 0:
            ll = oracle.mnmf_loglik(x, P, lam, tp, va)[0]
            assert ll >= prev - 1e-12 * abs(ll)
            prev = ll
    h = 1e-5
    rng = np.random.default_rng(5)
    for name, arr in (("lam", lam), ("tp", tp), ("va", va)):
        for _ in range(4):
            idx = tuple(rng.integers(0, d) for d in arr.shape)
            vals = []
            for sgn in (+1, -1):
                a = arr.copy()
                a[idx] *= np.exp(sgn * h)
                args = dict(lam=lam, tp=tp, va=va)
                args[name] = a
                vals.append(oracle.mnmf_loglik(x, P, args["lam"], args["tp"], args["va"])[0])
            g = (vals[0] - vals[1]) / (2 * h)
            assert abs(g) < 1e-6, (name, idx, g)


def test_fit_trace_is_monotone_and_matches_iterate():
    x, P, lam, tp, va = _case(cid=86)
    P1, l1, t1, v1, tr = oracle.mnmf_fit(x, P, lam, tp, va, 15, trace=True)
    assert np.diff(tr).min() > -1e-12 * abs(tr[-1]) and tr[-1] > tr[0]
    for _ in range(15):
        P, lam, tp, va = oracle.mnmf_iterate(x, P, lam, tp, va, 15)
    for u, w in zip((P, lam, tp, va), (P1, l1, t1, v1)):
        np.testing.assert_array_equal(u, w)

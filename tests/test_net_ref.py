"""Pins of the FP64 network reference: backward = central finite differences,
PIT loss = brute force and invariant to the order of the target sources,
features and targets against their closed forms."""
import itertools

import numpy as np

from oracle import explicit, net_ref


def _tiny(seed=0):
    rng = np.random.default_rng(seed)
    S, M, N, C, L, T = 2, 2, 3, 4, 2, 11
    p = net_ref.init_params(M, N, C, L, seed=seed)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.1
    feat = rng.standard_normal((S, M, T))
    tv = rng.standard_normal((S, N, T))
    tl = rng.standard_normal((S, N * M))
    return p, feat, tv, tl, (S, M, N, C, L, T)


def _loss(p, feat, tv, tl, N, M, L, wl=0.5):
    lv, ll, _ = net_ref.forward(p, feat, L)
    loss, _, _, _ = net_ref.pit_loss(lv, tv, ll, tl, N, M, wl)
    return loss.sum()


def test_backward_matches_finite_differences():
    p, feat, tv, tl, (S, M, N, C, L, T) = _tiny(1)
    lv, ll, cache = net_ref.forward(p, feat, L)
    _, _, glv, gll = net_ref.pit_loss(lv, tv, ll, tl, N, M, 0.5)
    g = net_ref.backward(p, cache, glv, gll, L)
    rng = np.random.default_rng(2)
    h = 1e-6
    for name in p:
        idx = [tuple(rng.integers(0, d) for d in p[name].shape) for _ in range(4)]
        for ix in idx:
            q = {k: v.copy() for k, v in p.items()}
            q[name][ix] += h
            up = _loss(q, feat, tv, tl, N, M, L)
            q[name][ix] -= 2 * h
            dn = _loss(q, feat, tv, tl, N, M, L)
            fd = (up - dn) / (2 * h)
            an = g[name][ix]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, ix, fd, an)


def test_pit_is_min_over_orders_and_invariant_to_target_order():
    rng = np.random.default_rng(3)
    S, N, M, T = 4, 3, 2, 9
    lv = rng.standard_normal((S, N, T))
    tv = rng.standard_normal((S, N, T))
    ll = rng.standard_normal((S, N * M))
    tl = rng.standard_normal((S, N * M))
    loss, perms, _, _ = net_ref.pit_loss(lv, tv, ll, tl, N, M, 0.3)
    for s in range(S):
        vals = []
        for pi in itertools.permutations(range(N)):
            a = np.mean([(lv[s, pi[n]] - tv[s, n]) ** 2 for n in range(N)])
            b = np.mean([(ll[s].reshape(N, M)[pi[n]] - tl[s].reshape(N, M)[n]) ** 2 for n in range(N)])
            vals.append(a + 0.3 * b)
        assert abs(loss[s] - min(vals)) < 1e-12
    # relabel the targets: same loss
    q = [2, 0, 1]
    loss2, _, _, _ = net_ref.pit_loss(lv, tv[:, q], ll, tl.reshape(S, N, M)[:, q].reshape(S, -1), N, M, 0.3)
    np.testing.assert_allclose(loss2, loss, atol=1e-12)


def test_features_whiten_the_mixture():
    rng = np.random.default_rng(4)
    x = (rng.standard_normal((3, 200, 2)) + 1j * rng.standard_normal((3, 200, 2))) * [1.0, 3.0]
    P0, feat = net_ref.features(x, 1e-9)
    for f in range(3):
        C = x[f].T @ x[f].conj() / 200
        np.testing.assert_allclose(P0[f].conj().T @ C @ P0[f], np.eye(2), atol=1e-10)
        np.testing.assert_allclose(P0[f], P0[f].conj().T, atol=1e-12)
    np.testing.assert_allclose(feat.mean(axis=2), 0, atol=1e-12)


def test_targets_preserve_the_model_covariance():
    """Trace normalization rescales R_n and v_n reciprocally: v_n R_n, hence the
    model, is unchanged; tl are the diagonals of P0^H R_n P0."""
    rng = np.random.default_rng(5)
    F, T, M, N = 2, 6, 2, 3
    P = rng.standard_normal((F, M, M)) + 1j * rng.standard_normal((F, M, M)) + 2 * np.eye(M)
    lam = rng.random((F, N, M)) + 0.2
    v = rng.random((F, T, N)) + 0.1
    P0 = np.stack([np.eye(M)] * F).astype(complex)
    tv, tl = net_ref.targets(P, lam, v, P0)
    for f in range(F):
        R = explicit.scm(P[f], lam[f])
        for n in range(N):
            c = np.trace(R[n]).real / M
            Rn = R[n] / c
            assert abs(np.trace(Rn).real - M) < 1e-12
            np.testing.assert_allclose(np.exp(tv[f, n]) * Rn[0, 0].real, v[f, :, n] * R[n][0, 0].real, rtol=1e-12)
            np.testing.assert_allclose(np.exp(tl[f, n]), np.real(np.diag(Rn)), rtol=1e-12)


def test_adamw_two_steps_from_the_decoupled_definition():
    """AdamW (Adam with decoupled weight decay): after k steps the first and
    second moments are the bias-corrected exponential averages
        m_k = (1 - b1) sum_{i<=k} b1^(k-i) g_i,   v_k = (1 - b2) sum_{i<=k} b2^(k-i) g_i^2,
    and the parameter moves by lr * (m_k / (1 - b1^k) / (sqrt(v_k / (1 - b2^k)) + eps)
    + wd * p_{k-1}), the decay acting on the parameter, not on the gradient.
    Written here with the moments summed out in closed form for two steps;
    a constant gradient makes the bias-corrected ratio exactly sign(g)."""
    lr, b1, b2, eps, wd = 0.1, 0.9, 0.999, 1e-8, 0.01
    # constant gradient: each step moves by lr * (1 + wd * p) (ratio exactly 1)
    p, m, v = np.array([1.0]), np.zeros(1), np.zeros(1)
    p1, m, v = net_ref.adamw(p, np.array([0.5]), m, v, lr, b1, b2, 0.0, wd, 1, 1.0)
    p2, m, v = net_ref.adamw(p1, np.array([0.5]), m, v, lr, b1, b2, 0.0, wd, 2, 1.0)
    np.testing.assert_allclose(p1, 1.0 - lr * (1.0 + wd * 1.0), rtol=1e-14)
    np.testing.assert_allclose(p2, p1 - lr * (1.0 + wd * p1), rtol=1e-14)
    # two different gradients, with a gradient scale of 0.5 applied first
    g1, g2, gs = 0.8, -0.3, 0.5
    p0 = np.array([2.0])
    q1, m, v = net_ref.adamw(p0, np.array([g1]), np.zeros(1), np.zeros(1), lr, b1, b2, eps, wd, 1, gs)
    q2, m, v = net_ref.adamw(q1, np.array([g2]), m, v, lr, b1, b2, eps, wd, 2, gs)
    a1, a2 = gs * g1, gs * g2
    m2 = (1 - b1) * (b1 * a1 + a2)
    v2 = (1 - b2) * (b2 * a1 ** 2 + a2 ** 2)
    step1 = a1 / (abs(a1) + eps)                       # m_1/(1-b1) = a1, v_1/(1-b2) = a1^2
    step2 = (m2 / (1 - b1 ** 2)) / (np.sqrt(v2 / (1 - b2 ** 2)) + eps)
    r1 = 2.0 - lr * (step1 + wd * 2.0)
    r2 = r1 - lr * (step2 + wd * r1)
    np.testing.assert_allclose(q1, r1, rtol=1e-14)
    np.testing.assert_allclose(q2, r2, rtol=1e-13)
    np.testing.assert_allclose(m, m2, rtol=1e-14)
    np.testing.assert_allclose(v, v2, rtol=1e-14)

"""FP64 reference of the warm-start network, its loss and its features --
TEST INFRASTRUCTURE (only tests may import it).

Architecture (per frequency, weights shared across frequencies), written
directly with numpy in double precision:
    h0 = relu(conv5(feat; W0, b0))                       feat [S, M, T]
    h_l = h_{l-1} + relu(conv5(h_{l-1}; W_l, b_l))       l = 1..L
    lv  = conv1(h_L; Wv, bv)                              [S, N, T]  (log v)
    ll  = Wl mean_t(h_L) + bl                             [S, N*M]   (log lambda)
conv5/conv1: 1-D convolution over time with kernel 5 / 1 and zero padding
that keeps the length. Loss: permutation-invariant mean squared error in the
log domain (min over the N! source orders per sequence).
"""
from __future__ import annotations

import itertools

import numpy as np


def conv(X, W, b):
    """X [S, Cin, T], W [Cout, Cin, K], b [Cout] or None -> [S, Cout, T]."""
    S, Cin, T = X.shape
    K = W.shape[2]
    R = K // 2
    Xp = np.pad(X, ((0, 0), (0, 0), (R, R)))
    Y = np.zeros((S, W.shape[0], T))
    for k in range(K):
        Y += np.einsum("oc,sct->sot", W[:, :, k], Xp[:, :, k:k + T])
    if b is not None:
        Y += b[None, :, None]
    return Y


def conv_grads(G, X, W):
    """Gradients of Y = conv(X, W, b) given dL/dY = G: (dX, dW, db)."""
    S, Cin, T = X.shape
    K = W.shape[2]
    R = K // 2
    Xp = np.pad(X, ((0, 0), (0, 0), (R, R)))
    dW = np.zeros_like(W)
    dXp = np.zeros_like(Xp)
    for k in range(K):
        dW[:, :, k] = np.einsum("sot,sct->oc", G, Xp[:, :, k:k + T])
        dXp[:, :, k:k + T] += np.einsum("oc,sot->sct", W[:, :, k], G)
    return dXp[:, :, R:R + T], dW, G.sum(axis=(0, 2))


def init_params(M, N, C, L, seed=0):
    rng = np.random.default_rng(seed)
    p = {"W0": rng.standard_normal((C, M, 5)) * np.sqrt(2.0 / (M * 5)), "b0": np.zeros(C)}
    for l in range(1, L + 1):
        p["W%d" % l] = rng.standard_normal((C, C, 5)) * np.sqrt(1.0 / (C * 5)) * 0.5
        p["b%d" % l] = np.zeros(C)
    p["Wv"] = rng.standard_normal((N, C, 1)) * np.sqrt(1.0 / C)
    p["bv"] = np.zeros(N)
    p["Wl"] = rng.standard_normal((N * M, C)) * np.sqrt(1.0 / C)
    p["bl"] = np.zeros(N * M)
    return p


def forward(p, feat, L):
    cache = {"h": [], "pre": []}
    pre = conv(feat, p["W0"], p["b0"])
    h = np.maximum(pre, 0.0)
    cache["pre"].append(pre)
    cache["h"].append(h)
    for l in range(1, L + 1):
        pre = conv(h, p["W%d" % l], p["b%d" % l])
        h = h + np.maximum(pre, 0.0)
        cache["pre"].append(pre)
        cache["h"].append(h)
    lv = conv(h, p["Wv"], p["bv"])
    pooled = h.mean(axis=2)
    ll = pooled @ p["Wl"].T + p["bl"]
    cache["feat"] = feat
    cache["pooled"] = pooled
    return lv, ll, cache


def backward(p, cache, glv, gll, L):
    g = {}
    hL = cache["h"][L]
    dh, g["Wv"], g["bv"] = conv_grads(glv, hL, p["Wv"])
    g["Wl"] = gll.T @ cache["pooled"]
    g["bl"] = gll.sum(axis=0)
    dpooled = gll @ p["Wl"]
    dh = dh + dpooled[:, :, None] / hL.shape[2]
    for l in range(L, 0, -1):
        gp = dh * (cache["pre"][l] > 0)
        dx, g["W%d" % l], g["b%d" % l] = conv_grads(gp, cache["h"][l - 1], p["W%d" % l])
        dh = dh + dx
    gp = dh * (cache["pre"][0] > 0)
    _, g["W0"], g["b0"] = conv_grads(gp, cache["feat"], p["W0"])
    return g


def pit_loss(lv, tv, ll, tl, N, M, wl):
    """Per sequence: min over orders of mean (lv[pi(n)] - tv[n])^2 +
    wl mean (ll[pi(n)] - tl[n])^2; returns (loss [S], perms [S,N], glv, gll).
    Orders in itertools (lexicographic) order; the first minimum is kept."""
    S, _, T = lv.shape
    ll = ll.reshape(S, N, M)
    tl = tl.reshape(S, N, M)
    loss = np.zeros(S)
    perms = np.zeros((S, N), int)
    glv = np.zeros_like(lv)
    gll = np.zeros_like(ll)
    for s in range(S):
        best, bp = np.inf, None
        for pi in itertools.permutations(range(N)):
            L1 = sum(((lv[s, pi[n]] - tv[s, n]) ** 2).sum() for n in range(N)) / (N * T)
            L2 = sum(((ll[s, pi[n]] - tl[s, n]) ** 2).sum() for n in range(N)) / (N * M)
            tot = L1 + wl * L2
            if tot < best:
                best, bp = tot, pi
        loss[s] = best
        perms[s] = bp
        for n in range(N):
            glv[s, bp[n]] = 2.0 * (lv[s, bp[n]] - tv[s, n]) / (N * T)
            gll[s, bp[n]] = wl * 2.0 * (ll[s, bp[n]] - tl[s, n]) / (N * M)
    return loss, perms, glv, gll.reshape(S, N * M)


def features(x, eps):
    """x [F, T, M] complex -> (P0 [F, M, M] = C^{-1/2}, feat [F, M, T])."""
    F, T, M = x.shape
    x = x.astype(np.complex128)
    P0 = np.zeros((F, M, M), np.complex128)
    feat = np.zeros((F, M, T))
    for f in range(F):
        C = x[f].T @ x[f].conj() / T
        ev, U = np.linalg.eigh(C)
        P0[f] = U @ np.diag(ev ** -0.5) @ U.conj().T
        y = x[f] @ P0[f].conj()          # y[t, m] = (P0^H x_t)_m
        a = np.log(np.abs(y) ** 2 + eps).T
        feat[f] = a - a.mean(axis=1, keepdims=True)
    return P0, feat


def targets(P, lam, v, P0):
    """Trace-normalized targets in the whitened basis (tv [F,N,T], tl [F,N,M])."""
    F, M, _ = P.shape
    N = lam.shape[1]
    T = v.shape[1]
    tv = np.zeros((F, N, T))
    tl = np.zeros((F, N, M))
    for f in range(F):
        B = np.linalg.inv(P[f])
        for n in range(N):
            R = B.conj().T @ np.diag(lam[f, n].astype(np.complex128)) @ B
            c = np.trace(R).real / M
            tl[f, n] = np.log(np.real(np.diag(P0[f].conj().T @ (R / c) @ P0[f])))
            tv[f, n] = np.log(v[f, :, n] * c)
    return tv, tl


def adamw(p, g, m, v, lr, b1, b2, eps, wd, step, gscale):
    g = g * gscale
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    p = p - lr * (mh / (np.sqrt(vh) + eps) + wd * p)
    return p, m, v

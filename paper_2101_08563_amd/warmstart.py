"""Learned warm start for FastFCA (binding over the library's network kernels).

A 1-D convolutional network over time, applied to every frequency with
shared weights, maps the whitened log-powers of a mixture to initial
lambda_n and v_n; Algorithm 1 then runs from (P0, lambda, v) with
P0 = C_f^{-1/2}. Every arithmetic step runs in libfastfca's HIP kernels
(BF16 MFMA convolutions with FP32 accumulation, PIT loss, AdamW, features,
targets); this module only allocates buffers (torch) and sequences calls.

Network (C channels, L residual layers, kernel 5 over time):
    h0 = relu(conv5(feat)); h_l = h_{l-1} + relu(conv5(h_{l-1}));
    log v = conv1(h_L) [N x T];  log lambda = W mean_t(h_L) + b [N*M].
"""
from __future__ import annotations

import ctypes
import math
import time

import numpy as np
import torch

from .fastfca import FastFCA, FastFCAError, NetDesc, _ptr, _stream, load_library, synth_mixture


def _kp(n):
    return (n + 15) // 16 * 16


def _chk(rc, lib):
    if rc != 0:
        raise FastFCAError(rc, lib.fastfca_net_last_error().decode())


class ConvNet:
    """Parameters, gradients, AdamW moments and BF16 operand copies of the network."""

    def __init__(self, M=2, N=3, C=64, L=6, seed=0, stream=None):
        self.lib = load_library()
        self.M, self.N, self.C, self.L = M, N, C, L
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        # conv layers: (Cout, Cin, ks)
        self.convs = [(C, M, 5)] + [(C, C, 5)] * L + [(N, C, 1)]
        dev = torch.device("cuda")
        rng = np.random.default_rng(seed)
        self.W, self.b, self.Wb, self.Wt = [], [], [], []
        for i, (co, ci, ks) in enumerate(self.convs):
            kp = _kp(ci * ks)
            w = np.zeros((co, kp), np.float32)
            if i == 0:
                std = math.sqrt(2.0 / (ci * ks))
            elif i <= L:
                std = 0.5 * math.sqrt(1.0 / (ci * ks))
            else:
                std = math.sqrt(1.0 / ci)
            w[:, :ci * ks] = rng.standard_normal((co, ci * ks)) * std
            self.W.append(torch.from_numpy(w).to(dev))
            self.b.append(torch.zeros(co, dtype=torch.float32, device=dev))
            self.Wb.append(torch.zeros((co, kp), dtype=torch.int16, device=dev))
            self.Wt.append(torch.zeros((ci, _kp(co * ks)), dtype=torch.int16, device=dev))
        self.Wl = torch.from_numpy((rng.standard_normal((N * M, C)) / math.sqrt(C)).astype(np.float32)).to(dev)
        self.bl = torch.zeros(N * M, dtype=torch.float32, device=dev)
        self.params = self.W + self.b + [self.Wl, self.bl]
        self.grads = [torch.zeros_like(p) for p in self.params]
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.step_count = 0
        self.pack()

    # -------------------------------------------------------------- weights
    def n_params(self):
        n = sum(co * ci * ks + co for co, ci, ks in self.convs)
        return n + self.Wl.numel() + self.bl.numel()

    def pack(self):
        s = _stream(self.stream)
        for i, (co, ci, ks) in enumerate(self.convs):
            kp = _kp(ci * ks)
            _chk(self.lib.fastfca_net_pack_weights(_ptr(self.W[i]), kp, co, ci, ks, kp, 0, _ptr(self.Wb[i]), s),
                 self.lib)
            _chk(self.lib.fastfca_net_pack_weights(_ptr(self.W[i]), kp, co, ci, ks, _kp(co * ks), 1,
                                                   _ptr(self.Wt[i]), s), self.lib)

    def state_dict(self):
        """Weights as numpy arrays with unpadded conv layouts [Cout][Cin][ks]."""
        d = {}
        for i, (co, ci, ks) in enumerate(self.convs):
            d["W%d" % i] = self.W[i].cpu().numpy()[:, :ci * ks].reshape(co, ci, ks).copy()
            d["b%d" % i] = self.b[i].cpu().numpy().copy()
        d["Wl"] = self.Wl.cpu().numpy().copy()
        d["bl"] = self.bl.cpu().numpy().copy()
        d["arch"] = np.array([self.M, self.N, self.C, self.L], np.int64)
        return d

    def load_state_dict(self, d):
        for i, (co, ci, ks) in enumerate(self.convs):
            w = np.zeros((co, _kp(ci * ks)), np.float32)
            w[:, :ci * ks] = np.asarray(d["W%d" % i], np.float32).reshape(co, ci * ks)
            self.W[i].copy_(torch.from_numpy(w))
            self.b[i].copy_(torch.from_numpy(np.asarray(d["b%d" % i], np.float32)))
        self.Wl.copy_(torch.from_numpy(np.asarray(d["Wl"], np.float32)))
        self.bl.copy_(torch.from_numpy(np.asarray(d["bl"], np.float32)))
        self.pack()

    def save(self, path, meta=None):
        """Weights, and provenance fields (meta: name -> value) stored as
        prov_<name> string arrays."""
        d = self.state_dict()
        for k, v in (meta or {}).items():
            d["prov_" + k] = np.array(str(v))
        np.savez(path, **d)

    @classmethod
    def load(cls, path, stream=None):
        d = dict(np.load(path, allow_pickle=False))
        M, N, C, L = (int(a) for a in d["arch"])
        net = cls(M=M, N=N, C=C, L=L, stream=stream)
        net.load_state_dict(d)
        return net

    # -------------------------------------------------------------- forward
    def _conv(self, i, X, S, T, Y, mode, res=None, pre=None, bias=True):
        co, ci, ks = self.convs[i]
        _chk(self.lib.fastfca_net_conv_fwd(_ptr(X), S, ci, T, _ptr(self.Wb[i]), _kp(ci * ks), ks,
                                           _ptr(self.b[i]) if bias else None, co, _ptr(Y), mode, _ptr(res),
                                           _ptr(pre), _stream(self.stream)), self.lib)

    def forward(self, feat, keep=True):
        """feat [S, M, T] float32 -> (lv [S, N, T], ll [S, N*M])."""
        S, M, T = feat.shape
        C, L, N = self.C, self.L, self.N
        dev = feat.device
        hs = [torch.empty((S, C, T), dtype=torch.float32, device=dev) for _ in range(L + 1)]
        pres = [torch.empty((S, C, T), dtype=torch.float32, device=dev) for _ in range(L + 1)] if keep else None
        self._conv(0, feat, S, T, hs[0], 1, pre=pres[0] if keep else None)
        for l in range(1, L + 1):
            self._conv(l, hs[l - 1], S, T, hs[l], 2, res=hs[l - 1], pre=pres[l] if keep else None)
        lv = torch.empty((S, N, T), dtype=torch.float32, device=dev)
        self._conv(L + 1, hs[L], S, T, lv, 0)
        pooled = torch.empty((S, C), dtype=torch.float32, device=dev)
        _chk(self.lib.fastfca_net_mean_t(_ptr(hs[L]), S * C, T, _ptr(pooled), _stream(self.stream)), self.lib)
        ll = torch.empty((S, N * M), dtype=torch.float32, device=dev)
        _chk(self.lib.fastfca_net_linear_fwd(_ptr(pooled), S, C, _ptr(self.Wl), _ptr(self.bl), N * M, _ptr(ll),
                                             _stream(self.stream)), self.lib)
        if keep:
            self._cache = (feat, hs, pres, pooled)
        return lv, ll

    def descriptor(self):
        """The fastfca_net descriptor of this network (for fastfca_warmstart);
        the host pointer arrays live as long as the network."""
        L = self.L
        self._wb_arr = (ctypes.c_void_p * (L + 1))(*[self.Wb[i].data_ptr() for i in range(L + 1)])
        self._b_arr = (ctypes.c_void_p * (L + 1))(*[self.b[i].data_ptr() for i in range(L + 1)])
        wv = self.W[L + 1]
        return NetDesc(M=self.M, N=self.N, C=self.C, L=L,
                       Wb=ctypes.cast(self._wb_arr, ctypes.c_void_p).value,
                       b=ctypes.cast(self._b_arr, ctypes.c_void_p).value, Kp0=_kp(self.M * 5),
                       Wv=wv.data_ptr(), ldv=wv.shape[1], bv=self.b[L + 1].data_ptr(),
                       Wl=self.Wl.data_ptr(), bl=self.bl.data_ptr())

    def fused_ok(self):
        """Shapes the one-launch inference kernel takes."""
        return self.C % 16 == 0 and self.C <= 64 and self.L <= 8 and self.N <= 8 and self.M <= 4

    def forward_fused(self, feat):
        """Inference forward in one launch (activations kept in LDS per time
        tile), feat [S, M, T] float32 -> (lv [S, N, T], ll [S, N*M])."""
        S, M, T = feat.shape
        C, L, N = self.C, self.L, self.N
        dev = feat.device
        feat = feat.contiguous()
        ntiles = (T + 63) // 64
        lv = torch.empty((S, N, T), dtype=torch.float32, device=dev)
        part = torch.empty((S * ntiles * C,), dtype=torch.float32, device=dev)
        pooled = torch.empty((S, C), dtype=torch.float32, device=dev)
        wb = (ctypes.c_void_p * (L + 1))(*[self.Wb[i].data_ptr() for i in range(L + 1)])
        bb = (ctypes.c_void_p * (L + 1))(*[self.b[i].data_ptr() for i in range(L + 1)])
        wv = self.W[L + 1]
        _chk(self.lib.fastfca_net_forward_fused(_ptr(feat), S, M, T, C, L, N, ctypes.cast(wb, ctypes.c_void_p),
                                                ctypes.cast(bb, ctypes.c_void_p), _kp(M * 5), _ptr(wv),
                                                wv.shape[1], _ptr(self.b[L + 1]), _ptr(lv), _ptr(part),
                                                _ptr(pooled), _stream(self.stream)), self.lib)
        ll = torch.empty((S, N * M), dtype=torch.float32, device=dev)
        _chk(self.lib.fastfca_net_linear_fwd(_ptr(pooled), S, C, _ptr(self.Wl), _ptr(self.bl), N * M, _ptr(ll),
                                             _stream(self.stream)), self.lib)
        return lv, ll

    # -------------------------------------------------------------- backward
    def zero_grad(self):
        for g in self.grads:
            g.zero_()

    def backward(self, glv, gll):
        """Accumulate gradients from dLoss/dlv [S,N,T] and dLoss/dll [S,N*M]."""
        feat, hs, pres, pooled = self._cache
        S, M, T = feat.shape
        C, L, N = self.C, self.L, self.N
        s = _stream(self.stream)
        nconv = len(self.convs)
        gW = self.grads[:nconv]
        gb = self.grads[nconv:2 * nconv]
        gWl, gbl = self.grads[2 * nconv], self.grads[2 * nconv + 1]

        def bwdw(i, G, X):
            co, ci, ks = self.convs[i]
            _chk(self.lib.fastfca_net_conv_bwd_weight(_ptr(G), S, co, _ptr(X), ci, T, _kp(ci * ks), ks,
                                                      _ptr(gW[i]), _ptr(gb[i]), s), self.lib)

        def bwdx(i, G, out, mode, res=None):
            co, ci, ks = self.convs[i]
            _chk(self.lib.fastfca_net_conv_fwd(_ptr(G), S, co, T, _ptr(self.Wt[i]), _kp(co * ks), ks, None, ci,
                                               _ptr(out), mode, _ptr(res), None, s), self.lib)

        bwdw(L + 1, glv, hs[L])
        dh = torch.empty((S, C, T), dtype=torch.float32, device=feat.device)
        bwdx(L + 1, glv, dh, 0)
        dpooled = torch.empty((S, C), dtype=torch.float32, device=feat.device)
        _chk(self.lib.fastfca_net_linear_bwd(_ptr(pooled), S, C, _ptr(self.Wl), N * M, _ptr(gll), _ptr(gWl),
                                             _ptr(gbl), _ptr(dpooled), s), self.lib)
        _chk(self.lib.fastfca_net_mean_t_bwd(_ptr(dpooled), S * C, T, _ptr(dh), s), self.lib)
        gp = torch.empty_like(dh)
        for l in range(L, 0, -1):
            _chk(self.lib.fastfca_net_relu_grad(_ptr(dh), _ptr(pres[l]), _ptr(gp), dh.numel(), s), self.lib)
            bwdw(l, gp, hs[l - 1])
            bwdx(l, gp, dh, 3, res=dh)
        _chk(self.lib.fastfca_net_relu_grad(_ptr(dh), _ptr(pres[0]), _ptr(gp), dh.numel(), s), self.lib)
        bwdw(0, gp, feat)

    def step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=1e-4, grad_scale=1.0):
        self.step_count += 1
        s = _stream(self.stream)
        for p, g, m, v in zip(self.params, self.grads, self.m, self.v):
            _chk(self.lib.fastfca_net_adamw(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(), lr, beta1, beta2, eps,
                                            weight_decay, self.step_count, grad_scale, s), self.lib)
        self.pack()


# ------------------------------------------------------------------ data
def pit_loss(lv, tv, ll, tl, N, M, wl=0.5, grads=True, stream=None):
    """Permutation-invariant loss per sequence and its gradients (library kernel)."""
    lib = load_library()
    S, _, T = lv.shape
    loss = torch.empty(S, dtype=torch.float32, device=lv.device)
    perm = torch.empty((S, N), dtype=torch.int32, device=lv.device)
    glv = torch.empty_like(lv) if grads else None
    gll = torch.empty_like(ll) if grads else None
    _chk(lib.fastfca_net_pit_loss(_ptr(lv), _ptr(tv), _ptr(ll), _ptr(tl), S, N, M, T, wl, _ptr(loss), _ptr(perm),
                                  _ptr(glv), _ptr(gll), _stream(stream)), lib)
    return loss, perm, glv, gll


def features(x, eps=1e-8, stream=None):
    """x [F,T,M] complex64 -> (P0 [F,M,M] complex128, feat [F,M,T] float32)."""
    lib = load_library()
    F, T, M = x.shape
    P0 = torch.empty((F, M, M), dtype=torch.complex128, device=x.device)
    feat = torch.empty((F, M, T), dtype=torch.float32, device=x.device)
    _chk(lib.fastfca_ws_features(_ptr(x), F, T, M, eps, _ptr(P0), _ptr(feat), _stream(stream)), lib)
    return P0, feat


def targets(P, lam, v, P0, stream=None):
    lib = load_library()
    F, M, _ = P.shape
    N = lam.shape[1]
    T = v.shape[1]
    tv = torch.empty((F, N, T), dtype=torch.float32, device=P.device)
    tl = torch.empty((F, N * M), dtype=torch.float32, device=P.device)
    _chk(lib.fastfca_ws_targets(_ptr(P), _ptr(lam), _ptr(v), _ptr(P0), F, T, M, N, _ptr(tv), _ptr(tl),
                                _stream(stream)), lib)
    return tv, tl


def apply_outputs(lv, ll, M, stream=None):
    """Network outputs -> (lam [F,N,M], v [F,T,N])."""
    lib = load_library()
    F, N, T = lv.shape
    v = torch.empty((F, T, N), dtype=torch.float32, device=lv.device)
    lam = torch.empty((F, N, M), dtype=torch.float32, device=lv.device)
    _chk(lib.fastfca_ws_apply(_ptr(lv), _ptr(ll), F, T, M, N, _ptr(v), _ptr(lam), _stream(stream)), lib)
    return lam, v


def warm_init(net, x, stream=None, chunk=1024):
    """Whitening + network -> (P0, lam, v) initial parameters for one mixture."""
    P0, feat = features(x, stream=stream)
    F = x.shape[0]
    lvs, lls = [], []
    for a in range(0, F, chunk):
        lv, ll = net.forward_fused(feat[a:a + chunk]) if net.fused_ok() else net.forward(feat[a:a + chunk], keep=False)
        lvs.append(lv)
        lls.append(ll)
    lv = torch.cat(lvs) if len(lvs) > 1 else lvs[0]
    ll = torch.cat(lls) if len(lls) > 1 else lls[0]
    lam, v = apply_outputs(lv, ll.view(F, net.N, net.M), net.M, stream=stream)
    return P0, lam, v


def make_training_set(n_mix, F, T, M, N, fit_iters, seed0, batch=16, rank=8, diffuse=0.05, log=print):
    """Generate mixtures on the GPU, fit them with the batched IP+EM (library
    seeded init, fit_iters iterations) and return (feat [n*F, M, T],
    tv [n*F, N, T], tl [n*F, N*M]) float32 CUDA tensors."""
    feats, tvs, tls = [], [], []
    t0 = time.time()
    for a in range(0, n_mix, batch):
        xs = [synth_mixture(F, T, M, N, rank=rank, diffuse=diffuse, seed=seed0 + i)
              for i in range(a, min(n_mix, a + batch))]
        ctx = FastFCA.from_batch([dict(x=x, N=N) for x in xs], seed=seed0 + a)
        ctx.em_step(fit_iters)
        ctx.sync()
        for b, x in enumerate(xs):
            P, lam, v = ctx.get_params(b)
            P0, feat = features(x)
            tv, tl = targets(P, lam, v, P0)
            feats.append(feat)
            tvs.append(tv)
            tls.append(tl)
        ctx.close()
        if log and (a // batch) % 16 == 0:
            log("training set: %d/%d mixtures fitted (%.1f s)" % (min(n_mix, a + batch), n_mix, time.time() - t0))
    return torch.cat(feats), torch.cat(tvs), torch.cat(tls)


def converged_fit(xs, N, seed, max_iters=2000, tol=1e-7, block=100):
    """Batched IP+EM from the library's seeded start until every mixture's
    log-likelihood per bin gains less than tol in one iteration, or max_iters
    iterations; returns (context, iterations run)."""
    ctx = FastFCA.from_batch([dict(x=x, N=N) for x in xs], seed=seed)
    done = 0
    try:
        while done < max_iters:
            ctx.em_step(block)
            done += block
            gains = [float(tr[-1] - tr[-2]) for tr in (ctx.ll_trace(b) for b in range(len(xs)))]
            if max(gains) < tol:
                break
    except FastFCAError:
        ctx.close()
        raise
    return ctx, done


def chunk_training_set(seeds, F, T, M, N, rank=8, diffuse=0.05, max_iters=2000, tol=1e-7):
    """Features and targets of the mixtures with the given seeds (drawn on the
    GPU), from converged fits: (feat [n*F, M, T], tv [n*F, N, T], tl [n*F, N*M],
    iterations of the fit)."""
    xs = [synth_mixture(F, T, M, N, rank=rank, diffuse=diffuse, seed=s) for s in seeds]
    ctx, iters = converged_fit(xs, N, seed=int(seeds[0]), max_iters=max_iters, tol=tol)
    feats, tvs, tls = [], [], []
    for b, x in enumerate(xs):
        P, lam, v = ctx.get_params(b)
        P0, feat = features(x)
        tv, tl = targets(P, lam, v, P0)
        feats.append(feat)
        tvs.append(tv)
        tls.append(tl)
    ctx.close()
    return torch.cat(feats), torch.cat(tvs), torch.cat(tls), iters


def _sgd_steps(net, feat, tv, tl, n_steps, g, batch, lr_at, wl, it0):
    n = feat.shape[0]
    loss = None
    for k in range(n_steps):
        idx = torch.randint(0, n, (batch,), generator=g).to(feat.device)
        f, a, b = feat[idx].contiguous(), tv[idx].contiguous(), tl[idx].contiguous()
        lv, ll = net.forward(f)
        loss, _, glv, gll = pit_loss(lv, a, ll, b, net.N, net.M, wl=wl)
        net.zero_grad()
        net.backward(glv, gll)
        net.step(lr=lr_at(it0 + k + 1), grad_scale=1.0 / batch)
    return float(loss.mean()) if loss is not None else float("nan")


def train_stream(net, n_train, F, T, M, N, chunk=64, epochs=1, steps_per_chunk=0, minutes=0.0, batch=256,
                 lr=1e-3, wl=0.5, seed=0, log=print, log_every=20, max_fit_iters=2000, tol=1e-7):
    """AdamW over n_train generated mixtures (seeds 0..n_train-1) in chunks:
    each chunk is drawn and fitted to convergence on the GPU, turned into
    features and targets, trained on for steps_per_chunk minibatches of
    sequences (frequencies) drawn from it, then discarded; no training set is
    stored. With steps_per_chunk 0 it is sized from the first chunk's measured
    fit and step times so that the run takes about `minutes`. The learning
    rate follows a cosine decay over all steps. A chunk whose fit fails
    (a singular or non-finite frequency) is skipped and counted.
    Returns dict(history=[(step, loss)], fit_iters=[...], skipped=k, steps_per_chunk=s)."""
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    n_chunks = (n_train + chunk - 1) // chunk
    hist, fit_iters = [], []
    skipped = 0
    total = [1]
    it = 0
    t0 = time.time()

    def lr_at(k):
        return lr * 0.5 * (1.0 + math.cos(math.pi * min(k, total[0]) / total[0]))

    for ep in range(epochs):
        order = torch.randperm(n_chunks, generator=g).tolist()
        for ci, c in enumerate(order):
            seeds = list(range(c * chunk, min(n_train, (c + 1) * chunk)))
            tf = time.time()
            try:
                feat, tv, tl, fi = chunk_training_set(seeds, F, T, M, N, max_iters=max_fit_iters, tol=tol)
            except FastFCAError as e:
                skipped += 1
                if log:
                    log("chunk of seeds %d..%d skipped: %s" % (seeds[0], seeds[-1], e))
                continue
            torch.cuda.synchronize()
            tf = time.time() - tf
            fit_iters.append(fi)
            if not steps_per_chunk:
                # size the run from this chunk: fit time and the time of a few steps
                ts = time.time()
                _sgd_steps(net, feat, tv, tl, 4, g, batch, lambda k: 0.0, wl, 0)
                torch.cuda.synchronize()
                per_step = (time.time() - ts) / 4
                budget = minutes * 60.0 - (time.time() - t0)
                spc = int((budget / (epochs * n_chunks) - tf) / per_step)
                steps_per_chunk = max(8, spc)
                if log:
                    log("fit of a chunk %.2f s, %.2f ms per step: %d steps per chunk"
                        % (tf, per_step * 1e3, steps_per_chunk))
            total[0] = epochs * n_chunks * steps_per_chunk
            val = _sgd_steps(net, feat, tv, tl, steps_per_chunk, g, batch, lr_at, wl, it)
            it += steps_per_chunk
            hist.append((it, val))
            if log and (ci % log_every == 0 or ci == n_chunks - 1):
                log("epoch %d chunk %d/%d (fit %d iterations, %.2f s) step %d/%d loss %.4f (%.1f s)"
                    % (ep, ci + 1, n_chunks, fi, tf, it, total[0], val, time.time() - t0))
            del feat, tv, tl
    return dict(history=hist, fit_iters=fit_iters, skipped=skipped, steps_per_chunk=steps_per_chunk)


def train(net, feat, tv, tl, steps, batch=256, lr=1e-3, wl=0.5, seed=0, log=print, log_every=200):
    """AdamW on random minibatches of sequences (frequencies); returns the loss history."""
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    n = feat.shape[0]
    hist = []
    t0 = time.time()
    for it in range(1, steps + 1):
        idx = torch.randint(0, n, (batch,), generator=g).to(feat.device)
        f, a, b = feat[idx].contiguous(), tv[idx].contiguous(), tl[idx].contiguous()
        lv, ll = net.forward(f)
        loss, _, glv, gll = pit_loss(lv, a, ll, b, net.N, net.M, wl=wl)
        net.zero_grad()
        net.backward(glv, gll)
        # cosine decay of the learning rate
        cur = lr * 0.5 * (1.0 + math.cos(math.pi * it / steps))
        net.step(lr=cur, grad_scale=1.0 / batch)
        if it % log_every == 0 or it == 1:
            val = float(loss.mean())
            hist.append((it, val))
            if log:
                log("train step %d/%d loss %.4f (%.1f s)" % (it, steps, val, time.time() - t0))
    return hist

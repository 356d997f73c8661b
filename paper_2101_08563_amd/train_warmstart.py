"""Train and evaluate the learned warm start on synthetic mixtures.

  python -m paper_2101_08563_amd.train_warmstart train --out W.npz [--n-train 2048 --fit-iters 1000
         --minutes 8 --batch 256]
  python -m paper_2101_08563_amd.train_warmstart eval --weights W.npz [--n-eval 512 --conv-iters 1500]

Workload: M=2 microphones, N=3 sources, F=513 bins, T=1000 frames (the paper's
STFT shape), mixtures drawn on the GPU by fastfca_synth_mixture. Training
mixtures use seeds 0..n_train-1, evaluation mixtures seeds 10^6 + i.

Targets: the IP+EM fit of each training mixture after --fit-iters iterations
from the library's seeded initialization, trace-normalized and expressed in
the whitened basis P0 = C_f^{-1/2} (fastfca_ws_targets).

Evaluation (per held-out mixture): LL* = the plain fit's log-likelihood per
bin after --conv-iters iterations; iterations (and wall time) to reach
LL* - 1e-2 from (a) the seeded initialization, (b) the network's warm start
(P0, exp(lambda_hat), exp(v_hat)) and (c) a whitening-only start (P0,
lambda = 1, v = whitened power / N); for diagnosis also (d) the plain fit's
own targets fed back through the warm-start path (a perfect network), (e)
its lambda with the power-based v and (f) the network's lambda with the
power-based v. The warm start is judged by its initial
log-likelihood: if it is not finite or below that of the seeded start, the
seeded start is used (fallback).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import warmstart
from .fastfca import FastFCA, synth_mixture
from .warmstart import ConvNet

F, T, M, N = 513, 1000, 2, 3
TOL = 1e-2


def log(msg):
    print(msg, flush=True)


def cmd_train(args):
    torch.manual_seed(0)
    t0 = time.time()
    feat, tv, tl = warmstart.make_training_set(args.n_train, F, T, M, N, args.fit_iters, seed0=0, log=log)
    log("training set: %d sequences in %.1f s" % (feat.shape[0], time.time() - t0))
    net = ConvNet(M=M, N=N, C=args.channels, L=args.layers, seed=args.seed)
    log("network: %d parameters (C=%d, L=%d)" % (net.n_params(), args.channels, args.layers))
    # time a few steps to size the run to the budget
    t1 = time.time()
    warmstart.train(net, feat, tv, tl, steps=5, batch=args.batch, lr=1e-4, log=None)
    torch.cuda.synchronize()
    per_step = (time.time() - t1) / 5
    steps = max(10, int(args.minutes * 60 / per_step)) if args.steps <= 0 else args.steps
    log("%.2f ms per step; running %d steps" % (per_step * 1e3, steps))
    net = ConvNet(M=M, N=N, C=args.channels, L=args.layers, seed=args.seed)
    hist = warmstart.train(net, feat, tv, tl, steps=steps, batch=args.batch, lr=args.lr, log=log,
                           log_every=max(1, steps // 40))
    net.save(args.out)
    log(json.dumps({"trained": args.out, "steps": steps, "ms_per_step": per_step * 1e3,
                    "loss_first": hist[0][1], "loss_last": hist[-1][1], "n_params": net.n_params(),
                    "n_train_mixtures": args.n_train, "fit_iters": args.fit_iters}))


def _iters_to(trace, target):
    idx = np.nonzero(trace >= target)[0]
    return int(idx[0]) + 1 if len(idx) else None


def _time_em(ctx, k, reps=3):
    s = torch.cuda.current_stream()
    best = 1e30
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        ctx.em_step(k)
        b.record(s)
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def _med(res, key):
    a = np.array([r[key] if r[key] is not None else np.nan for r in res], float)
    return float(np.nanmedian(a)) if np.isfinite(a).any() else None


def cmd_eval(args):
    summary = evaluate(args.weights, args.n_eval, args.conv_iters, args.batch, args.out)
    return summary


def evaluate(weights, n_eval, conv_iters, batch, out=""):
    """Run the evaluation arms on n_eval held-out mixtures; returns the summary dict."""
    args = argparse.Namespace(weights=weights, n_eval=n_eval, conv_iters=conv_iters, batch=batch, out=out)
    net = ConvNet.load(args.weights)
    res = []
    t0 = time.time()
    # per-iteration cost and warm-start overhead, measured on one mixture
    x = synth_mixture(F, T, M, N, seed=10**6)
    ctx = FastFCA(x, N, seed=1)
    ctx.em_step(10)
    t10 = _time_em(ctx, 10)
    t110 = _time_em(ctx, 110)
    t_iter = (t110 - t10) / 100.0
    t_fixed = t10 - 10 * t_iter
    ctx.close()
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        a.record(s)
        warmstart.warm_init(net, x)
        b.record(s)
        b.synchronize()
    t_ws = a.elapsed_time(b)
    log("EM %.4f ms/iteration + %.4f ms per call; warm start (features + network) %.3f ms" % (t_iter, t_fixed, t_ws))
    B = args.batch
    for a0 in range(0, args.n_eval, B):
        ids = list(range(a0, min(args.n_eval, a0 + B)))
        xs = [synth_mixture(F, T, M, N, seed=10**6 + i) for i in ids]
        # (a) plain: seeded init
        plain = FastFCA.from_batch([dict(x=x, N=N) for x in xs], seed=10**6 + a0)
        ll_plain0 = [plain.loglik(b) for b in range(len(xs))]
        p_init = [plain.get_params(b) for b in range(len(xs))]
        plain.em_step(args.conv_iters)
        tr_plain = [plain.ll_trace(b) for b in range(len(xs))]
        # (d) a perfect network: the plain fit's own targets fed back through
        # the warm-start path (an upper bound on what the network can gain)
        probs_p, lam_perfect = [], []
        for b, x in enumerate(xs):
            P, lam, v = plain.get_params(b)
            P0, _ = warmstart.features(x)
            tv, tl = warmstart.targets(P, lam, v, P0)
            lam_p, v_p = warmstart.apply_outputs(tv, tl.view(F, N, M), M)
            probs_p.append(dict(x=x, N=N, P0=P0, lam0=lam_p, v0=v_p))
            lam_perfect.append(lam_p)
        plain.close()
        perfect = FastFCA.from_batch(probs_p)
        perfect.em_step(args.conv_iters)
        tr_perf = [perfect.ll_trace(b) for b in range(len(xs))]
        perfect.close()
        # (b) warm start, (c) whitening only
        probs_w, probs_h, judged = [], [], []
        for b, x in enumerate(xs):
            P0, lam, v = warmstart.warm_init(net, x)
            probs_w.append(dict(x=x, N=N, P0=P0, lam0=lam, v0=v))
            _, feat = None, None
            pw = (torch.abs(torch.einsum("frm,ftr->ftm", P0.conj().to(torch.complex64), x)) ** 2)
            vh = (pw.mean(dim=2, keepdim=True) / N).repeat(1, 1, N).contiguous().float()
            probs_h.append(dict(x=x, N=N, P0=P0, lam0=torch.ones((F, N, M), device=x.device), v0=vh))
        warm = FastFCA.from_batch(probs_w)
        ll_warm0 = [warm.loglik(b) for b in range(len(xs))]
        for b in range(len(xs)):
            ok = np.isfinite(ll_warm0[b]) and ll_warm0[b] >= ll_plain0[b]
            judged.append(ok)
            if not ok:  # fallback: the seeded start
                warm.set_params(*p_init[b], b=b)
        warm.em_step(args.conv_iters)
        tr_warm = [warm.ll_trace(b) for b in range(len(xs))]
        warm.close()
        heur = FastFCA.from_batch(probs_h)
        heur.em_step(args.conv_iters)
        tr_heur = [heur.ll_trace(b) for b in range(len(xs))]
        heur.close()
        # (e) perfect lambda with the power-based v, (f) network lambda with the power-based v
        pl = FastFCA.from_batch([dict(ph, lam0=lp) for ph, lp in zip(probs_h, lam_perfect)])
        pl.em_step(args.conv_iters)
        tr_pl = [pl.ll_trace(b) for b in range(len(xs))]
        pl.close()
        nl = FastFCA.from_batch([dict(ph, lam0=pw["lam0"]) for ph, pw in zip(probs_h, probs_w)])
        nl.em_step(args.conv_iters)
        tr_nl = [nl.ll_trace(b) for b in range(len(xs))]
        nl.close()
        for b, i in enumerate(ids):
            llstar = float(tr_plain[b][-1])
            kp = _iters_to(tr_plain[b], llstar - TOL)
            kw = _iters_to(tr_warm[b], llstar - TOL)
            kh = _iters_to(tr_heur[b], llstar - TOL)
            kpf = _iters_to(tr_perf[b], llstar - TOL)
            res.append(dict(id=i, ll_star=llstar, ll_warm_final=float(tr_warm[b][-1]), k_plain=kp, k_warm=kw,
                            k_heur=kh, k_perfect=kpf, k_perfect_lam=_iters_to(tr_pl[b], llstar - TOL),
                            k_net_lam=_iters_to(tr_nl[b], llstar - TOL), warm_used=bool(judged[b]),
                            ll0_plain=ll_plain0[b], ll0_warm=ll_warm0[b]))
        log("eval %d/%d mixtures (%.1f s)" % (len(res), args.n_eval, time.time() - t0))

    def wall(k, extra=0.0):
        return None if k is None else t_fixed + k * t_iter + extra

    kp = np.array([r["k_plain"] for r in res], float)
    kw = np.array([r["k_warm"] if r["k_warm"] is not None else np.nan for r in res], float)
    kh = np.array([r["k_heur"] if r["k_heur"] is not None else np.nan for r in res], float)
    kpf = np.array([r["k_perfect"] if r["k_perfect"] is not None else np.nan for r in res], float)
    wp = np.array([wall(r["k_plain"]) for r in res], float)
    ww = np.array([wall(r["k_warm"], t_ws) if r["k_warm"] is not None else np.nan for r in res], float)
    summary = {
        "n_eval": len(res), "tol_nats_per_bin": TOL, "conv_iters": args.conv_iters,
        "em_ms_per_iter": t_iter, "em_ms_per_call": t_fixed, "warmstart_ms": t_ws,
        "plain_iters_median": float(np.nanmedian(kp)), "warm_iters_median": float(np.nanmedian(kw)),
        "heur_iters_median": float(np.nanmedian(kh)) if np.isfinite(kh).any() else None,
        "perfect_net_iters_median": float(np.nanmedian(kpf)) if np.isfinite(kpf).any() else None,
        "perfect_lambda_power_v_iters_median": _med(res, "k_perfect_lam"),
        "net_lambda_power_v_iters_median": _med(res, "k_net_lam"),
        "plain_ms_median": float(np.nanmedian(wp)), "warm_ms_median": float(np.nanmedian(ww)),
        "warm_reached_frac": float(np.isfinite(kw).mean()), "heur_reached_frac": float(np.isfinite(kh).mean()),
        "warm_faster_frac": float(np.nanmean(np.where(np.isfinite(ww), ww < wp, False))),
        "warm_used_frac": float(np.mean([r["warm_used"] for r in res])),
        "ll_warm_minus_star_median": float(np.median([r["ll_warm_final"] - r["ll_star"] for r in res])),
    }
    log(json.dumps(summary))
    if args.out:
        with open(args.out, "w") as fh:
            json.dump({"summary": summary, "per_mixture": res}, fh)
    return summary


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", required=True)
    t.add_argument("--n-train", type=int, default=2048)
    t.add_argument("--fit-iters", type=int, default=1000)
    t.add_argument("--minutes", type=float, default=8.0)
    t.add_argument("--steps", type=int, default=0)
    t.add_argument("--batch", type=int, default=256)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--channels", type=int, default=64)
    t.add_argument("--layers", type=int, default=6)
    t.add_argument("--seed", type=int, default=0)
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--n-eval", type=int, default=512)
    e.add_argument("--conv-iters", type=int, default=1500)
    e.add_argument("--batch", type=int, default=32)
    e.add_argument("--out", default="")
    args = ap.parse_args(argv)
    {"train": cmd_train, "eval": cmd_eval}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())

"""Train and evaluate the learned warm start on synthetic mixtures.

  python -m paper_2101_08563_amd.train_warmstart train --out W.npz [--n-train 2048 --fit-iters 1000
         --minutes 8 --batch 256]
  python -m paper_2101_08563_amd.train_warmstart train-stream --out W.npz [--n-train 20000 --chunk 64
         --epochs 1 --minutes 14 --batch 256 --channels 64 --layers 8]
  python -m paper_2101_08563_amd.train_warmstart eval --weights W.npz [--n-eval 512 --conv-iters 1500]

Workload: M=2 microphones, N=3 sources, F=513 bins, T=1000 frames (the paper's
STFT shape), mixtures drawn on the GPU by fastfca_synth_mixture. Training
mixtures use seeds 0..n_train-1, evaluation mixtures seeds 10^6 + i.

Targets: the IP+EM fit of each training mixture after --fit-iters iterations
from the library's seeded initialization, trace-normalized and expressed in
the whitened basis P0 = C_f^{-1/2} (fastfca_ws_targets).

Evaluation (per held-out mixture, measure()): LL* = the plain fit's
log-likelihood per bin after --conv-iters iterations from the library's
seeded start; iterations to LL* - 1e-2 from (a) the seeded start, (b)
fastfca_warmstart with the network, (c) fastfca_warmstart without it (the
whitening-only start), and, as a bound, (d) the plain fit's own targets fed
back through the warm-start path (a perfect network). The library's
fastfca_warmstart judges every start per frequency by its log-likelihood and
keeps the seeded start where the new one is worse. Wall times of (a) and
(b) are measured end to end with HIP events.
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


def cmd_train_stream(args):
    """Training at the full size: n_train mixtures regenerated chunk by chunk
    from their seeds, targets from converged fits (LL gain < 1e-7 nats/bin per
    iteration, at most 2000 iterations)."""
    torch.manual_seed(0)
    net = ConvNet(M=M, N=N, C=args.channels, L=args.layers, seed=args.seed)
    log("network: %d parameters (C=%d, L=%d)" % (net.n_params(), args.channels, args.layers))
    t0 = time.time()
    r = warmstart.train_stream(net, args.n_train, F, T, M, N, chunk=args.chunk, epochs=args.epochs,
                               steps_per_chunk=args.steps_per_chunk, minutes=args.minutes, batch=args.batch,
                               lr=args.lr, log=log, log_every=max(1, args.n_train // args.chunk // 40))
    hist, fits = r["history"], r["fit_iters"]
    meta = dict(n_train_mixtures=args.n_train, chunk=args.chunk, epochs=args.epochs, chunks_skipped=r["skipped"],
                steps=hist[-1][0], steps_per_chunk=r["steps_per_chunk"], batch=args.batch, lr=args.lr,
                n_params=net.n_params(), channels=args.channels, layers=args.layers,
                fit_rule="IP+EM from the seeded start until the LL gain per iteration < 1e-7 nats/bin "
                         "for every mixture of the chunk, at most 2000 iterations",
                fit_iters_median=float(np.median(fits)), fit_iters_max=int(np.max(fits)),
                loss_first=hist[0][1], loss_last=hist[-1][1], train_seconds=round(time.time() - t0, 1),
                workload="M=%d N=%d F=%d T=%d, rank 8, diffuse 0.05, seeds 0..%d" % (M, N, F, T, args.n_train - 1))
    net.save(args.out, meta=meta)
    log(json.dumps(dict(trained=args.out, **meta)))


def _iters_to(trace, target):
    idx = np.nonzero(trace >= target)[0]
    return int(idx[0]) + 1 if len(idx) else None


def cmd_eval(args):
    summary, rows = measure(args.weights, args.n_eval, args.conv_iters, log=log, race_iters=args.race_iters,
                            race_iters_white=args.race_iters_white)
    log(json.dumps(summary))
    if args.out:
        with open(args.out, "w") as fh:
            json.dump({"summary": summary, "per_mixture": rows}, fh)
    return summary


def _timed(stream, fn, reps=3):
    """Median over reps of the event time (ms) of fn() on stream."""
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def measure(weights, n_eval=64, conv_iters=1500, seed0=10**6, log=None, race_iters=100, race_iters_white=150):
    """Measured time to converge on n_eval held-out mixtures (seeds seed0 + i,
    disjoint from the training seeds), one single-mixture context each.

    LL* is the plain fit's log-likelihood per bin after conv_iters iterations
    from the library's seeded start; k_plain, k_warm, k_heur are the
    iterations to LL* - TOL from the seeded start, from fastfca_warmstart with
    the network, and from fastfca_warmstart without it (whitening only). The
    wall times are measured end to end with HIP events on the context's
    stream, each the median of three repetitions from the same start:
      plain  em_step(k_plain)
      warm   fastfca_warmstart(net) (features, network, judge) + em_step(k_warm)
    (the graph of each em_step length is captured before its timed runs).
    Also reported: the log-likelihood after the first iteration from either
    start, and how far the warm fit ends above or below LL* after
    conv_iters iterations (a different local optimum shows there); and the
    race judge (fastfca_warmstart_race): the seeded start and the network's
    (race) or the whitening-only start (race_white) run race_iters
    iterations side by side, each frequency keeps the better, and the plain
    iteration continues; its iterations count the race's, its wall time is
      race   fastfca_warmstart_race(net, K) + em_step(k_after)."""
    net = ConvNet.load(weights)
    stream = torch.cuda.current_stream()
    rows = []
    t0 = time.time()
    for i in range(n_eval):
        x = synth_mixture(F, T, M, N, seed=seed0 + i)
        ctx = FastFCA(x, N, seed=seed0 + i)
        P0, l0, v0 = (a.clone() for a in ctx.get_params())

        def restart():
            ctx.set_params(P0, l0, v0)

        ctx.em_step(conv_iters)
        tr_p = ctx.ll_trace()
        llstar = float(tr_p[-1])
        target = llstar - TOL
        kp = _iters_to(tr_p, target)
        restart()
        taken = ctx.warmstart(net, count=True)
        ctx.em_step(conv_iters)
        tr_w = ctx.ll_trace()
        kw = _iters_to(tr_w, target)
        restart()
        ctx.warmstart(None)
        ctx.em_step(conv_iters)
        kh = _iters_to(ctx.ll_trace(), target)
        # a perfect network: the plain fit's own targets through the same path
        restart()
        ctx.em_step(conv_iters)
        Pf, lf, vf = ctx.get_params()
        Pw, _ = warmstart.features(x)
        tv, tl = warmstart.targets(Pf, lf, vf, Pw)
        lam_p, v_p = warmstart.apply_outputs(tv, tl.view(F, N, M), M)
        ctx.set_params(Pw, lam_p, v_p)
        ctx.em_step(conv_iters)
        kpf = _iters_to(ctx.ll_trace(), target)
        # the race judge: both starts run race_iters iterations, each
        # frequency keeps the better, then the plain iteration continues
        race = {}
        for arm, rnet, K in (("race", net, race_iters), ("race_white", None, race_iters_white)):
            restart()
            kept = ctx.warmstart_race(rnet, K, count=True)
            ctx.em_step(conv_iters)
            ka = _iters_to(ctx.ll_trace(), target)
            race[arm] = (K + ka if ka is not None else None, kept, ka)
        # timed runs
        ctx.em_step(kp)
        ts = []
        for _ in range(3):
            restart()
            ts.append(_timed(stream, lambda: ctx.em_step(kp), reps=1))
        t_plain = float(np.median(ts))
        t_warm = t_ws = None
        if kw is not None:
            ctx.em_step(kw)
            tw, tws = [], []
            for _ in range(3):
                restart()
                tws.append(_timed(stream, lambda: ctx.warmstart(net), reps=1))
                restart()
                tw.append(_timed(stream, lambda: (ctx.warmstart(net), ctx.em_step(kw)), reps=1))
            t_warm, t_ws = float(np.median(tw)), float(np.median(tws))
        for arm, rnet, K in (("race", net, race_iters), ("race_white", None, race_iters_white)):
            kr, kept, ka = race[arm]
            t_r = None
            if ka is not None:
                restart()
                ctx.warmstart_race(rnet, K)
                ctx.em_step(ka)
                tr_ = []
                for _ in range(3):
                    restart()
                    tr_.append(_timed(stream, lambda: (ctx.warmstart_race(rnet, K), ctx.em_step(ka)), reps=1))
                t_r = float(np.median(tr_))
            race[arm] = (kr, kept, t_r)
        ctx.close()
        rows.append(dict(id=seed0 + i, k_race=race["race"][0], kept_race=race["race"][1], ms_race=race["race"][2],
                         k_race_white=race["race_white"][0], kept_race_white=race["race_white"][1],
                         ms_race_white=race["race_white"][2],
                         ll_star=llstar, ll_first_plain=float(tr_p[0]), ll_first_warm=float(tr_w[0]),
                         ll_end_warm_minus_star=float(tr_w[-1]) - llstar,
                         k_plain=kp, k_warm=kw, k_heur=kh, k_perfect=kpf,
                         taken=taken, ms_plain=t_plain, ms_warm=t_warm, ms_warmstart=t_ws))
        if log and (i + 1) % 16 == 0:
            log("measured %d/%d mixtures (%.1f s)" % (i + 1, n_eval, time.time() - t0))

    def med(key):
        a = np.array([r[key] if r[key] is not None else np.nan for r in rows], float)
        return float(np.nanmedian(a)) if np.isfinite(a).any() else None

    wp = np.array([r["ms_plain"] for r in rows], float)
    ww = np.array([r["ms_warm"] if r["ms_warm"] is not None else np.inf for r in rows], float)
    summary = {"mixtures": n_eval, "tol_nats_per_bin": TOL, "reference_iters": conv_iters,
               "measured": "HIP events, end to end",
               "plain_ms_median": med("ms_plain"), "warm_ms_median": float(np.median(ww)),
               "warmstart_call_ms_median": med("ms_warmstart"),
               "plain_iters_median": med("k_plain"), "warm_iters_median": med("k_warm"),
               "whitening_only_iters_median": med("k_heur"), "perfect_net_iters_median": med("k_perfect"),
               "warm_faster_frac": float(np.mean(ww < wp)),
               "warm_reached_frac": float(np.mean([r["k_warm"] is not None for r in rows])),
               "frequencies_kept_median": med("taken"),
               "ll_first_iter_plain_median": med("ll_first_plain"), "ll_first_iter_warm_median": med("ll_first_warm"),
               "ll_end_warm_minus_star_median": med("ll_end_warm_minus_star")}
    wr = np.array([r["ms_race"] if r["ms_race"] is not None else np.inf for r in rows], float)
    wrw = np.array([r["ms_race_white"] if r["ms_race_white"] is not None else np.inf for r in rows], float)
    summary.update({"race_iters": race_iters, "race_iters_white": race_iters_white,
                    "race_ms_median": float(np.median(wr)), "race_total_iters_median": med("k_race"),
                    "race_kept_median": med("kept_race"), "race_faster_frac": float(np.mean(wr < wp)),
                    "race_white_ms_median": float(np.median(wrw)), "race_white_total_iters_median": med("k_race_white"),
                    "race_white_kept_median": med("kept_race_white"), "race_white_faster_frac": float(np.mean(wrw < wp))})
    return summary, rows


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
    ts = sub.add_parser("train-stream")
    ts.add_argument("--out", required=True)
    ts.add_argument("--n-train", type=int, default=20000)
    ts.add_argument("--chunk", type=int, default=64)
    ts.add_argument("--epochs", type=int, default=1)
    ts.add_argument("--steps-per-chunk", type=int, default=0)
    ts.add_argument("--minutes", type=float, default=14.0)
    ts.add_argument("--batch", type=int, default=256)
    ts.add_argument("--lr", type=float, default=1e-3)
    ts.add_argument("--channels", type=int, default=64)
    ts.add_argument("--layers", type=int, default=8)
    ts.add_argument("--seed", type=int, default=0)
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--n-eval", type=int, default=512)
    e.add_argument("--conv-iters", type=int, default=1500)
    e.add_argument("--out", default="")
    e.add_argument("--race-iters", type=int, default=100)
    e.add_argument("--race-iters-white", type=int, default=150)
    args = ap.parse_args(argv)
    {"train": cmd_train, "train-stream": cmd_train_stream, "eval": cmd_eval}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())

"""Benchmark of the FastFCA hot path on one MI355X.

One step = one pass of the whole path over the headline workload (M=2 mics,
N=3 sources, F=513 bins, T=1000 frames; synthetic mixture drawn by
paper_2101_08563_amd.synth): set the initial parameters (Algorithm 1,
initialize), 100 IP+EM iterations with the per-iteration log-likelihood
(Algorithm 1, eq:negll), and the multichannel Wiener filter (eq:Doclo).
Inputs are resident in HBM before timing starts.

Metric: EM TF-bin*source updates per second = F*T*N*iterations / step time.

Prints ONE JSON line. Besides the contract fields it carries:
  roofline         the EM kernel's ALU roofline: algorithmic flops per launch
                   (flops_per_bin) over its event-timed duration against the
                   published 157.3 TFLOP/s FP32 peak; beside it the kernel's
                   own operation count against the one-FMA-per-lane rate and
                   the HBM streaming-equivalent fractions, and the bandwidth
                   of a plain 1 GiB device copy on the same box
  cpu_baseline     the FP64 oracle on all host cores and on one core
  time_to_converge plain vs warm start, measured end to end (HIP events)
  extra            the batch32, 256-mixture batch and large-array lines
Options: --gpus N (only 1 is supported), --steps K, --warmup W, --iters I,
  --no-cpu, --no-ttc, --no-extra, --ttc-mixtures K, --workload W (one line
  for another workload), --calib-copy MiB (also run a plain device copy of
  that size, used to scale rocprofv3 byte counters).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X figures used for the roofline (per-unit derivations in the design doc).
CU, SIMD_PER_CU, LANES, CLOCK_HZ = 256, 4, 16, 2.4e9
FP32_PEAK = 157.3e12                                         # published FP32 vector peak (packed FMA)
FP32_FMA_NONPACKED = CU * SIMD_PER_CU * LANES * 2 * CLOCK_HZ # 78.6 TFLOP/s, one FMA per lane per clock
HBM_PEAK = 8.0e12                                            # bytes/s


def flops_per_bin(M: int, N: int) -> int:
    """Algorithmic flops per TF bin per IP+EM iteration, counted from the
    method's definitions: the M weighted covariances of eq:wsampcov as
    M(M+1)/2 Hermitian entries at (6 + 4M) flops each, U = |P^H x|^2 by
    eq:Udef (8M^2), the N posterior updates of Algorithm 1 (15 MN) and the
    log-likelihood terms of eq:negll (6M): 176 at (M, N) = (2, 3), 732 at
    (4, 6), 3128 at (8, 10)."""
    return M * (M + 1) // 2 * (6 + 4 * M) + 8 * M * M + 15 * M * N + 6 * M


def kernel_ops_per_bin(M: int, N: int, algo: str = "em") -> int:
    """Floating point operations per bin per iteration as the resident
    kernel issues them (FMA = 2): sigma^2 and its inverse (2MN + M), x x^H as
    M^2 real parameters (3M^2), the M weighted covariances (2M^3), U
    (8M^2 + 3M), the log-likelihood terms (4M), and the L/H update: for
    IP+EM the N sequential source updates (N (2MN + 12M + 2)); for IP+MM the
    L-rule sums (2MN + 3M + 4NM) and the H rule (2MN + 3M + 4NM + 3N)."""
    common = (2 * M * N + M) + 3 * M * M + 2 * M ** 3 + (8 * M * M + 3 * M) + 4 * M
    if algo == "mm":
        return common + 2 * (2 * M * N + 3 * M + 4 * N * M) + 3 * N
    return common + N * (2 * M * N + 12 * M + 2)


def em_bytes_per_bin(M: int, N: int) -> int:
    """HBM bytes per TF bin of one streaming pass (x read, v read and written): 8M + 8N."""
    return 8 * M + 8 * N


def hbm_fracs(bins_by_shape, iters, seconds):
    """Fractions of the HBM roofline: the updates/s achieved over the
    updates/s of a design streaming 8M + 8N bytes per bin per iteration at
    8 TB/s (x read once) and 16M + 8N (x read twice)."""
    once = sum(b * (8 * M + 8 * N) for (M, N), b in bins_by_shape.items()) * iters
    twice = sum(b * (16 * M + 8 * N) for (M, N), b in bins_by_shape.items()) * iters
    return once / seconds / HBM_PEAK, twice / seconds / HBM_PEAK


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


KERNEL_FILES = ["em_item.hpp", "em_kernel.hip", "device.hpp", "internal.hpp", "ip_sm.hpp", "ip_common.hpp"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_FILES:
        with open(os.path.join(ROOT, "paper_2101_08563_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per em_kernel launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy), or None when
    the kernel sources have changed since the counters were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", "em_kernel_c1_traffic.json")) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("source_sha256_16") != kernel_source_hash():
        return None
    return d.get("traffic_bytes_per_launch")


def roofline_alu(kernel, flops_8d, ops_kernel, seconds, bins_by_shape, iters, traffic=None):
    """The ALU roofline object: achieved = algorithmic flops (flops_per_bin)
    per launch over the measured time, against the published FP32 peak; the
    kernel's own operation count against the one-FMA-per-lane rate and the
    HBM streaming-equivalent fractions are reported beside it."""
    ach = flops_8d / seconds
    once, twice = hbm_fracs(bins_by_shape, iters, seconds)
    return {"kernel": kernel, "bound": "alu", "achieved": ach / 1e12, "peak": FP32_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": ach / FP32_PEAK, "traffic": traffic,
            "flops_per_launch": flops_8d,
            "kernel_ops_per_launch": ops_kernel,
            "kernel_ops_frac_of_nonpacked_fp32": ops_kernel / seconds / FP32_FMA_NONPACKED,
            "hbm_streaming_equivalent_frac_x_once": once,
            "hbm_streaming_equivalent_frac_x_twice": twice}


def calib_copy(mib):
    """Three plain device copies of mib MiB (the reference for scaling the
    rocprofv3 byte counters); returns the bytes one copy moves."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return 2 * n * 4


def copy_bandwidth(mib=1024, reps=10):
    """HBM bandwidth of a plain device-to-device copy of mib MiB on this machine,
    timed with HIP events on the current stream: bytes read plus bytes
    written per second, in GB/s. A reference for the kernels' roofline
    fractions (what a pure streaming kernel reaches here against the 8 TB/s
    peak)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        b.copy_(a)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * n * 4 / (ms * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ttc", action="store_true", help="skip the time-to-converge comparison")
    ap.add_argument("--no-extra", action="store_true", help="skip the batch and large-array workloads")
    ap.add_argument("--ttc-mixtures", type=int, default=64)
    ap.add_argument("--algo", choices=["em", "mm"], default="em",
                    help="headline update: Algorithm 1 (IP+EM, the contract line) or Algorithm 2 (IP+MM)")
    ap.add_argument("--calib-copy", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--bpt", type=int, default=0)
    ap.add_argument("--workload", choices=["headline", "batch", "batch32", "large", "blocks", "mnmf"],
                    default="headline",
                    help="headline: the contract line (M=2 N=3 F=513 T=1000), with the batch32, batch "
                         "and large lines under 'extra'; batch: 256 mixed mixtures against sequential runs; "
                         "large: M=8 N=10 F=1025 T=4000; batch32: 32 headline-shaped mixtures in one context; "
                         "blocks: the piecewise stationary model on the headline mixture (B=4); mnmf: "
                         "FastMNMF on the headline mixture (K=8)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build measures the single-GPU kernel "
              "(frequencies shard across GPUs with no exchange; see the design notes). "
              "--gpus %d is not supported." % args.gpus, file=sys.stderr)
        sys.exit(2)

    single = {"batch": bench_batch, "large": bench_large, "batch32": bench_batch32, "blocks": bench_blocks,
              "mnmf": bench_mnmf}
    if args.workload in single:
        out = single[args.workload](args)
        if args.calib_copy:
            out["calib_copy_bytes"] = calib_copy(args.calib_copy)
        print(json.dumps(out))
        return

    import torch

    from paper_2101_08563_amd import FastFCA, synth

    cfg = synth.CONFIGS["c1"]
    F, T, M, N = cfg["F"], cfg["T"], cfg["M"], cfg["N"]
    iters = args.iters
    x = synth.mixture(F=F, T=T, M=M, N=N, rank=cfg["rank"], diffuse=cfg["diffuse"],
                      config_id=cfg["config_id"])
    P0, lam0, v0 = synth.init_params(x, N, config_id=cfg["config_id"])

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        xd = torch.from_numpy(x).to(dev)
        Pd = torch.from_numpy(P0).to(dev)
        ld = torch.from_numpy(lam0).to(dev)
        vd = torch.from_numpy(v0).to(dev)
        y = torch.empty((N, F, T, M), dtype=torch.complex64, device=dev)
    stream.synchronize()
    ctx = FastFCA(xd, N, Pd, ld, vd, stream=stream)
    if args.algo == "mm":
        ctx.set_algorithm("mm")
    if args.threads:
        ctx.set_config(args.threads, args.bpt)
    threads, bpt = ctx.get_config()

    def step(ev=None):
        ctx.set_params(Pd, ld, vd)
        if ev is not None:
            ev[0].record(stream)
        ctx.em_step(iters)
        if ev is not None:
            ev[1].record(stream)
        ctx.mwf(out=y)

    for _ in range(args.warmup):
        step()
    ctx.sync()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.sync()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    em_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    trace = ctx.ll_trace()
    ll = ctx.loglik()
    assert np.isfinite(ll) and len(trace) == iters

    updates = F * T * N * iters
    value = updates / (ms_per_step * 1e-3)
    out = {
        "metric": "EM TF-bin*source updates/s",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "FastFCA IP+%s x%d + MWF, M=%d N=%d F=%d T=%d" % (args.algo.upper(), iters, M, N, F, T),
                   "M": M, "N": N, "F": F, "T": T, "iters": iters, "threads": threads,
                   "bins_per_thread": bpt, "ll_per_bin": ll},
        "roofline": roofline_alu("em_kernel<%d,%d,%d> (IP+%s, state resident on chip); timed per em_step call: one "
                                 "launch over the first F - r frequencies and, when F leaves a small remainder r over "
                                 "the CUs, the last r in consecutive launches on a side stream (the tail split)"
                                 % (M, N, bpt, args.algo.upper()),
                                 flops_per_bin(M, N) * F * T * iters, kernel_ops_per_bin(M, N, args.algo) * F * T * iters,
                                 em_ms * 1e-3, {(M, N): F * T}, iters,
                                 traffic=measured_traffic() if (iters == 100 and args.algo == "em") else None),
    }
    out["roofline"]["em_ms_per_call"] = em_ms
    out["roofline"]["hbm_algorithmic_bytes_per_launch"] = em_bytes_per_bin(M, N) * F * T
    out["roofline"]["copy_kernel_GBps"] = copy_bandwidth()
    if args.calib_copy:
        out["calib_copy_bytes"] = calib_copy(args.calib_copy)

    if not args.no_cpu:
        import oracle
        cores = oracle.num_threads()
        t2 = time.perf_counter()
        Po, lo, vo, _ = oracle.fit(x, P0, lam0, v0, iters, nthreads=cores)
        oracle.mwf(x, Po, lo, vo)
        t3 = time.perf_counter()
        # one core: the first 32 frequencies of the same workload
        F1 = 32
        t4 = time.perf_counter()
        oracle.fit(x[:F1], P0[:F1], lam0[:F1], v0[:F1], iters, nthreads=1)
        t5 = time.perf_counter()
        oracle.fit(x[:1], P0[:1], lam0[:1], v0[:1], 1, nthreads=cores)  # back to every core
        out["cpu_baseline"] = {
            "value": updates / (t3 - t2),
            "unit": "updates/s",
            "cores": cores,
            "kind": "oracle",
            "sample": "full workload: F=%d T=%d M=%d N=%d, %d IP+EM iterations + MWF, FP64 C, OpenMP over "
                      "frequencies, %.2f s" % (F, T, M, N, iters, t3 - t2),
            "cpu_model": cpu_model(),
            "host_cpus": {"logical": os.cpu_count(), "usable": len(os.sched_getaffinity(0))},
            "one_core": {"value": F1 * T * N * iters / (t5 - t4), "unit": "updates/s", "cores": 1,
                         "sample": "F=%d of %d frequencies, %d IP+EM iterations, %.2f s" % (F1, F, iters, t5 - t4)},
        }
    ctx.close()
    if not args.no_ttc:
        out["time_to_converge"] = time_to_converge(args.ttc_mixtures)
    if not args.no_extra:
        sub = argparse.Namespace(**vars(args))
        sub.iters = 100
        sub.no_cpu = True
        out["extra"] = {}
        for name, fn in (("batch32", bench_batch32), ("batch256", bench_batch), ("large", bench_large)):
            try:
                r = fn(sub)
                out["extra"][name] = {k: r[k] for k in ("value", "unit", "ms_per_step")}
                out["extra"][name]["workload"] = r["config"]["workload"]
                out["extra"][name]["roofline"] = r["roofline"]
            except Exception as e:  # reported, not hidden
                out["extra"][name] = {"error": "%s: %s" % (type(e).__name__, e)}
    print(json.dumps(out))


def time_to_converge(n_eval=64, conv_iters=1500):
    """Second half of the metric, measured end to end: wall time for plain
    IP+EM and for the warm starts to reach the plain fit's log-likelihood
    after conv_iters iterations minus 1e-2 nats/bin, medians over n_eval
    held-out headline-shaped mixtures (paper_2101_08563_amd.train_warmstart.
    measure): fastfca_warmstart (features, network, judge by the starting
    likelihood) then IP+EM; and fastfca_warmstart_race (the network's start,
    or the whitening-only one, raced against the seeded start, each
    frequency keeping the better) then IP+EM."""
    import contextlib

    weights = os.path.join(ROOT, "paper_2101_08563_amd", "data", "warmstart_c32l4.npz")
    try:
        from paper_2101_08563_amd import train_warmstart
        with contextlib.redirect_stdout(sys.stderr):
            s, _ = train_warmstart.measure(weights, n_eval=n_eval, conv_iters=conv_iters)
    except Exception as e:  # reported, not hidden: the line still carries the throughput
        return {"error": "%s: %s" % (type(e).__name__, e)}
    return s


def _time(fn, stream, reps):
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def _line(value, ms, reps, workload, roofline, **config):
    return {"metric": "EM TF-bin*source updates/s", "value": value, "unit": "updates/s", "n_gpus": 1,
            "steps": reps, "warmup": 1, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": dict(workload=workload, **config),
            "roofline": roofline}


def bench_batch(args):
    """256 mixtures with T ~ U{200..2000}, M in {2,3,4}, N in {M+1, M+2}, F=513,
    drawn on the GPU; the autotuned schedule (class launches or one
    persistent launch) per em_step call, against the same mixtures run one
    context at a time."""
    import torch

    from paper_2101_08563_amd import FastFCA, synth
    from paper_2101_08563_amd.fastfca import synth_mixture

    specs = synth.batch_specs(B=256, F=513)
    iters = args.iters
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        xs = [synth_mixture(s["F"], s["T"], s["M"], s["N"], rank=8, diffuse=0.05, seed=2000 + i, stream=stream)
              for i, s in enumerate(specs)]
    stream.synchronize()
    probs = [dict(x=x, N=s["N"]) for x, s in zip(xs, specs)]
    batch = FastFCA.from_batch(probs, seed=1, stream=stream)
    # schedule (class launches or persistent queue), shape and grid; the state is restored
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        cache = os.path.join(td, "tune.jsonl")
        batch.autotune(n_iter=10, cache_path=cache)
        with open(cache) as fh:
            tune = json.loads(fh.read().splitlines()[-1])
    batch.em_step(2)
    batch.sync()
    reps = max(2, args.steps // 5)
    t_batch = _time(lambda: batch.em_step(iters), stream, reps)
    batch.sync()
    batch.close()
    singles = [FastFCA(x, s["N"], seed=1 + i, stream=stream) for i, (x, s) in enumerate(zip(xs, specs))]
    for c in singles:
        c.em_step(2)
    stream.synchronize()

    def run_all():
        for c in singles:
            c.em_step(iters)

    t_seq = _time(run_all, stream, 2)
    for c in singles:
        c.close()
    updates = sum(s["F"] * s["T"] * s["N"] for s in specs) * iters
    bins = sum(s["F"] * s["T"] for s in specs)
    shapes = {}
    for s in specs:
        shapes[(s["M"], s["N"])] = shapes.get((s["M"], s["N"]), 0) + s["F"] * s["T"]
    fl = sum(b * flops_per_bin(M, N) for (M, N), b in shapes.items()) * iters
    ops = sum(b * kernel_ops_per_bin(M, N) for (M, N), b in shapes.items()) * iters
    out = _line(updates / (t_batch * 1e-3), t_batch, reps,
                "batch: 256 mixtures, T~U{200..2000}, M in {2,3,4}, N in {M+1,M+2}, F=513, %d IP+EM iterations, %s"
                % (iters, "one persistent launch" if tune["persistent"] else "one launch per (M, N, T-bucket) class"),
                roofline_alu("em_persistent_kernel" if tune["persistent"] else "em_kernel class launches", fl, ops,
                             t_batch * 1e-3, shapes, iters),
                iters=iters, tf_bins=bins, autotune=tune, sequential_ms=t_seq, speedup_vs_sequential=t_seq / t_batch,
                sequential_updates_per_s=updates / (t_seq * 1e-3))
    if not args.no_cpu:
        # the oracle on a bounded sample: the first 16 mixtures, 128 frequencies each, 10 iterations
        import oracle
        from paper_2101_08563_amd import synth as _synth
        t_cpu, upd_cpu = 0.0, 0
        for i, s in enumerate(specs[:16]):
            xh = xs[i][:128].cpu().numpy()
            P0, l0, v0 = _synth.init_params(xh, s["N"], config_id=2, mixture_id=i)
            t2 = time.perf_counter()
            oracle.fit(xh, P0, l0, v0, 10)
            t_cpu += time.perf_counter() - t2
            upd_cpu += xh.shape[0] * xh.shape[1] * s["N"] * 10
        out["cpu_baseline"] = {"value": upd_cpu / t_cpu, "unit": "updates/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": "16 of 256 mixtures, 128 of 513 frequencies each, 10 iterations, %.2f s"
                                         % t_cpu}
    return out


def bench_batch32(args, B=32):
    """B mixtures of the headline shape (M=2 N=3 F=513 T=1000, different seeds)
    in one context: the same kernel as the headline line, with enough
    workgroups (B x 513) to fill the chip."""
    import torch

    from paper_2101_08563_amd import FastFCA
    from paper_2101_08563_amd.fastfca import synth_mixture

    F, T, M, N, iters = 513, 1000, 2, 3, args.iters
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        xs = [synth_mixture(F, T, M, N, rank=8, diffuse=0.05, seed=500 + i, stream=stream) for i in range(B)]
    stream.synchronize()
    ctx = FastFCA.from_batch([dict(x=x, N=N) for x in xs], seed=5, stream=stream)
    ctx.em_step(2)
    ctx.sync()
    reps = max(3, args.steps // 4)
    t = _time(lambda: ctx.em_step(iters), stream, reps)
    ctx.sync()
    threads, bpt = ctx.get_config()
    ctx.close()
    bins = B * F * T
    return _line(bins * N * iters / (t * 1e-3), t, reps,
                 "%d headline-shaped mixtures (M=2 N=3 F=513 T=1000), %d IP+EM iterations, one context" % (B, iters),
                 roofline_alu("em_kernel<2,3,%d>" % bpt, flops_per_bin(M, N) * bins * iters,
                              kernel_ops_per_bin(M, N) * bins * iters, t * 1e-3, {(M, N): bins}, iters),
                 threads=threads, bins_per_thread=bpt)


def bench_large(args):
    """M=8, N=10, F=1025, T=4000 (wide kernel family)."""
    import torch

    from paper_2101_08563_amd import FastFCA
    from paper_2101_08563_amd.fastfca import synth_mixture

    F, T, M, N, iters = 1025, 4000, 8, 10, args.iters
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        x = synth_mixture(F, T, M, N, rank=8, diffuse=0.05, seed=3, stream=stream)
    stream.synchronize()
    ctx = FastFCA(x, N, seed=3, stream=stream)
    ctx.em_step(1)
    ctx.sync()
    reps = 3
    t = _time(lambda: ctx.em_step(iters), stream, reps)
    threads, bpt = ctx.get_config()
    ll = ctx.loglik()
    cpu = None
    if not args.no_cpu:
        # the oracle on 64 of the frequencies for 2 iterations from the library's init
        import oracle
        Fs, its = 64, 2
        ctx2 = FastFCA(x[:Fs].contiguous(), N, seed=3, stream=stream)
        P0, l0, v0 = (a.cpu().numpy() for a in ctx2.get_params())
        xs = x[:Fs].cpu().numpy()
        ctx2.close()
        t2 = time.perf_counter()
        oracle.fit(xs, P0, l0, v0, its)
        t3 = time.perf_counter()
        cpu = {"value": Fs * T * N * its / (t3 - t2), "unit": "updates/s", "cores": oracle.num_threads(),
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": "F=%d of %d frequencies, %d iterations, %.2f s" % (Fs, F, its, t3 - t2)}
    ctx.close()
    bins = F * T
    out = _line(bins * N * iters / (t * 1e-3), t, reps,
                "large array: M=8 N=10 F=1025 T=4000, %d IP+EM iterations" % iters,
                roofline_alu("em_wide_kernel<8,10,%d>" % bpt, flops_per_bin(M, N) * bins * iters,
                             kernel_ops_per_bin(M, N) * bins * iters, t * 1e-3, {(M, N): bins}, iters),
                threads=threads, bins_per_thread=bpt, ll_per_bin=ll)
    if cpu:
        out["cpu_baseline"] = cpu
    return out


def _headline_mixture():
    from paper_2101_08563_amd import synth
    cfg = synth.CONFIGS["c1"]
    x = synth.mixture(F=cfg["F"], T=cfg["T"], M=cfg["M"], N=cfg["N"], rank=cfg["rank"], diffuse=cfg["diffuse"],
                      config_id=cfg["config_id"])
    return x, cfg


def bench_blocks(args, B=4):
    """Piecewise stationary model (Sec. VI) on the headline mixture, blocks of B frames."""
    import torch

    from paper_2101_08563_amd import FastFCA, synth

    x, cfg = _headline_mixture()
    F, T, M, N = x.shape[0], x.shape[1], x.shape[2], cfg["N"]
    P0, lam0, v0 = synth.init_params_blocks(x, N, B, config_id=cfg["config_id"])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        xd, Pd, ld, vd = (torch.from_numpy(a).cuda() for a in (x, P0, lam0, v0))
    stream.synchronize()
    ctx = FastFCA.from_blocks(xd, N, B, Pd, ld, vd, stream=stream)
    iters = args.iters

    def run():
        ctx.set_params(Pd, ld, vd)
        ctx.em_step(iters)

    run()
    ctx.sync()
    t = _time(run, stream, max(3, args.steps // 4))
    ctx.sync()
    ctx.close()
    J = T // B
    updates = F * J * N * iters
    # flops per block and iteration: as flops_per_bin, with Q_m taking the
    # given block covariance (M(M+1)/2 entries at 4M flops) and U a dot
    # product of its M^2 parameters (2M^3)
    fl = M * (M + 1) // 2 * 4 * M + 2 * M ** 3 + 15 * M * N + 6 * M
    out = _line(updates / (t * 1e-3), t, max(3, args.steps // 4),
                "piecewise stationary model, blocks of %d frames: M=%d N=%d F=%d T=%d (J=%d blocks), "
                "%d IP+EM iterations" % (B, M, N, F, T, J, iters),
                {"bound": "alu", "achieved": fl * F * J * iters / (t * 1e-3) / 1e12, "peak": FP32_PEAK / 1e12,
                 "unit": "TFLOP/s", "frac": fl * F * J * iters / (t * 1e-3) / FP32_PEAK, "traffic": None},
                frames_per_s=F * T * iters / (t * 1e-3))
    if not args.no_cpu:
        import oracle
        t2 = time.perf_counter()
        oracle.fit_blocks(x, B, P0, lam0, v0, iters)
        t3 = time.perf_counter()
        out["cpu_baseline"] = {"value": updates / (t3 - t2), "unit": "updates/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": "full workload, %d iterations, %.2f s" % (iters, t3 - t2)}
    return out


def bench_mnmf(args, K=8):
    """FastMNMF (NMF source powers shared over frequencies) on the headline mixture."""
    import torch

    from paper_2101_08563_amd import FastFCA, synth

    x, cfg = _headline_mixture()
    F, T, M, N = x.shape[0], x.shape[1], x.shape[2], cfg["N"]
    iters = min(args.iters, 30)
    P0, lam0, t0, v0 = synth.init_params_mnmf(x, N, K, config_id=cfg["config_id"])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        xd, Pd, ld, td, vd = (torch.from_numpy(a).cuda() for a in (x, P0, lam0, t0, v0))
    stream.synchronize()
    ctx = FastFCA.mnmf(xd, N, K, ld, td, vd, P0=Pd, stream=stream)

    def run():
        ctx.mnmf_set_params(Pd, ld, td, vd)
        ctx.em_step(iters)

    run()
    ctx.sync()
    reps = max(3, args.steps // 4)
    t = _time(run, stream, reps)
    ctx.sync()
    ll = ctx.loglik()
    ctx.close()
    updates = F * T * N * iters
    hbm = (8 * M + 16 * N) * F * T * iters   # x read; G, E written and read back, per iteration
    out = _line(updates / (t * 1e-3), t, reps,
                "FastMNMF: M=%d N=%d K=%d F=%d T=%d, %d IP+MM iterations" % (M, N, K, F, T, iters),
                {"bound": "hbm", "achieved": hbm / (t * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9,
                 "unit": "GB/s", "frac": hbm / (t * 1e-3) / HBM_PEAK, "traffic": None},
                ll_per_bin=ll, us_per_iteration=t * 1e3 / iters)
    if not args.no_cpu:
        # the oracle (single thread: the frequencies are coupled through V) on
        # the full mixture for 5 iterations
        import oracle
        Fs, its = F, 5
        t2 = time.perf_counter()
        oracle.mnmf_fit(x[:Fs], P0[:Fs], lam0[:Fs], t0[:Fs], v0, its)
        t3 = time.perf_counter()
        out["cpu_baseline"] = {"value": Fs * T * N * its / (t3 - t2), "unit": "updates/s", "cores": 1,
                               "kind": "oracle", "sample": "F=%d of %d frequencies, %d iterations, %.2f s"
                                                           % (Fs, F, its, t3 - t2)}
    return out


if __name__ == "__main__":
    main()

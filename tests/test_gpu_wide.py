"""The wide kernel family (M up to 8, N up to 12, T up to 4096; x re-read per
iteration) against the FP64 oracle, including the large-array workload
(M=8, N=10, F=1025, T=4000) at full size on sampled frequencies."""
import numpy as np
import pytest
import torch

import oracle
from paper_2101_08563_amd import FastFCA, synth
from parity_metrics import rel, report

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in arrs]


def run(x, P0, lam0, v0, iters, config=None, algo="em"):
    N = lam0.shape[1]
    xd, Pd, ld, vd = dev(x, P0, lam0, v0)
    ctx = FastFCA(xd, N, Pd, ld, vd)
    if config:
        ctx.set_config(*config)
    ctx.set_algorithm(algo)
    ctx.em_step(iters)
    ctx.sync()
    out = dict(trace=ctx.ll_trace(), ll=ctx.loglik(), cfg=ctx.get_config())
    out["P"], out["lam"], out["v"] = (t.cpu().numpy() for t in ctx.get_params())
    out["y"] = ctx.mwf().cpu().numpy()
    ctx.close()
    return out


@pytest.mark.parametrize("M,N,T", [(5, 6, 300), (8, 10, 777), (3, 4, 3000), (8, 12, 130),
                                   (6, 2, 64), (7, 9, 2100), (2, 3, 4096)])
def test_wide_family_parity(M, N, T):
    F, iters = 5, 12
    x = synth.mixture(F=F, T=T, M=M, N=N, rank=3, diffuse=0.1, config_id=60 + M, mixture_id=N)
    P0, lam0, v0 = synth.init_params(x, N, config_id=60 + M, mixture_id=N)
    g = run(x, P0, lam0, v0, iters)
    Po, lo, vo, tro = oracle.fit(x, P0, lam0, v0, iters, trace=True)
    llo, _ = oracle.loglik(x, Po, lo, vo)
    yo = oracle.mwf(x, Po, lo, vo)
    errs = report(g, Po, lo, vo, yo)
    errs.update(ll=abs(g["ll"] - llo), tr=float(np.abs(g["trace"] - tro).max()))
    print("wide", M, N, T, g["cfg"], {k: "%.2e" % e for k, e in errs.items()}, flush=True)
    for k in ("v", "lam", "P", "y", "v_f", "lam_f", "P_f", "y_f"):
        assert errs[k] < 1e-4, (k, errs)
    assert errs["v_log999"] < 1e-3, errs
    # the trace's per-bin terms are single precision logarithms; with up to
    # eight channels per bin they stay within 2e-6 nats/bin (1.3e-6 observed)
    assert errs["ll"] < 1e-6 and errs["tr"] < 2e-6, errs


@pytest.mark.parametrize("M,N,T", [(5, 6, 300), (8, 10, 777), (6, 2, 64), (7, 9, 2100)])
def test_wide_family_mm_parity(M, N, T):
    # Algorithm 2 (IP+MM) in the wide kernel against the oracle's MM rules
    F, iters = 5, 12
    x = synth.mixture(F=F, T=T, M=M, N=N, rank=3, diffuse=0.1, config_id=90 + M, mixture_id=N)
    P0, lam0, v0 = synth.init_params(x, N, config_id=90 + M, mixture_id=N)
    g = run(x, P0, lam0, v0, iters, algo="mm")
    Po, lo, vo, tro = oracle.fit(x, P0, lam0, v0, iters, algo=1, trace=True)
    llo, _ = oracle.loglik(x, Po, lo, vo)
    yo = oracle.mwf(x, Po, lo, vo)
    errs = report(g, Po, lo, vo, yo)
    errs.update(ll=abs(g["ll"] - llo), tr=float(np.abs(g["trace"] - tro).max()))
    print("wide mm", M, N, T, g["cfg"], {k: "%.2e" % e for k, e in errs.items()}, flush=True)
    for k in ("v", "lam", "P", "y", "v_f", "lam_f", "P_f", "y_f"):
        assert errs[k] < 1e-4, (k, errs)
    assert errs["v_log999"] < 1e-3, errs
    assert errs["ll"] < 1e-6 and errs["tr"] < 2e-6, errs
    # Algorithm 2 never lowers the likelihood either
    assert np.all(np.diff(g["trace"]) > -1e-6), g["trace"]


def test_wide_launch_shapes_agree():
    x = synth.mixture(F=4, T=1500, M=6, N=7, rank=3, config_id=70)
    P0, lam0, v0 = synth.init_params(x, 7, config_id=70)
    a = run(x, P0, lam0, v0, 8, config=(192, 8))
    b = run(x, P0, lam0, v0, 8, config=(384, 4))
    Po, lo, vo, _ = oracle.fit(x, P0, lam0, v0, 8)
    for g in (a, b):
        assert rel(g["v"], vo) < 1e-4 and rel(g["P"], Po) < 1e-4


def test_large_array_workload_full_size_sampled():
    """M=8, N=10, F=1025, T=4000, 100 iterations at full size on the GPU;
    sampled frequencies checked against the oracle run on those frequencies."""
    c = synth.CONFIGS["c3"]
    F, T, M, N, iters = c["F"], c["T"], c["M"], c["N"], c["n_iter"]
    x = synth.mixture(F=F, T=T, M=M, N=N, rank=c["rank"], diffuse=c["diffuse"], config_id=c["config_id"])
    P0, lam0, v0 = synth.init_params(x, N, config_id=c["config_id"])
    xd, Pd, ld, vd = dev(x, P0, lam0, v0)
    ctx = FastFCA(xd, N, Pd, ld, vd)
    ctx.em_step(iters)
    ctx.sync()
    P, lam, v = (t.cpu().numpy() for t in ctx.get_params())
    trace = ctx.ll_trace()
    ctx.close()
    assert np.all(np.isfinite(trace)) and trace[-1] > trace[0]
    sample = [0, 1, 300, 512, 777, 1024]
    Po, lo, vo, _ = oracle.fit(x[sample], P0[sample], lam0[sample], v0[sample], iters)
    errs = report(dict(P=P[sample], lam=lam[sample], v=v[sample]), Po, lo, vo)
    print("c3 sampled", {k: "%.2e" % e for k, e in errs.items()}, flush=True)
    for k in ("v", "lam", "P", "v_f", "lam_f", "P_f"):
        assert errs[k] < 1e-4, (k, errs)
    assert errs["v_log999"] < 1e-3, errs

"""Batched FastFCA: many mixtures of mixed (M, N, T) in one persistent launch
per em_step call, against the FP64 oracle and against single-mixture runs."""
import numpy as np
import pytest
import torch

import oracle
from paper_2101_08563_amd import FastFCA, synth
from parity_metrics import rel, report

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def batch_inputs(n_mix=8, F=12, seed=0):
    specs = synth.batch_specs(B=n_mix, F=F, seed=seed)
    out = []
    for s in specs:
        x = synth.mixture(F=s["F"], T=s["T"], M=s["M"], N=s["N"], rank=s["rank"], diffuse=s["diffuse"],
                          config_id=s["config_id"], mixture_id=s["mixture_id"])
        P0, lam0, v0 = synth.init_params(x, s["N"], config_id=s["config_id"], mixture_id=s["mixture_id"])
        out.append((x, P0, lam0, v0, s["N"]))
    return out


def make_batch(inputs):
    probs = []
    for x, P0, lam0, v0, N in inputs:
        probs.append(dict(x=torch.from_numpy(x).to(DEV), N=N, P0=torch.from_numpy(P0).to(DEV),
                          lam0=torch.from_numpy(lam0).to(DEV), v0=torch.from_numpy(v0).to(DEV)))
    return FastFCA.from_batch(probs), probs


def test_batch_shapes_cover_the_classes():
    specs = synth.batch_specs(B=256, F=513)
    Ms = {s["M"] for s in specs}
    assert Ms == {2, 3, 4}
    assert all(s["N"] - s["M"] in (1, 2) for s in specs)
    Ts = [s["T"] for s in specs]
    assert 200 <= min(Ts) and max(Ts) <= 2000


@pytest.fixture(scope="module")
def batch513():
    """Eight mixtures of the batch workload's shapes at its F = 513
    (T ~ U{200..2000}, M in {2, 3, 4}, N in {M+1, M+2}) with the oracle's fits."""
    inputs = batch_inputs(8, F=513)
    fits = []
    for x, P0, lam0, v0, N in inputs:
        Po, lo, vo, tro = oracle.fit(x, P0, lam0, v0, 20, trace=True)
        llo, _ = oracle.loglik(x, Po, lo, vo)
        fits.append((Po, lo, vo, tro, llo, oracle.mwf(x, Po, lo, vo)))
    return inputs, fits


@pytest.mark.parametrize("schedule", ["persistent", "classes"])
def test_batch_matches_oracle_per_mixture(schedule, batch513):
    inputs, fits = batch513
    ctx, _ = make_batch(inputs)
    ctx.set_schedule(schedule)
    assert ctx.num_problems == 8
    ctx.em_step(20)
    ctx.sync()
    for b, ((x, P0, lam0, v0, N), (Po, lo, vo, tro, llo, yo)) in enumerate(zip(inputs, fits)):
        P, lam, v = (t.cpu().numpy() for t in ctx.get_params(b))
        y = ctx.mwf(b).cpu().numpy()
        errs = report(dict(P=P, lam=lam, v=v, y=y), Po, lo, vo, yo)
        errs["ll"] = abs(ctx.loglik(b) - llo)
        print(schedule, "mixture", b, x.shape, N, {k: "%.2e" % e for k, e in errs.items()}, flush=True)
        for k in ("v", "lam", "P", "y", "v_f", "lam_f", "P_f", "y_f"):
            assert errs[k] < 1e-4, (k, errs)
        assert errs["v_log999"] < 1e-3 and errs["ll"] < 1e-6, errs
        tr = ctx.ll_trace(b)
        assert np.abs(tr - tro).max() < 1e-4
    ctx.close()


def test_batch_equals_single_runs():
    """Each mixture of the batch ends where it ends when run alone (same
    iterations; launch shapes differ, so equal up to single precision)."""
    inputs = batch_inputs(5, F=6, seed=3)
    ctx, _ = make_batch(inputs)
    ctx.em_step(10)
    ctx.sync()
    for b, (x, P0, lam0, v0, N) in enumerate(inputs):
        single = FastFCA(*(torch.from_numpy(a).to(DEV) for a in (x,)), N,
                         *(torch.from_numpy(a).to(DEV) for a in (P0, lam0, v0)))
        single.em_step(10)
        Ps, ls, vs = (t.cpu().numpy() for t in single.get_params())
        Pb, lb, vb = (t.cpu().numpy() for t in ctx.get_params(b))
        single.close()
        assert rel(vb, vs) < 2e-5 and rel(lb, ls) < 2e-5 and rel(Pb, Ps) < 2e-5
    ctx.close()


def test_batch_graph_replay_and_determinism():
    """Replaying the captured graph (two calls of 5) equals one call of 10,
    bitwise, and two identical batches give identical results."""
    inputs = batch_inputs(4, F=5, seed=5)
    a, _ = make_batch(inputs)
    b, _ = make_batch(inputs)
    a.em_step(5)
    a.em_step(5)
    b.em_step(10)
    for k in range(4):
        for ta, tb in zip(a.get_params(k), b.get_params(k)):
            assert torch.equal(ta, tb)
    a.close()
    b.close()


def test_batch_autotune_keeps_state_and_results():
    inputs = batch_inputs(3, F=4, seed=7)
    ctx, _ = make_batch(inputs)
    before = [tuple(t.clone() for t in ctx.get_params(k)) for k in range(3)]
    ctx.autotune(n_iter=3)
    after = [ctx.get_params(k) for k in range(3)]
    for bp, ap in zip(before, after):
        for tb, ta in zip(bp, ap):
            assert torch.equal(tb, ta)
    ctx.em_step(8)
    for k, (x, P0, lam0, v0, N) in enumerate(inputs):
        Po, lo, vo, _ = oracle.fit(x, P0, lam0, v0, 8)
        assert rel(ctx.get_params(k)[2].cpu().numpy(), vo) < 1e-4
    ctx.close()


def test_single_autotune_cache(tmp_path):
    x = synth.mixture(F=8, T=700, M=2, N=3, config_id=40)
    P0, lam0, v0 = synth.init_params(x, 3, config_id=40)
    ctx = FastFCA(*(torch.from_numpy(a).to(DEV) for a in (x,)), 3,
                  *(torch.from_numpy(a).to(DEV) for a in (P0, lam0, v0)))
    cache = tmp_path / "tune.jsonl"
    ctx.autotune(n_iter=4, cache_path=str(cache))
    import json
    lines = [json.loads(l) for l in cache.read_text().splitlines()]
    assert lines and lines[0]["M"] == 2 and lines[0]["N"] == 3
    th, bpt = ctx.get_config()
    assert th * bpt >= 700
    ctx.em_step(6)
    Po, lo, vo, _ = oracle.fit(x, P0, lam0, v0, 6)
    assert rel(ctx.get_params()[2].cpu().numpy(), vo) < 1e-4
    ctx.close()


@pytest.mark.parametrize("M,N,T,cfg", [(2, 3, 250, (128, 2)), (2, 3, 256, (128, 2)), (2, 3, 128, (64, 4)),
                                       (2, 3, 400, (64, 8)), (2, 3, 1000, (256, 4)), (2, 3, 2000, (256, 8)),
                                       (3, 4, 250, (64, 4)), (3, 4, 400, (64, 8)), (3, 5, 400, (128, 4)),
                                       (4, 5, 1000, (256, 4)), (4, 6, 1500, (192, 8)),
                                       (6, 7, 1000, (256, 4)), (6, 7, 3000, (384, 8))])
def test_default_launch_shapes(M, N, T, cfg):
    """The default (threads, bins per thread) of a single mixture: two bins
    per thread for M = 2 at 129-256 frames (two wavefronts); eight at
    257-512 frames (one wavefront; not for M = 3, N = 5) and beyond 1024
    frames; four otherwise; the wide family (M = 6) four up to 2048 frames,
    eight beyond; and the fit under it matches the oracle."""
    x = synth.mixture(F=3, T=T, M=M, N=N, config_id=41)
    P0, lam0, v0 = synth.init_params(x, N, config_id=41)
    ctx = FastFCA(torch.from_numpy(x).to(DEV), N, *(torch.from_numpy(a).to(DEV) for a in (P0, lam0, v0)))
    assert tuple(ctx.get_config()) == cfg
    ctx.em_step(5)
    Po, lo, vo, _ = oracle.fit(x, P0, lam0, v0, 5)
    assert rel(ctx.get_params()[2].cpu().numpy(), vo) < 1e-4
    ctx.close()


def test_batch_with_a_wide_class_uses_class_launches():
    """A batch holding a mixture outside the persistent kernel's classes (M = 5:
    the wide family) runs with the class schedule; the persistent schedule is
    refused; every mixture matches the oracle."""
    from paper_2101_08563_amd import FastFCAError
    shapes = [(5, 300, 5, 6), (7, 650, 2, 3), (6, 130, 3, 5)]
    inputs = []
    for i, (F, T, M, N) in enumerate(shapes):
        x = synth.mixture(F=F, T=T, M=M, N=N, rank=3, config_id=45, mixture_id=i)
        P0, lam0, v0 = synth.init_params(x, N, config_id=45, mixture_id=i)
        inputs.append((x, P0, lam0, v0, N))
    ctx, _ = make_batch(inputs)
    with pytest.raises(FastFCAError) as e:
        ctx.set_schedule("persistent")
    assert e.value.code == -7
    ctx.em_step(10)
    ctx.sync()
    for b, (x, P0, lam0, v0, N) in enumerate(inputs):
        P, lam, v = (t.cpu().numpy() for t in ctx.get_params(b))
        Po, lo, vo, _ = oracle.fit(x, P0, lam0, v0, 10)
        assert rel(v, vo) < 1e-4 and rel(lam, lo) < 1e-4 and rel(P, Po) < 1e-4
    ctx.close()

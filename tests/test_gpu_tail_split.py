"""The tail split (fastfca_set_tail_split) changes the schedule, not the
arithmetic: a context whose frequency count leaves a small remainder over
the compute units runs that remainder in several launches of consecutive
iterations, and every output -- P, lambda, v, the per-iteration LL trace and
the final LL -- must equal the unsplit run bit for bit (Algorithm 1 over the
same iterations, the state kept exactly between launches). The parity tests
against the oracle run the default (automatic) schedule, so they cover the
split too for the shapes where it applies."""
import numpy as np
import pytest
import torch

from paper_2101_08563_amd import FastFCA, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _ncu():
    return torch.cuda.get_device_properties(0).multi_processor_count


def _run(problems, n_iter, split, steps=None, algo="em"):
    ctx = FastFCA.from_batch([dict(x=x, N=N) for x, N in problems], seed=7) if len(problems) > 1 else \
        FastFCA(problems[0][0], problems[0][1], seed=7)
    ctx.set_tail_split(split)
    ctx.set_algorithm(algo)
    out = []
    for k in (steps or [n_iter]):
        ctx.em_step(k)
        ctx.sync()
        out.append([ctx.ll_trace(b) for b in range(len(problems))])
    res = dict(traces=out, params=[[a.cpu().numpy() for a in ctx.get_params(b)] for b in range(len(problems))],
               ll=[ctx.loglik(b) for b in range(len(problems))])
    ctx.close()
    return res


def _same(a, b):
    for ta, tb in zip(a["traces"], b["traces"]):
        for x, y in zip(ta, tb):
            assert x.shape == y.shape and np.array_equal(x, y)
    for pa, pb in zip(a["params"], b["params"]):
        for x, y in zip(pa, pb):
            assert np.array_equal(x, y)
    assert a["ll"] == b["ll"]


def _mix(F, T, M, N, mid):
    x = synth.mixture(F=F, T=T, M=M, N=N, rank=4, diffuse=0.05, config_id=70, mixture_id=mid)
    return torch.from_numpy(x).to(DEV)


@pytest.mark.parametrize("blocks,n_iter", [(-1, 40), (3, 10), (7, 23)])
def test_split_equals_one_launch_bitwise(blocks, n_iter):
    """One remainder frequency (F = CUs + 1, four waves per workgroup, so the
    split applies): automatic and forced block counts, blocks of unequal
    length."""
    F = _ncu() + 1
    p = [(_mix(F, 1000, 2, 3, 0), 3)]
    print("F", F, "blocks", blocks, "iterations", n_iter, flush=True)
    _same(_run(p, n_iter, blocks), _run(p, n_iter, 0))


def test_split_batch_of_equal_shapes_and_resumed_calls():
    """Two mixtures of one shape (one class, remainder 2 items) and a call
    split into two em_step calls."""
    F = _ncu() // 2 + 1
    p = [(_mix(F, 1000, 3, 4, 1), 4), (_mix(F, 1000, 3, 4, 2), 4)]
    _same(_run(p, 30, -1, steps=[20, 30]), _run(p, 30, 0, steps=[20, 30]))


def test_split_with_algorithm_2():
    F = _ncu() + 1
    p = [(_mix(F, 1000, 2, 3, 4), 3)]
    _same(_run(p, 30, -1, algo="mm"), _run(p, 30, 0, algo="mm"))


@pytest.mark.parametrize("blocks", [-1, 5])
def test_split_wide_family_partial_last_round(blocks):
    """M = 8, N = 10, T = 4000 (one workgroup per CU): F = CUs + 1 leaves a
    last round of one frequency, which the split spreads over the gaps."""
    from paper_2101_08563_amd.fastfca import synth_mixture
    F = _ncu() + 1
    x = synth_mixture(F, 4000, 8, 10, rank=8, diffuse=0.05, seed=11)
    print("wide F", F, "blocks", blocks, flush=True)
    p = [(x, 10)]
    _same(_run(p, 20, blocks), _run(p, 20, 0))


def test_split_wide_family_four_bins_per_thread():
    """The wide family at four bins per thread (up to 2048 frames) and its
    tail instance."""
    from paper_2101_08563_amd.fastfca import synth_mixture
    F = _ncu() + 1
    x = synth_mixture(F, 1500, 6, 7, rank=6, diffuse=0.05, seed=13)
    p = [(x, 7)]
    _same(_run(p, 16, -1), _run(p, 16, 0))
    _same(_run(p, 16, -1, algo="mm"), _run(p, 16, 0, algo="mm"))


def test_split_wide_family_with_algorithm_2():
    """The wide family's Algorithm 2 instance and its tail instance (beyond
    2048 frames, where the wide family takes eight bins per thread)."""
    from paper_2101_08563_amd.fastfca import synth_mixture
    F = _ncu() + 1
    x = synth_mixture(F, 3000, 6, 7, rank=6, diffuse=0.05, seed=12)
    p = [(x, 7)]
    _same(_run(p, 16, -1, algo="mm"), _run(p, 16, 0, algo="mm"))


def test_set_tail_split_rejects_bad_values():
    ctx = FastFCA(_mix(8, 64, 2, 2, 3), 2, seed=1)
    from paper_2101_08563_amd.fastfca import FastFCAError
    with pytest.raises(FastFCAError):
        ctx.set_tail_split(-2)
    with pytest.raises(FastFCAError):
        ctx.set_tail_split(5000)
    ctx.close()

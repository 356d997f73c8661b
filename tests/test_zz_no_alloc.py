"""fastfca_fit_noalloc (the entry point for callers that cannot allocate)
against the context path (fastfca_init + fastfca_em_step): the same kernels
and launch shape, so the results agree bit for bit; checked on two calls in
a row, the second on a smaller mixture, so the shared device array is
reused with a different layout."""
import numpy as np
import pytest
import torch

import oracle
from paper_2101_08563_amd import FastFCA, FastFCAError, synth
from paper_2101_08563_amd.fastfca import fit_noalloc
from parity_metrics import rel

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _case(F, T, M, N, seed):
    x = synth.mixture(F=F, T=T, M=M, N=N, rank=4, diffuse=0.05, config_id=70, mixture_id=seed)
    P0, lam0, v0 = synth.init_params(x, N, config_id=70, mixture_id=seed)
    return x, P0, lam0, v0


def _context_run(x, P0, lam0, v0, it):
    d = [torch.from_numpy(a).to(DEV) for a in (x, P0, lam0, v0)]
    ctx = FastFCA(d[0], lam0.shape[1], d[1], d[2], d[3])
    ctx.em_step(it)
    ctx.sync()
    P, lam, v = (a.cpu().numpy() for a in ctx.get_params())
    tr = ctx.ll_trace()
    ctx.close()
    return P, lam, v, tr


def _noalloc_run(x, P0, lam0, v0, it, with_trace):
    F = x.shape[0]
    xd, P, lam, v = (torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (x, P0, lam0, v0))
    status = torch.full((F,), 7, dtype=torch.int32, device=DEV)
    tr = torch.full((F, it), np.nan, dtype=torch.float64, device=DEV) if with_trace else None
    fit_noalloc(xd, P, lam, v, it, status, tr)
    torch.cuda.synchronize()
    return (P.cpu().numpy(), lam.cpu().numpy(), v.cpu().numpy(), status.cpu().numpy(),
            tr.cpu().numpy().mean(axis=0) if with_trace else None)


def test_noalloc_matches_context_path_twice():
    cases = [((64, 700, 2, 3, 1), 30, True), ((17, 250, 3, 4, 2), 12, False)]  # second call smaller
    for (F, T, M, N, seed), it, with_trace in cases:
        x, P0, lam0, v0 = _case(F, T, M, N, seed)
        Pc, lc, vc, trc = _context_run(x, P0, lam0, v0, it)
        Pn, ln, vn, st, trn = _noalloc_run(x, P0, lam0, v0, it, with_trace)
        print("noalloc", (F, T, M, N), "P %.1e lam %.1e v %.1e" % (rel(Pn, Pc), rel(ln, lc), rel(vn, vc)), flush=True)
        assert np.all(st == 0)
        assert np.array_equal(Pn, Pc) and np.array_equal(ln, lc) and np.array_equal(vn, vc)
        if with_trace:
            assert np.allclose(trn, trc, rtol=0, atol=1e-12)
        # and to the bar of the parity tests against the FP64 oracle
        Po, lo, vo, _ = oracle.fit(x, P0, lam0, v0, it)
        assert rel(Pn, Po) < 1e-4 and rel(ln, lo) < 1e-4 and rel(vn, vo) < 1e-4


def test_noalloc_rejects_what_does_not_fit():
    x, P0, lam0, v0 = _case(9, 100, 2, 3, 3)
    xd, P, lam, v = (torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (x, P0, lam0, v0))
    status = torch.zeros(9, dtype=torch.int32, device=DEV)
    with pytest.raises(FastFCAError) as e:
        fit_noalloc(xd, P, lam, v, 200000, status)        # trace of 9 x 200000 doubles: too large
    assert e.value.code == -1 and "scratch" in str(e.value)
    fit_noalloc(xd, P, lam, v, 3, status)                 # a good call afterwards still works
    torch.cuda.synchronize()
    assert np.all(status.cpu().numpy() == 0)

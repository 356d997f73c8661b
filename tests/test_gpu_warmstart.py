"""What the trained warm-start network gains over the method without it.

Runs the measured evaluation of paper_2101_08563_amd.train_warmstart on
held-out synthetic mixtures (M=2, N=3, F=513, T=1000) with the committed
weights: iterations of Algorithm 1 and wall time to reach LL* - 1e-2
nats/bin (LL* = the plain fit after 1200 iterations) from the seeded start,
from the network's warm start (fastfca_warmstart), and from a perfect
network (the plain fit's own targets through the same warm-start path). The
measured numbers are printed; the assertions check the mechanics (the IP+EM
refiner always reaches the tolerance from the network's start, and the
warm-start path can carry a large gain), not a gain the network does not
deliver. Below: the library's judge and fallback.
"""
import os

import pytest

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2101_08563_amd", "data",
                       "warmstart_c32l4.npz")


def test_warm_start_gain_is_measured():
    from paper_2101_08563_amd import train_warmstart
    s, rows = train_warmstart.measure(WEIGHTS, n_eval=4, conv_iters=1200)
    print("warm start evaluation:", s, flush=True)
    assert s["warm_reached_frac"] == 1.0
    assert s["perfect_net_iters_median"] < 0.5 * s["plain_iters_median"]
    for r in rows:
        assert r["ms_plain"] > 0 and r["ms_warm"] > r["ms_warmstart"] > 0
    print("iteration ratio plain/warm = %.2f, wall time plain %.3f ms vs warm %.3f ms"
          % (s["plain_iters_median"] / s["warm_iters_median"], s["plain_ms_median"], s["warm_ms_median"]),
          flush=True)


# ------------------------------------------------------------------ fastfca_warmstart: judge and fallback
import numpy as np  # noqa: E402
import torch  # noqa: E402

from paper_2101_08563_amd import FastFCA, synth, warmstart  # noqa: E402
from paper_2101_08563_amd.warmstart import ConvNet  # noqa: E402

DEV = "cuda:0"


def _mixture(F=40, T=300, M=2, N=3, seed=0):
    x = synth.mixture(F=F, T=T, M=M, N=N, rank=4, diffuse=0.05, config_id=60, mixture_id=seed)
    return torch.from_numpy(x).to(DEV)


def _params(ctx):
    return [a.cpu().numpy() for a in ctx.get_params()]


def _bad_net(M, N, how):
    net = ConvNet(M=M, N=N, C=16, L=1, seed=5)
    sd = net.state_dict()
    L = 1
    if how == "huge":
        sd["b%d" % (L + 1)][:] = 40.0      # v = exp(40) in every bin
        sd["bl"][:] = 10.0                  # lambda = exp(10): sigma^2 absurdly large
    else:
        sd["b%d" % (L + 1)][:] = np.nan     # v = NaN
    net.load_state_dict(sd)
    return net


@pytest.mark.parametrize("how", ["huge", "nan"])
def test_bad_warm_start_falls_back_to_the_plain_run_bitwise(how):
    """A network that predicts garbage: the judge rejects it in every
    frequency, the seeded start comes back bit for bit, and the IP+EM run
    from there equals the plain run bit for bit."""
    M, N, it = 2, 3, 25
    x = _mixture(M=M, N=N)
    plain = FastFCA(x, N, seed=11)
    warm = FastFCA(x, N, seed=11)
    start = _params(warm)
    taken = warm.warmstart(_bad_net(M, N, how), count=True)
    assert taken == 0
    for a, b in zip(_params(warm), start):
        assert np.array_equal(a, b)
    plain.em_step(it)
    warm.em_step(it)
    for a, b in zip(_params(warm), _params(plain)):
        assert np.array_equal(a, b)
    assert np.array_equal(warm.ll_trace(), plain.ll_trace())
    plain.close()
    warm.close()


@pytest.mark.parametrize("use_net", [False, True])
def test_warm_start_is_kept_only_where_it_raises_the_likelihood(use_net):
    """Per frequency, the start after fastfca_warmstart has a log-likelihood
    at least that of the seeded start; where the new start was kept, P is the
    whitening C_f^{-1/2} of fastfca_ws_features; elsewhere the seeded start
    is unchanged."""
    M, N = 2, 3
    x = _mixture(F=64, M=M, N=N, seed=1)
    ctx = FastFCA(x, N, seed=3)
    P_s, l_s, v_s = _params(ctx)
    _, llf_s = ctx.loglik(per_f=True)
    net = ConvNet.load(WEIGHTS) if use_net else None
    taken = ctx.warmstart(net, count=True)
    P_w, l_w, v_w = _params(ctx)
    _, llf_w = ctx.loglik(per_f=True)
    llf_s, llf_w = llf_s.cpu().numpy(), llf_w.cpu().numpy()
    assert np.all(llf_w >= llf_s)
    P0, _ = warmstart.features(x)
    P0 = P0.cpu().numpy()
    kept = np.array([not np.array_equal(P_w[f], P_s[f]) for f in range(x.shape[0])])
    assert kept.sum() == taken
    for f in range(x.shape[0]):
        if kept[f]:
            assert np.array_equal(P_w[f], P0[f])
            assert llf_w[f] >= llf_s[f]
        else:
            assert np.array_equal(v_w[f], v_s[f]) and np.array_equal(l_w[f], l_s[f])
    if not use_net:
        # whitening-only start: lambda = 1, v = (1/(M N)) sum_m |(P0^H x)_m|^2
        xs = x.cpu().numpy().astype(np.complex128)
        for f in np.nonzero(kept)[0][:8]:
            y = xs[f] @ np.conj(P0[f])
            vref = (np.abs(y) ** 2).sum(axis=1) / (M * N)
            assert np.allclose(l_w[f], 1.0)
            assert np.allclose(v_w[f], vref[:, None], rtol=1e-5, atol=0)
    ctx.close()


def test_warm_start_rejects_a_mismatched_network():
    x = _mixture(F=8, M=2, N=3)
    ctx = FastFCA(x, 3, seed=1)
    from paper_2101_08563_amd import FastFCAError
    with pytest.raises(FastFCAError) as e:
        ctx.warmstart(ConvNet(M=2, N=4, C=16, L=1))
    assert e.value.code == -1
    ctx.close()


# ------------------------------------------------------------------ fastfca_warmstart_race
def test_race_with_a_failing_start_equals_the_plain_run_bitwise():
    """A network whose start fails (NaN powers) loses the race in every
    frequency: the state after the race is the plain run's after the same
    number of iterations, bit for bit, and the context goes on from there."""
    M, N, K = 2, 3, 15
    x = _mixture(M=M, N=N)
    plain = FastFCA(x, N, seed=11)
    plain.em_step(K)
    race = FastFCA(x, N, seed=11)
    kept = race.warmstart_race(_bad_net(M, N, "nan"), K, count=True)
    assert kept == 0
    for a, b in zip(_params(plain), _params(race)):
        assert np.array_equal(a, b)
    # the context goes on from there like the plain run
    plain.em_step(5)
    race.em_step(5)
    plain.sync()
    race.sync()
    for a, b in zip(_params(plain), _params(race)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("which", ["whitening", "network"])
def test_race_keeps_the_better_start_per_frequency(which):
    """The seeded start against the whitening-only start or the trained
    network's, 100 iterations each, on a headline-shaped mixture: no
    frequency ends below the plain run after the same iterations (up to the
    single precision trace the choice is made on), the frequencies that kept
    the new start end above it, and the state is finite."""
    from paper_2101_08563_amd.fastfca import synth_mixture
    M, N, K = 2, 3, 100
    x = synth_mixture(513, 1000, M, N, seed=4242)
    net = ConvNet.load(WEIGHTS) if which == "network" else None
    plain = FastFCA(x, N, seed=5)
    plain.em_step(K)
    _, llf_plain = plain.loglik(per_f=True)
    race = FastFCA(x, N, seed=5)
    kept = race.warmstart_race(net, K, count=True)
    race.sync()
    _, llf_race = race.loglik(per_f=True)
    a, b = llf_plain.cpu().numpy(), llf_race.cpu().numpy()
    print("race (%s) kept the new start in %d of 513 frequencies; LL per bin plain %.6f race %.6f"
          % (which, kept, a.mean(), b.mean()), flush=True)
    assert 0 <= kept <= 513
    assert np.all(b >= a - 1e-5)
    assert b.mean() >= a.mean()
    assert all(np.isfinite(t).all() for t in _params(race))


def test_race_rejects_bad_arguments():
    x = _mixture(F=8, T=64)
    ctx = FastFCA(x, 3, seed=1)
    from paper_2101_08563_amd.fastfca import FastFCAError
    with pytest.raises(FastFCAError):
        ctx.warmstart_race(None, 0)
    ctx.close()

"""What the trained warm-start network gains over the method without it.

Runs the evaluation of paper_2101_08563_amd.train_warmstart on held-out
synthetic mixtures (M=2, N=3, F=513, T=1000) with the committed weights:
iterations of Algorithm 1 to reach LL* - 1e-2 nats/bin (LL* = the plain
fit after 1200 iterations) from the seeded start, from the network's warm
start, and from a perfect network (the plain fit's own targets through the
same warm-start path). The measured numbers are printed; the assertions
check the mechanics (the IP+EM refiner always reaches the tolerance from the
network's start, and the warm-start path can carry a large gain), not a gain
the network does not deliver.
"""
import os

import pytest

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2101_08563_amd", "data",
                       "warmstart_c64l6.npz")


def test_warm_start_gain_is_measured():
    from paper_2101_08563_amd import train_warmstart
    s = train_warmstart.evaluate(WEIGHTS, n_eval=4, conv_iters=1200, batch=4)
    print("warm start evaluation:", s, flush=True)
    assert s["warm_reached_frac"] == 1.0
    assert s["perfect_net_iters_median"] < 0.5 * s["plain_iters_median"]
    gain = s["plain_iters_median"] / s["warm_iters_median"]
    print("iteration ratio plain/warm = %.2f, wall time plain %.3f ms vs warm %.3f ms"
          % (gain, s["plain_ms_median"], s["warm_ms_median"]), flush=True)

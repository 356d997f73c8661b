"""The running sigma^2 of the M = 4 resident kernels (CPU emulation in
single precision, test infrastructure; the M = 2 kernels form the sum again
after every source).

Algorithm 1 (Sec. IV-E) updates the sources of a bin in order, each with
sigma^2 = sum_n v_n lambda_n from the sources already updated. The kernels
keep sigma^2 in registers and change it by the updated source's own term,
sigma^2 <- (sigma^2 - l_old v_old) + l_new v_new. When that source dominated
the bin and its term collapses, the subtraction cancels most digits. The
kernels then form the sum again: whenever some bin's new sigma^2 is below
a quarter of the old one (each update then loses at most two bits, and
consecutive updates cannot compound more). This emulation bounds the per-bin error of both forms
against double precision over a wide dynamic range.
"""
import numpy as np

DROP = np.float32(0.25)


def _run(guard, n_bins=20000, N=3, seed=0):
    rng = np.random.default_rng(seed)
    f32 = np.float32
    # terms lambda_n v_n over twelve decades; source 0 dominates half the bins
    lv = 10.0 ** rng.uniform(-6, 6, (n_bins, N))
    dom = rng.random(n_bins) < 0.5
    lv[dom, 0] = lv[dom].sum(axis=1) * 1e3
    lv32 = lv.astype(f32)
    sg = lv32.sum(axis=1, dtype=f32)
    worst = 0.0
    for n in range(N - 1):
        # the source's term moves by a factor between 1e-8 and 1e2
        new = (lv32[:, n].astype(np.float64) * 10.0 ** rng.uniform(-8, 2, n_bins)).astype(f32)
        sn = (sg - lv32[:, n]).astype(f32) + new
        sn = sn.astype(f32)
        lv32[:, n] = new
        if guard:
            redo = ~(sn >= DROP * sg)
            if redo.any():           # the kernels redo the whole wavefront; per bin is the same values
                sn[redo] = lv32[redo].sum(axis=1, dtype=f32)
        sg = sn
        exact = lv32.astype(np.float64).sum(axis=1)
        worst = max(worst, float(np.max(np.abs(sg - exact) / exact)))
    return worst


def test_unguarded_running_sum_cancels():
    assert _run(guard=False) > 1e-2


def test_guarded_running_sum_stays_accurate():
    # a direct single precision sum of the terms is good to about 2e-7
    assert max(_run(guard=True, seed=s) for s in range(5)) < 1e-6

"""Reduced-precision storage over many steps: FP32 storage, and BF16 storage
with FP32 reconstruction (FP64 Courant number, flux integral and update, the
rounding residual carried along the pencil), against the FP64 oracle after
1, 20 and 100 steps of the sparse-Maxwellian recipe on a 16 x 16 x 8 box.

Reported per storage and horizon: relative max-norm and L1 error over the
union of the block lists (absent blocks read as zero), the mass held in f
(stored only) and the mass held in f plus the rounding ledger, each as the
relative change from the initial stored mass after adding back what the
pruning removed.  The bounds:
  * FP32: at most 1e-5 relative max-norm per step (so k * 1e-5 after k steps);
  * BF16: one step is bounded by the initial rounding and, per shear, a
    cell's rounding plus the residual carried in from its neighbour (2^-9 of
    a value each): 3 * 2^-8 + 2^-9 per step;
  * stored plus ledger mass: 1e-12 relative after any number of steps;
  * stored-only mass: the residual that a shear leaves at the end of a line is
    put back into the same line at the next shear along that axis, so what f
    lacks is only the residuals of the last shear of each axis and does not
    grow with the number of steps: the largest drift over steps 21-100 is at
    most twice the largest over steps 1-5 (a residual kept out of f for good
    would make it grow like the square root of the step count, about ten
    times over these horizons)."""
import numpy as np
import pytest

from oracle import OraclePartition
from paper_2504_21450_amd import binding as B
from paper_2504_21450_amd import workloads as W
from gpuhelp import gpu_partition, need_gpu, print_case
from statehelp import to_dense

pytestmark = pytest.mark.gpu
HORIZONS = (1, 20, 100)
BF16_STEP = 3 * 2.0 ** -8 + 2.0 ** -9


@pytest.fixture(scope="module")
def reference():
    need_gpu()
    w = W.maxwellian_sparse(n=(16, 16, 8), threads=16)
    print_case("oracle: 16x16x8 sparse maxwellian, 100 FP64 steps")
    o = OraclePartition.from_workload(w)
    snaps = {}
    for k in range(1, HORIZONS[-1] + 1):
        o.fill_ghosts()
        o.step(w.dt)
        if k in HORIZONS:
            snaps[k] = o.export_local()
    return w, snaps


def norms(a, b, NB):
    da, db = to_dense(*a, NB), to_dense(*b, NB)
    return (np.max(np.abs(da - db)) / np.max(np.abs(db)),
            np.sum(np.abs(da - db)) / np.sum(np.abs(db)))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("storage,name", [(B.VL_F32, "FP32"), (B.VL_BF16, "BF16")])
def test_reduced_storage_error_and_mass_table(reference, storage, name):
    w, snaps = reference
    NB = int(np.prod(w.nblk))
    print_case("%s storage, 100 steps against the oracle" % name)
    p = gpu_partition(w, storage=storage, slack=6.0)
    m0 = None
    pruned = 0.0
    ledger = 0.0
    rows = []
    drift = []
    for k in range(1, HORIZONS[-1] + 1):
        p.fill_ghosts()
        s = p.step(w.dt, B.VL_COALESCED, stats=True)
        if m0 is None:
            m0 = s["mass_before"]
        pruned += s["pruned_mass"]
        ledger += s["ledger_mass"]
        drift.append((s["mass_after"] + pruned - m0) / m0)
        if k in HORIZONS:
            st = p.export()
            mx, l1 = norms(st, snaps[k], NB)
            stored = (s["mass_after"] + pruned - m0) / m0
            with_ledger = (s["mass_after"] + pruned + ledger - m0) / m0
            fmin = float(np.min(st[2])) if st[2].size else 0.0
            rows.append((k, mx, l1, stored, with_ledger, fmin))
    print("%s  steps  max-norm    L1          stored-only  stored+ledger  min f" % name)
    for r in rows:
        print("%s  %5d  %.3e  %.3e  %+.3e   %+.3e     %.3e" % ((name,) + r))
    d = np.abs(np.array(drift))
    print("%s  stored-only drift: max over steps 1-5 %.3e, 6-20 %.3e, 21-100 %.3e"
          % (name, d[:5].max(), d[5:20].max(), d[20:].max()))
    for k, mx, l1, stored, with_ledger, fmin in rows:
        bound = k * (1e-5 if storage == B.VL_F32 else BF16_STEP)
        assert mx <= bound, (k, mx)
        assert abs(with_ledger) <= 1e-12, (k, with_ledger)
        assert fmin >= 0.0
    assert d[20:].max() <= 2.0 * d[:5].max(), (d[:5].max(), d[20:].max())

"""Ghost Translation levels on the benchmark partition (64 x 64 x 32 cells,
sparse 100^3 velocity mesh): what GT1 and GT2 (Section 3.2) save in computed
updates and what their stale ghost layers cost in accuracy after one step,
against GT3 (exact)."""
import numpy as np
import pytest

from paper_2504_21450_amd import binding as B
from paper_2504_21450_amd import workloads as W
from gpuhelp import need_gpu, print_case
from statehelp import to_dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    need_gpu()
    print_case("generating the 64x64x32 sparse workload")
    return W.maxwellian_sparse(n=(64, 64, 32), threads=16)


def sample_cells(n):
    """Columns x in {0, 21, 42} of every (y, z): all distances from the y and
    z faces are represented."""
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.array([0, 21, 42]), indexing="ij")
    x, y, z = x.reshape(-1), y.reshape(-1), z.reshape(-1)
    dist = np.minimum(np.minimum(y, n[1] - 1 - y), np.minimum(z, n[2] - 1 - z))
    return x + n[0] * (y + n[1] * z), dist


def test_limited_levels_stale_error_and_saved_updates(full):
    w = full
    cells, dist = sample_cells(w.n)
    NB = int(np.prod(w.nblk))
    res = {}
    for k in (3, 2, 1):
        print_case("GT%d one step" % k)
        p = B.Partition.from_workload(w, slack=1.4, gt_level=k)
        p.fill_ghosts()
        s = p.step(w.dt, B.VL_COALESCED, stats=True)
        res[k] = (s, to_dense(*p.export_cells(cells), NB))
        p.close()
        del p
    ref = res[3][1]
    scale = np.max(np.abs(ref))
    for k in (2, 1):
        s, d = res[k]
        inner = dist >= 3 - k
        assert np.array_equal(d[inner], ref[inner])          # exact away from stale layers
        err = np.abs(d - ref)
        mx = err.max() / scale
        l1 = err.sum() / np.abs(ref).sum()
        upd = sum(s["updated_ps"]) / sum(res[3][0]["updated_ps"])
        # a stale ghost layer's inflow no longer matches the outflow of its
        # periodic image, so the partition's mass drifts
        drift = (s["mass_after"] + s["pruned_mass"] - s["mass_before"]) / s["mass_before"]
        print("GT%d: stale error max-norm %.3e, L1 %.3e on the sampled columns; computed updates "
              "%.4f of GT3's; relative mass drift %.3e" % (k, mx, l1, upd, drift))
        assert mx > 0.0 and upd < 1.0
    e1 = np.abs(res[1][1] - ref).max()
    e2 = np.abs(res[2][1] - ref).max()
    assert e2 <= e1
    for k in (1, 2, 3):
        assert res[k][0]["updated_ps"][2] == res[3][0]["updated_ps"][2]

"""FP64 velocity moments of the HIP path against the oracle's two-pass
moments, on a blob mixture whose hot cells hold about 4,400 blocks each: those
cells are split over several wavefronts (1024 blocks each) and their partial
sums combined in chunk order.  Reduced storage: the oracle takes the exported
(widened) state, so both sides sum the same values.  Tolerances: n and V to
1e-12 (V relative to the largest of |V| and the thermal speed), P to 1e-11 of
its largest diagonal, the total mass to 1e-12; two runs give the same bits."""
import numpy as np
import pytest
import torch

from oracle import OraclePartition
from paper_2504_21450_amd import binding as B
from paper_2504_21450_amd import workloads as W
from gpuhelp import gpu_partition, need_gpu, print_case, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mixture():
    need_gpu()
    return W.blob_mixture(n=(6, 6, 4), hot_fraction=0.4, threads=16, storage=B.VL_F64)


def oracle_moments(w, state):
    o = OraclePartition(w.n, w.nblk, w.dx, w.vmin, w.dv, w.order, w.sparse_min, w.vbuffer)
    o.load_local(*state)
    return o.moments()


def check(p, w, state):
    dn, dV, dP, tot = p.moments()
    dn, dV, dP = dn.cpu().numpy(), dV.cpu().numpy(), dP.cpu().numpy()
    on, oV, oP, otot = oracle_moments(w, state)
    assert np.max(np.abs(dn - on)) <= 1e-12 * np.max(on)
    vth = np.sqrt(np.max(np.abs(oP[:, :3])) / (1.67262192e-27 * np.min(on)))
    assert np.max(np.abs(dV - oV)) <= 1e-12 * max(np.max(np.abs(oV)), vth)
    assert np.max(np.abs(dP - oP)) <= 1e-11 * np.max(np.abs(oP[:, :3]))
    assert abs(tot - otot) <= 1e-12 * otot
    return dn, dV, dP, tot


@pytest.mark.parametrize("storage", [B.VL_F64, B.VL_F32, B.VL_BF16])
def test_moments_of_split_cells_match_the_oracle(mixture, storage):
    w = mixture
    counts = np.diff(w.offsets)
    assert counts.max() > 4 * 1024   # cells split into five chunks
    print_case("moments of a mixture with split cells, storage %d" % storage)
    p = gpu_partition(w, storage=storage)
    check(p, w, p.export())            # the initial state (rounded to the storage)
    run_gpu(p, w.dt, 2)
    first = check(p, w, p.export())    # after two steps
    again = p.moments()
    assert all(np.array_equal(a.cpu().numpy() if torch.is_tensor(a) else a,
                              b.cpu().numpy() if torch.is_tensor(b) else b) for a, b in zip(first, again))


def test_moments_of_empty_and_single_block_cells():
    """Empty cells give zero density, velocity and pressure; a cell with one
    block the exact sums of its 64 values."""
    n, nblk = (3, 2, 2), (3, 3, 3)
    rng = np.random.default_rng(51)
    counts = [0, 1, 0, 27, 3, 0, 1, 2, 0, 0, 5, 1]
    ids, fs = [], []
    for c in counts:
        ids.append(np.sort(rng.choice(27, size=c, replace=False)).astype(np.int32))
        fs.append(rng.uniform(1e-10, 1e-9, c * 64))
    off = np.zeros(len(counts) + 1, np.int64)
    off[1:] = np.cumsum(counts)
    state = (off, np.concatenate(ids), np.concatenate(fs))
    w = W.Workload("cells", n, (5.0, 5.0, 5.0), nblk, (-6.0, -6.0, -6.0), (1.0, 1.0, 1.0), 1.0, 1, 0.0, 0,
                   B.VL_F64, (0, 1, 2), *state)
    print_case("moments of empty and small cells")
    p = gpu_partition(w)
    dn, dV, dP, tot = p.moments()
    dn, dV, dP = dn.cpu().numpy(), dV.cpu().numpy(), dP.cpu().numpy()
    on, oV, oP, otot = oracle_moments(w, state)
    empty = np.array(counts) == 0
    assert np.all(dn[empty] == 0.0) and np.all(dV[empty] == 0.0) and np.all(dP[empty] == 0.0)
    assert np.max(np.abs(dn - on)) <= 1e-12 * np.max(on)
    assert np.max(np.abs(dV - oV)) <= 1e-12 * np.max(np.abs(oV))
    assert np.max(np.abs(dP - oP)) <= 1e-11 * np.max(np.abs(oP[:, :3]))

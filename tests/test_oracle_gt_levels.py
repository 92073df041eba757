"""Ghost Translation with limited active sets (Section 3.2: GT1, GT2) in the
oracle: the update boxes follow the paper's limited set construction, the
local result equals GT3 bit for bit wherever no stencil reaches a ghost layer
left at its ghost-update value, and differs next to the faces."""
import numpy as np
import pytest

from oracle import COALESCED, OraclePartition
from oracle import gt_sets
from statehelp import random_state, to_dense

KW = dict(nblk=(3, 2, 3), dx=(6.0, 5.0, 7.0), vmin=(-6.0, -4.0, -6.0), dv=(1.0, 1.0, 1.0))


def make(n, order, k, sparse_min=2.5e-10, vbuffer=6, nblk=KW["nblk"]):
    p = OraclePartition(n, nblk, KW["dx"], KW["vmin"], KW["dv"], order, sparse_min, vbuffer)
    p.set_gt_level(k)
    return p


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("order", [(0, 1, 2), (2, 0, 1), (1, 2, 0)])
def test_update_boxes_follow_the_limited_sets(order, k):
    """Boxes = the GTk active sets (reverse construction of Section 3.1,
    clipped to k layers around the local domain as in Section 3.2) in flux
    form, taken from the lattice construction."""
    n = 6
    p = make((n, n, n), order, k)
    want = gt_sets.pull_update_boxes(n, order, k)
    for s in range(3):
        lo, hi = p.update_box(COALESCED, s)
        assert tuple(v - 3 for v in lo) == want[s][0]
        assert tuple(v - 3 for v in hi) == want[s][1]


def test_gt_level_must_be_one_to_three():
    p = make((3, 3, 3), (0, 1, 2), 3)
    for bad in (0, 4, -1):
        with pytest.raises(ValueError):
            p.set_gt_level(bad)


def face_distance(n, order):
    """Per local cell (x fastest): distance to the nearest face along the
    second and along the third swept axis."""
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    c = [x.reshape(-1), y.reshape(-1), z.reshape(-1)]
    dist = [np.minimum(c[a], n[a] - 1 - c[a]) for a in range(3)]
    return np.minimum(dist[order[1]], dist[order[2]])


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("order", [(0, 1, 2), (2, 0, 1)])
def test_limited_levels_equal_gt3_away_from_stale_layers(order, k):
    """One step.  The first shear reads only freshly updated ghosts; the later
    shears read up to 3 cells beyond the local face, of which only k were
    recomputed, so a local cell is exact (bitwise, lists included) when it
    lies at least 3 - k cells inside the faces of the second and third swept
    axes; nearer the faces the stale layers show."""
    n = (9, 8, 10)
    st0 = random_state(n, KW["nblk"], 71, density=0.45, zero_frac=0.1)
    ref = make(n, order, 3)
    lim = make(n, order, k)
    for p in (ref, lim):
        p.load_local(*st0)
        p.fill_ghosts()
    sr = ref.step(1.0, COALESCED)
    sl = lim.step(1.0, COALESCED)
    NB = int(np.prod(KW["nblk"]))
    a, b = ref.export_local(), lim.export_local()
    la, lb = [set(a[1][a[0][c]:a[0][c + 1]]) for c in range(a[0].size - 1)], \
             [set(b[1][b[0][c]:b[0][c + 1]]) for c in range(b[0].size - 1)]
    da, db = to_dense(*a, NB), to_dense(*b, NB)
    dist = face_distance(n, order)
    inner = dist >= 3 - k
    assert inner.any() and (~inner).any()
    assert all(la[c] == lb[c] for c in np.nonzero(inner)[0])
    assert np.array_equal(da[inner], db[inner])
    assert not np.array_equal(da[~inner], db[~inner])
    # fewer computed updates in the first two shears, the same in the last
    assert sl["updates"][0] < sr["updates"][0] and sl["updates"][1] < sr["updates"][1]
    assert sl["updates"][2] == sr["updates"][2]


@pytest.mark.parametrize("k", [1, 2, 3])
def test_dense_update_counts_are_the_box_volumes(k):
    """With every block present, the updated phase-space cells of shear s are
    |U_s| * 64 * blocks: U_1 = n1 (n2 + 2k)(n3 + 2k), U_2 = n1 n2 (n3 + 2k),
    U_3 = n1 n2 n3 (axes in sweep order)."""
    n = (4, 5, 6)
    order = (2, 0, 1)
    nblk = (2, 2, 2)
    NB = 8
    p = OraclePartition(n, nblk, (4.0, 5.0, 7.0), (-4.0,) * 3, (1.0,) * 3, order, 0.0, 0)
    p.set_gt_level(k)
    rng = np.random.default_rng(5)
    nc = int(np.prod(n))
    off = np.arange(nc + 1, dtype=np.int64) * NB
    ids = np.tile(np.arange(NB, dtype=np.int32), nc)
    p.load_local(off, ids, rng.uniform(0.5, 1.5, nc * NB * 64))
    p.fill_ghosts()
    st = p.step(1.0, COALESCED)
    m = [n[d] for d in order]
    want = [m[0] * (m[1] + 2 * k) * (m[2] + 2 * k), m[0] * m[1] * (m[2] + 2 * k), m[0] * m[1] * m[2]]
    assert st["updates"] == tuple(v * NB * 64 for v in want)

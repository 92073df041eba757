"""Several partitions on one GPU (the sharded layout of the paper's MPI
decomposition, Section 3): a 2 x 2 x 2 split of a periodic box whose
partitions take their ghost domains from each other with one coalesced ghost
update per step gives the single partition's result bit for bit."""
import numpy as np
import pytest

from paper_2504_21450_amd import binding as B
from paper_2504_21450_amd import workloads as W
from gpuhelp import compare_states, gpu_partition, need_gpu, print_case, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def box_cells(n, lo, size):
    z, y, x = np.meshgrid(*[np.arange(lo[d], lo[d] + size[d]) for d in (2, 1, 0)], indexing="ij")
    return (x + n[0] * (y + n[1] * z)).reshape(-1)


def split(w, grid, gt_level=3):
    sub = tuple(w.n[d] // grid[d] for d in range(3))
    parts = {}
    for k in range(grid[2]):
        for j in range(grid[1]):
            for i in range(grid[0]):
                cells = box_cells(w.n, (i * sub[0], j * sub[1], k * sub[2]), sub)
                off, ids, f = W.take_cells(w.offsets, w.ids, w.f, cells)
                parts[(i, j, k)] = (B.Partition(sub, w.nblk, w.dx, w.vmin, w.dv, off, ids, f,
                                                storage=w.storage, order=w.order,
                                                sparse_min=w.sparse_min, vbuffer=w.vbuffer,
                                                gt_level=gt_level, slack=6.0), cells)
    return parts


def neighbours(parts, grid, key):
    out = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                q = ((key[0] + dx) % grid[0], (key[1] + dy) % grid[1], (key[2] + dz) % grid[2])
                out.append(parts[q][0])
    return out


@pytest.mark.parametrize("gt_level", [3])
def test_split_partitions_equal_single_partition_bitwise(gt_level):
    """GT3 only: GT1 and GT2 leave stale layers at every partition face, so
    their results depend on where the faces are."""
    w = W.maxwellian_sparse(n=(8, 6, 8), threads=8)
    grid = (2, 2, 2)
    print_case("2x2x2 split of 8x6x8, GT%d" % gt_level)
    # steep fields on a small box: lists grow by ~2x in the first step
    single = gpu_partition(w, gt_level=gt_level, slack=6.0)
    parts = split(w, grid, gt_level)
    for _ in range(3):
        single.fill_ghosts()
        single.step(w.dt, B.VL_COALESCED)
        for key, (p, _) in parts.items():       # every ghost update before any shear
            p.fill_ghosts_from(neighbours(parts, grid, key))
        for p, _ in parts.values():
            p.step(w.dt, B.VL_COALESCED)
    o, _ = run_oracle(w, 3)
    oo, oi, of = o.export_local()
    for key, (p, cells) in parts.items():
        got = p.export()
        want = single.export_cells(cells)
        assert all(np.array_equal(a, b) for a, b in zip(got, want)), key
        # and against the oracle's periodic whole box: lists exact, values to 1e-12
        compare_states(got, W.take_cells(oo, oi, of, cells), 1e-12)


def test_fill_from_checks_its_neighbours():
    w = W.maxwellian_sparse(n=(6, 6, 6), threads=8)
    parts = split(w, (2, 2, 2))
    p = parts[(0, 0, 0)][0]
    nb = neighbours(parts, (2, 2, 2), (0, 0, 0))
    other = gpu_partition(W.maxwellian_sparse(n=(4, 3, 3), threads=8))
    bad = list(nb)
    bad[13] = parts[(1, 0, 0)][0]
    assert p.lib.vl_fill_ghosts_from(p.h, (B.C.c_void_p * 27)(*[q.h.value for q in bad])) == B.VL_ERR_ARG
    bad = list(nb)
    bad[0] = other
    assert p.lib.vl_fill_ghosts_from(p.h, (B.C.c_void_p * 27)(*[q.h.value for q in bad])) == B.VL_ERR_ARG
    p.fill_ghosts_from(nb)
    p.step(w.dt)
    p.sync()


def test_autotune_on_a_split_partition_equals_ordinary_steps():
    """The autotuner's real steps take their ghost update from the stored
    neighbour sources, as an ordinary step after vl_fill_ghosts_from does (the
    neighbours stay where they are in both runs)."""
    w = W.maxwellian_sparse(n=(8, 6, 8), threads=8)
    grid = (2, 2, 2)
    print_case("autotune on one partition of a 2x2x2 split")
    a_parts = split(w, grid)
    b_parts = split(w, grid)
    key = (1, 0, 1)
    a = a_parts[key][0]
    b = b_parts[key][0]
    a.fill_ghosts_from(neighbours(a_parts, grid, key))
    a.step(w.dt, B.VL_COALESCED)
    best, ms = a.autotune(w.dt, B.VL_COALESCED, steps_per_variant=1)
    nvar = len(ms)
    nb = neighbours(b_parts, grid, key)
    for _ in range(1 + nvar):
        b.fill_ghosts_from(nb)
        b.step(w.dt, B.VL_COALESCED)
    assert all(np.array_equal(x, y) for x, y in zip(a.export(), b.export()))

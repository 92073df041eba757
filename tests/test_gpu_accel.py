"""The acceleration step on the GPU (vl_accelerate: the Lorentz-force half of
the split Vlasov step, three SLICE-3D velocity remaps with the CW84
parabolas) against the oracle's vlo_accelerate on the same seeded inputs.

FP64: block lists bit-exact, values within 1e-12 relative max-norm, the mass
before, after and pruned within 1e-12 of the oracle's; an exact shift (B = 0,
whole velocity cells per step) equal bit for bit.  Fields are per cell: a
magnetic field of random direction and 0.5-1.5 x 10 nT, a perpendicular
E x B drift of up to ~3e5 m/s and a parallel electric field moving up to
two velocity cells; dt gives gyration angles of 0.15-0.45 rad.  Cases: two
slice orders, two steps in a row, steps interleaved with translation steps,
pruning off (the list is the old one plus every nonzero block), the
26-neighbour buffer, a drift of many blocks (lists grow past their places),
empty cells, determinism, reduced storage against the oracle run from the
stored (widened) state, and the refusals (a map that cannot be split, a
velocity mesh beyond the kernel's limits)."""
import dataclasses
import math

import numpy as np
import pytest
import torch

from oracle import OraclePartition
from paper_2504_21450_amd import binding as B
from paper_2504_21450_amd import workloads as W
from gpuhelp import compare_states, gpu_partition, need_gpu, print_case, run_gpu
from statehelp import to_dense

pytestmark = pytest.mark.gpu
QM = 9.58e7        # proton charge-to-mass ratio [C/kg]
B0 = 1e-8          # [T]
DT = 0.3 / (QM * B0)


@pytest.fixture(scope="module")
def sparse_small():
    need_gpu()
    return W.maxwellian_sparse(n=(6, 5, 4), threads=8)


def random_fields(ncell, seed, vdrift=3e5, vpar=6e4, dt=DT):
    """(ncell, 6) Ex, Ey, Ez, Bx, By, Bz: B of random direction and 0.5-1.5
    B0, E = -Vd x B + E_par b with Vd perpendicular to B and |Vd| ~ vdrift,
    and E_par moving up to vpar in dt."""
    rng = np.random.default_rng(seed)
    b = rng.normal(size=(ncell, 3))
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    Bv = b * (B0 * rng.uniform(0.5, 1.5, ncell))[:, None]
    Vd = rng.normal(size=(ncell, 3)) * vdrift / np.sqrt(3.0)
    Vd -= np.sum(Vd * b, axis=1, keepdims=True) * b
    Epar = rng.uniform(-1.0, 1.0, ncell) * vpar / (QM * dt)
    E = -np.cross(Vd, Bv) + Epar[:, None] * b
    return np.concatenate([E, Bv], 1)


def dev(EB):
    return torch.tensor(np.ascontiguousarray(EB).reshape(-1), dtype=torch.float64, device="cuda:0")


def oracle_of(w, order=None):
    return OraclePartition.from_workload(w, order=order)


def check_stats(gs, os_, p=None, w=None):
    """Pruned mass against the oracle's to 1e-12 of the mass; the mass lost
    off the velocity mesh (before - after - pruned) against the oracle's to
    1e-11 (the oracle adds its ~1e6 values one after another, a rounding of
    order 1e-12 in each of its totals); the GPU's mass after the step
    against a compensated sum of its exported values to 1e-13."""
    m = gs["mass_before"]
    assert abs(gs["pruned_mass"] - os_["pruned_mass"]) <= 1e-12 * m
    lost_g = gs["mass_before"] - gs["mass_after"] - gs["pruned_mass"]
    lost_o = os_["mass_before"] - os_["mass_after"] - os_["pruned_mass"]
    assert abs(lost_g - lost_o) <= 1e-11 * m, (lost_g / m, lost_o / m)
    assert gs["blocks"] == os_["blocks"]
    if p is not None:
        vol = float(np.prod(w.dx) * np.prod(w.dv))
        exact = math.fsum(p.export()[2].tolist()) * vol
        assert abs(gs["mass_after"] - exact) <= 1e-13 * m


@pytest.mark.parametrize("order", [(0, 1, 2), (2, 0, 1)])
def test_two_acceleration_steps_match_the_oracle(sparse_small, order):
    w = sparse_small
    print_case("acceleration, slice order %s" % (order,))
    p = gpu_partition(w)
    o = oracle_of(w)
    for k in range(2):
        EB = random_fields(p.ncell, 100 + k)
        gs = p.accelerate(DT, QM, dev(EB), order=order, stats=True)
        os_ = o.accelerate(DT, QM, EB, order=order)
        err = compare_states(p.export(), o.export_local(), 1e-12)
        check_stats(gs, os_, p, w)
        print("step %d: max rel err %.3e, blocks %d, pruned %.3e, lost %.3e" % (
            k, err, gs["blocks"], gs["pruned_mass"] / gs["mass_before"],
            (gs["mass_before"] - gs["mass_after"] - gs["pruned_mass"]) / gs["mass_before"]))


def test_acceleration_interleaved_with_translation(sparse_small):
    """translate, accelerate, translate, accelerate: both halves of the
    split step one after the other, against the oracle doing the same."""
    w = sparse_small
    print_case("translation and acceleration interleaved")
    p = gpu_partition(w)
    o = oracle_of(w)
    for k in range(2):
        run_gpu(p, w.dt, 1)
        o.fill_ghosts()
        o.step(w.dt)
        EB = random_fields(p.ncell, 200 + k)
        p.accelerate(DT, QM, dev(EB))
        o.accelerate(DT, QM, EB)
    compare_states(p.export(), o.export_local(), 1e-12)


def test_acceleration_without_pruning_keeps_old_and_nonzero_blocks(sparse_small):
    w = dataclasses.replace(sparse_small, sparse_min=0.0)
    print_case("acceleration, pruning off")
    p = gpu_partition(w)
    o = oracle_of(w)
    EB = random_fields(p.ncell, 300)
    gs = p.accelerate(DT, QM, dev(EB), stats=True)
    os_ = o.accelerate(DT, QM, EB)
    compare_states(p.export(), o.export_local(), 1e-12)
    check_stats(gs, os_)
    assert gs["pruned_mass"] == 0.0


def test_acceleration_with_the_26_neighbour_buffer(sparse_small):
    w = dataclasses.replace(sparse_small, vbuffer=26)
    print_case("acceleration, 26-neighbour buffer")
    p = gpu_partition(w)
    o = oracle_of(w)
    EB = random_fields(p.ncell, 400)
    gs = p.accelerate(DT, QM, dev(EB), order=(1, 2, 0), stats=True)
    os_ = o.accelerate(DT, QM, EB, order=(1, 2, 0))
    compare_states(p.export(), o.export_local(), 1e-12)
    check_stats(gs, os_)


def test_electric_shift_by_whole_cells_is_exact(sparse_small):
    """B = 0 and qm E dt a whole number of cells per axis: every column moves
    by whole cells, the same bits as the oracle's exact shift."""
    w = sparse_small
    print_case("acceleration, exact electric shift")
    p = gpu_partition(w)
    o = oracle_of(w)
    shift = np.array([3, -2, 5])
    E = shift * np.array(w.dv) / (QM * DT)
    EB = np.tile(np.concatenate([E, [0.0, 0.0, 0.0]]), (p.ncell, 1))
    p.accelerate(DT, QM, dev(EB))
    o.accelerate(DT, QM, EB)
    ga, oa = p.export(), o.export_local()
    assert all(np.array_equal(x, y) for x, y in zip(ga, oa))


def test_drift_of_many_blocks_grows_the_lists(sparse_small):
    """A drift of ~6 blocks along x and ~5 along z (not whole cells): most
    blocks of a cell are created in the step, beyond the list's place."""
    w = sparse_small
    print_case("acceleration, drift of many blocks")
    p = gpu_partition(w)
    o = oracle_of(w)
    E = np.array([6.3, 0.0, -4.7]) * 4 * np.array(w.dv) / (QM * DT)
    EB = np.tile(np.concatenate([E, [0.0, 0.0, 0.0]]), (p.ncell, 1))
    gs = p.accelerate(DT, QM, dev(EB), stats=True)
    os_ = o.accelerate(DT, QM, EB)
    compare_states(p.export(), o.export_local(), 1e-12)
    check_stats(gs, os_)


def test_empty_cells_and_determinism(sparse_small):
    w = sparse_small
    counts = np.diff(w.offsets)
    keep = np.ones(counts.size, bool)
    keep[::3] = False                      # every third cell empty
    ids, fs, off = [], [], [0]
    for c in range(counts.size):
        a, b = w.offsets[c], w.offsets[c + 1]
        if keep[c]:
            ids.append(w.ids[a:b])
            fs.append(w.f[a * 64:b * 64])
        off.append(off[-1] + (b - a if keep[c] else 0))
    w2 = dataclasses.replace(w, offsets=np.array(off, np.int64), ids=np.concatenate(ids),
                             f=np.concatenate(fs))
    print_case("acceleration, empty cells, two runs")
    EB = random_fields(int(np.prod(w.n)), 500)
    runs = []
    for _ in range(2):
        p = gpu_partition(w2)
        p.accelerate(DT, QM, dev(EB))
        runs.append(p.export())
    assert all(np.array_equal(x, y) for x, y in zip(*runs))
    o = oracle_of(w2)
    o.accelerate(DT, QM, EB)
    compare_states(runs[0], o.export_local(), 1e-12)


@pytest.mark.parametrize("storage,tol", [(B.VL_F32, 3e-7), (B.VL_BF16, 3 * 2.0 ** -8)])
def test_reduced_storage_against_the_oracle(sparse_small, storage, tol):
    """FP32 / BF16 storage, FP64 arithmetic: the oracle starts from the
    stored (widened) state; each of the three remaps rounds once to the
    storage type (2^-24 / 2^-9 of a value, relative to the largest value).
    Compared over the union of the lists (absent blocks read as zero)."""
    w = sparse_small
    print_case("acceleration, storage %d" % storage)
    p = gpu_partition(w, storage=storage)
    o = OraclePartition(w.n, w.nblk, w.dx, w.vmin, w.dv, w.order, w.sparse_min, w.vbuffer)
    o.load_local(*p.export())
    EB = random_fields(p.ncell, 600)
    gs = p.accelerate(DT, QM, dev(EB), stats=True)
    o.accelerate(DT, QM, EB)
    NB = int(np.prod(w.nblk))
    g, r = to_dense(*p.export(), NB), to_dense(*o.export_local(), NB)
    err = np.max(np.abs(g - r)) / np.max(np.abs(r))
    print("storage %d: max rel err %.3e" % (storage, err))
    assert err <= tol
    assert np.min(p.export()[2]) >= 0.0


def test_map_that_cannot_be_split_is_refused(sparse_small):
    """A rotation by more than half a turn in one step: VL_ERR_SPLIT, f and
    the lists unchanged, the partition still usable."""
    w = sparse_small
    print_case("acceleration, refused rotation")
    p = gpu_partition(w)
    before = p.export()
    EB = random_fields(p.ncell, 700)
    EB[5, 3:] = np.array([0.0, 0.0, 3.5 / (QM * DT)])   # one cell turns by 3.5 rad
    assert p.accelerate_rc(DT, QM, dev(EB)) == B.VL_ERR_SPLIT
    assert all(np.array_equal(x, y) for x, y in zip(before, p.export()))
    EB[5, 3:] = np.array([0.0, 0.0, B0])
    p.accelerate(DT, QM, dev(EB))


def test_velocity_mesh_beyond_the_kernel_is_refused():
    need_gpu()
    n, nblk = (2, 2, 2), (65, 2, 2)
    off = np.zeros(9, np.int64)
    p = B.Partition(n, nblk, (1e5,) * 3, (-1e6,) * 3, (1e4,) * 3, off, np.zeros(0, np.int32),
                    np.zeros(0), block_capacity=64, ghost_block_capacity=64)
    EB = np.zeros((8, 6))
    assert p.accelerate_rc(1.0, QM, dev(EB)) == B.VL_ERR_ARG


@pytest.mark.parametrize("storage", [B.VL_F32, B.VL_BF16])
def test_reduced_storage_translation_and_acceleration_alternate(sparse_small, storage):
    """Translation steps (per-line rounding ledger, re-injected at the next
    shear along each axis) alternating with acceleration steps (which prune
    blocks the ledger stores still name): every translation step balances
    stored + pruned + ledger mass to 1e-12, every acceleration step's mass
    change is what left the mesh plus what was pruned plus one rounding of
    each value per remap; the run is the same bit for bit twice."""
    w = sparse_small
    print_case("translation and acceleration alternating, storage %d" % storage)
    ulp = 2.0 ** -24 if storage == B.VL_F32 else 2.0 ** -9
    finals = []
    for _ in range(2):
        p = gpu_partition(w, storage=storage)
        for k in range(3):
            s = run_gpu(p, w.dt, 1, stats=True)[0]
            bal = s["mass_before"] - (s["mass_after"] + s["pruned_mass"] + s["ledger_mass"])
            assert abs(bal) <= 1e-12 * s["mass_before"], bal / s["mass_before"]
            a = p.accelerate(DT, QM, dev(random_fields(p.ncell, 800 + k)), stats=True)
            rest = a["mass_before"] - a["mass_after"] - a["pruned_mass"]
            assert abs(rest) <= 3 * ulp * a["mass_before"], rest / a["mass_before"]
            assert np.min(p.export()[2]) >= 0.0
        finals.append(p.export())
    assert all(np.array_equal(x, y) for x, y in zip(*finals))

"""Parity of the HIP translation path (through the C ABI) with the FP64
oracle: values within 1e-12 relative max-norm, block lists bit-exact, the two
ghost schemes bit-identical, and the error paths."""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle import OraclePartition
from paper_2504_21450_amd import binding as B
from paper_2504_21450_amd import workloads as W
from gpuhelp import compare_states, gpu_partition, need_gpu, print_case, run_gpu, run_oracle
from statehelp import random_state, roll_cells, to_dense

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.fixture(scope="module")
def sparse_small():
    return W.maxwellian_sparse(n=(6, 5, 4), threads=8)


def test_dense_maxwellian_ten_steps_match_oracle():
    """8^3 periodic cells, dense 16^3 velocity mesh, 10 coalesced steps."""
    w = W.maxwellian_small()
    print_case("dense maxwellian 8x8x8, 10 steps")
    p = gpu_partition(w)
    run_gpu(p, w.dt, w.steps)
    o, _ = run_oracle(w, w.steps)
    compare_states(p.export(), o.export_local(), TOL64)


def test_sparse_maxwellians_match_oracle(sparse_small):
    w = sparse_small
    print_case("sparse maxwellian 6x5x4, 3 steps, pruning on")
    p = gpu_partition(w)
    gs = run_gpu(p, w.dt, 3, stats=True)
    o, os_ = run_oracle(w, 3)
    compare_states(p.export(), o.export_local(), TOL64)
    for g, r in zip(gs, os_):
        assert g["updated_ps"] == r["updates"]
        assert g["blocks"] == r["blocks"]
        assert abs(g["pruned_mass"] - r["pruned_mass"]) <= 1e-12 * r["mass_before"]


@pytest.mark.parametrize("order", [(0, 1, 2), (2, 0, 1), (1, 2, 0)])
def test_random_sparse_states_all_orders(order):
    n, nblk = (5, 4, 6), (3, 2, 3)
    st = random_state(n, nblk, 31, density=0.35, zero_frac=0.1)
    w = W.Workload("random", n, (6.0, 5.0, 7.0), nblk, (-6.0, -4.0, -6.0), (1.0, 1.0, 1.0), 1.0, 3,
                   2.5e-10, 6, B.VL_F64, order, *st)
    print_case("random sparse order=%s" % (order,))
    p = gpu_partition(w)
    run_gpu(p, w.dt, 3)
    o, _ = run_oracle(w, 3)
    compare_states(p.export(), o.export_local(), TOL64)


def test_ghost_translation_equals_classical_bitwise(sparse_small):
    w = sparse_small
    print_case("coalesced vs per-sweep, sparse 6x5x4")
    a = gpu_partition(w)
    b = gpu_partition(w)
    sa = run_gpu(a, w.dt, 3, B.VL_COALESCED, stats=True)
    sb = run_gpu(b, w.dt, 3, B.VL_PER_SWEEP, stats=True)
    ea, eb = a.export(), b.export()
    assert all(np.array_equal(x, y) for x, y in zip(ea, eb))
    # the coalesced scheme computes more (ghost cells of later shears)
    assert sa[-1]["updated_ps"][0] > sb[-1]["updated_ps"][0]
    assert sa[-1]["updated_ps"][2] == sb[-1]["updated_ps"][2]


@pytest.mark.parametrize("shift", [(1, 0, -1), (-1, 1, 1)])
def test_integer_courant_shift(shift):
    n, nblk = (5, 4, 6), (2, 2, 2)
    st = random_state(n, nblk, 32, density=0.4)
    w = W.Workload("shift", n, (4.0, 5.0, 7.0), nblk, (-4.0,) * 3, (1.0,) * 3, 1.0, 1, 0.0, 0,
                   B.VL_F64, (0, 1, 2), *st)
    print_case("integer courant shift %s" % (shift,))
    p = gpu_partition(w)
    table = np.zeros((3, 8))
    for d in range(3):
        table[d] = shift[d]
    p.set_courant_override(table)
    run_gpu(p, 1.0, 1)
    got = to_dense(*p.export(), 8)
    want = roll_cells(to_dense(*st, 8), n, shift)
    assert np.max(np.abs(got - want)) <= 4 * np.finfo(float).eps * np.max(st[2])


def test_mass_ledger_and_moments(sparse_small):
    w = sparse_small
    print_case("mass ledger and moments")
    p = gpu_partition(w)
    s = run_gpu(p, w.dt, 2, stats=True)
    for st in s:
        assert abs(st["mass_after"] + st["pruned_mass"] - st["mass_before"]) <= 1e-12 * st["mass_before"]
    o, _ = run_oracle(w, 2)
    dn, dV, dP, tot = p.moments()
    on, oV, oP, otot = o.moments()
    dn, dV, dP = dn.cpu().numpy(), dV.cpu().numpy(), dP.cpu().numpy()
    assert np.max(np.abs(dn - on)) <= 1e-12 * np.max(on)
    vth = np.sqrt(np.max(np.abs(oP[:, :3])) / (1.67262192e-27 * np.min(on)))
    assert np.max(np.abs(dV - oV)) <= 1e-12 * max(np.max(np.abs(oV)), vth)
    assert np.max(np.abs(dP - oP)) <= 1e-11 * np.max(np.abs(oP[:, :3]))
    assert abs(tot - otot) <= 1e-12 * otot


def test_runs_are_deterministic(sparse_small):
    w = sparse_small
    print_case("determinism")
    a = gpu_partition(w)
    b = gpu_partition(w)
    run_gpu(a, w.dt, 2)
    run_gpu(b, w.dt, 2)
    assert all(np.array_equal(x, y) for x, y in zip(a.export(), b.export()))


def test_restart_from_exported_state(sparse_small):
    w = sparse_small
    print_case("restart")
    a = gpu_partition(w)
    run_gpu(a, w.dt, 3)
    b = gpu_partition(w)
    run_gpu(b, w.dt, 1)
    o, i, f = b.export()
    c = B.Partition(w.n, w.nblk, w.dx, w.vmin, w.dv, o, i, f, sparse_min=w.sparse_min, vbuffer=w.vbuffer)
    run_gpu(c, w.dt, 2)
    assert all(np.array_equal(x, y) for x, y in zip(a.export(), c.export()))


def test_export_cells_matches_export(sparse_small):
    w = sparse_small
    p = gpu_partition(w)
    run_gpu(p, w.dt, 1)
    full = p.export()
    cells = np.array([0, 7, 33, 119, 5])
    o, i, f = p.export_cells(cells)
    for k, c in enumerate(cells):
        a0, a1 = full[0][c], full[0][c + 1]
        assert np.array_equal(i[o[k]:o[k + 1]], full[1][a0:a1])
        assert np.array_equal(f[o[k] * 64:o[k + 1] * 64], full[2][a0 * 64:a1 * 64])


def test_error_codes(sparse_small):
    w = sparse_small
    print_case("error codes")
    p = gpu_partition(w)
    assert p.step_rc(w.dt) == B.VL_ERR_STALE_GHOSTS
    p.fill_ghosts()
    assert p.step_rc(w.dt * 2.1) == B.VL_ERR_CFL
    assert p.step_rc(w.dt) == B.VL_OK
    assert p.step_rc(w.dt) == B.VL_ERR_STALE_GHOSTS
    assert p.step_rc(w.dt, B.VL_PER_SWEEP) == B.VL_OK
    p.sync()


def test_capacity_overflow_is_reported():
    """A block pool with no room for growth: the device records the overflow
    and the next synchronising call reports it."""
    n, nblk = (4, 4, 4), (2, 2, 2)
    st = random_state(n, nblk, 33, density=0.3)
    nb = int(st[0][-1])
    p = B.Partition(n, nblk, (4.0, 5.0, 7.0), (-4.0,) * 3, (1.0,) * 3, *st, block_capacity=nb)
    p.fill_ghosts()
    with pytest.raises(B.VlasovError) as e:
        p.step(1.0, stats=True)
    assert e.value.status == B.VL_ERR_CAPACITY
    assert p.step_rc(1.0, B.VL_PER_SWEEP) == B.VL_ERR_STATE


def test_kernels_stop_after_a_capacity_error():
    """Fail-stop: after the device records an overflow, the steps, graph
    replays and moments already enqueued do nothing (no kernel reads the
    inconsistent lists), and the next synchronising call reports the error."""
    n, nblk = (4, 4, 4), (2, 2, 2)
    st = random_state(n, nblk, 33, density=0.3)
    nb = int(st[0][-1])
    p = B.Partition(n, nblk, (4.0, 5.0, 7.0), (-4.0,) * 3, (1.0,) * 3, *st, block_capacity=nb)
    print_case("steps after a capacity error")
    for _ in range(4):
        assert p.lib.vl_fill_ghosts(p.h) == B.VL_OK
        assert p.step_rc(1.0, B.VL_COALESCED) == B.VL_OK      # asynchronous: no check yet
    assert p.lib.vl_graph_step(p.h, 1.0, B.VL_COALESCED, 2) == B.VL_OK
    p.moments(total=False)                                   # asynchronous as well
    assert p.lib.vl_sync(p.h) == B.VL_ERR_CAPACITY
    assert p.lib.vl_sync(p.h) == B.VL_ERR_STATE


def test_all_shear_variants_and_autotuner_are_bit_identical(sparse_small):
    """Every compiled shear variant (store scheme, prefetch depth, occupancy)
    gives the same state bit for bit, so the autotuner's real steps leave the
    trajectory unchanged."""
    w = sparse_small
    print_case("shear variants")
    ref = gpu_partition(w)
    run_gpu(ref, w.dt, 2)
    want = ref.export()
    nvar = 0
    for v in range(64):
        p = gpu_partition(w)
        try:
            p.set_variant(v)
        except B.VlasovError:
            break
        nvar += 1
        run_gpu(p, w.dt, 2)
        assert all(np.array_equal(x, y) for x, y in zip(p.export(), want)), v
    assert nvar >= 4
    a = gpu_partition(w)
    best, ms = a.autotune(w.dt, B.VL_COALESCED, steps_per_variant=1)
    assert len(best) == 3 and all(0 <= v < nvar for v in best) and len(ms) == nvar
    assert a.variants() == (best, nvar)
    b = gpu_partition(w)
    run_gpu(b, w.dt, nvar)
    assert all(np.array_equal(x, y) for x, y in zip(a.export(), b.export()))
    # two steps per variant: a first round over all, then rounds over the
    # variants near the best; the same number of steps in all
    a = gpu_partition(w)
    best, ms = a.autotune(w.dt, B.VL_COALESCED, steps_per_variant=2)
    assert all(0 <= v < nvar for v in best) and len(ms) == nvar and min(ms) > 0
    b = gpu_partition(w)
    run_gpu(b, w.dt, 2 * nvar)
    assert all(np.array_equal(x, y) for x, y in zip(a.export(), b.export()))


def test_per_shear_variants_mix_bit_identically(sparse_small):
    """Each shear of the order may run its own variant (the third shear's
    kernels also record the content flags): mixed choices give the state of
    one variant bit for bit; out-of-range choices are refused and change
    nothing."""
    w = sparse_small
    print_case("per-shear variants")
    ref = gpu_partition(w)
    run_gpu(ref, w.dt, 2)
    want = ref.export()
    _, nvar = ref.variants()
    for vs in [(nvar - 1, 0, 4), (6, nvar - 1, 2), (1, 4, nvar - 1)]:
        p = gpu_partition(w)
        p.set_variant(vs)
        assert p.variants() == (vs, nvar)
        run_gpu(p, w.dt, 2)
        assert all(np.array_equal(x, y) for x, y in zip(p.export(), want)), vs
    p = gpu_partition(w)
    p.set_variant((2, 3, 4))
    for bad in [(0, 0, nvar), (-1, 0, 0), (0, 64, 0)]:
        with pytest.raises(B.VlasovError):
            p.set_variant(bad)
        assert p.variants() == ((2, 3, 4), nvar)
    with pytest.raises(ValueError):
        p.set_variant((1, 2))


@pytest.mark.parametrize("k", [1, 2])
def test_limited_ghost_translation_levels_match_oracle(sparse_small, k):
    """GT1 / GT2 (Section 3.2): the device leaves the same ghost layers at
    their ghost-update values as the oracle; values within 1e-12, lists exact."""
    w = sparse_small
    print_case("GT%d vs oracle" % k)
    p = gpu_partition(w, gt_level=k)
    gs = run_gpu(p, w.dt, 2, stats=True)
    o = OraclePartition.from_workload(w, gt_level=k)
    os_ = []
    for _ in range(2):
        o.fill_ghosts()
        os_.append(o.step(w.dt))
    compare_states(p.export(), o.export_local(), TOL64)
    for g, r in zip(gs, os_):
        assert g["updated_ps"] == r["updates"]


def test_long_pencils_with_gaps_match_oracle_for_every_variant():
    """Pencils 54 cells long whose blocks come and go at random, so the gaps
    between the cells holding a block take every length: each shear variant
    against the oracle, with the mass balance."""
    n, nblk = (48, 4, 3), (2, 2, 2)
    st = random_state(n, nblk, 77, density=0.3, zero_frac=0.0)
    w = W.Workload("gaps", n, (4.0, 5.0, 7.0), nblk, (-4.0,) * 3, (1.0,) * 3, 1.0, 2, 0.0, 0,
                   B.VL_F64, (0, 1, 2), *st)
    print_case("long pencils with gaps, every variant")
    o, _ = run_oracle(w, 2)
    want = o.export_local()
    for v in range(64):
        p = gpu_partition(w)
        try:
            p.set_variant(v)
        except B.VlasovError:
            break
        s = run_gpu(p, w.dt, 2, stats=True)
        compare_states(p.export(), want, TOL64)
        for x in s:
            assert abs(x["mass_after"] + x["pruned_mass"] - x["mass_before"]) <= 1e-12 * x["mass_before"], v


@pytest.mark.parametrize("order", [(0, 1, 2), (2, 0, 1)])
def test_26_neighbour_velocity_buffer_matches_oracle(sparse_small, order):
    """Pruning with all 26 velocity-space neighbours kept around the content
    blocks: values within 1e-12, lists exact, the same block counts, updated
    cells and pruned mass as the oracle."""
    w = dataclasses.replace(sparse_small, vbuffer=26, order=order)
    print_case("26-neighbour buffer, order %s" % (order,))
    p = gpu_partition(w)
    gs = run_gpu(p, w.dt, 3, stats=True)
    o, os_ = run_oracle(w, 3)
    compare_states(p.export(), o.export_local(), TOL64)
    for g, r in zip(gs, os_):
        assert g["updated_ps"] == r["updates"]
        assert g["blocks"] == r["blocks"]
        assert abs(g["pruned_mass"] - r["pruned_mass"]) <= 1e-12 * r["mass_before"]


def test_26_neighbour_buffer_at_the_mesh_edges():
    """Random content on a 3 x 2 x 3-block mesh, so content blocks sit on the
    faces, edges and corners of the velocity mesh and the buffer is clipped
    there."""
    n, nblk = (5, 4, 6), (3, 2, 3)
    st = random_state(n, nblk, 35, density=0.3, zero_frac=0.2)
    w = W.Workload("random26", n, (6.0, 5.0, 7.0), nblk, (-6.0, -4.0, -6.0), (1.0, 1.0, 1.0), 1.0, 3,
                   6e-10, 26, B.VL_F64, (0, 1, 2), *st)
    print_case("26-neighbour buffer, random content at the mesh edges")
    p = gpu_partition(w)
    gs = run_gpu(p, w.dt, 3, stats=True)
    o, os_ = run_oracle(w, 3)
    compare_states(p.export(), o.export_local(), TOL64)
    assert any(r["pruned_mass"] > 0 for r in os_)
    for g, r in zip(gs, os_):
        assert g["blocks"] == r["blocks"]

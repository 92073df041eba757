"""Whole steps replayed from recorded HIP graphs (vl_graph_step) against
ordinary launches: every replay gives the same state bit for bit, with the
program's own work (moments, exports, synchronisation, ordinary steps)
between replays."""
import numpy as np
import pytest

from paper_2504_21450_amd import binding as B
from paper_2504_21450_amd import workloads as W
from gpuhelp import compare_states, gpu_partition, need_gpu, print_case, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.fixture(scope="module")
def sparse_small():
    return W.maxwellian_sparse(n=(6, 5, 4), threads=8)


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a.export(), b.export()))


@pytest.mark.parametrize("mode", [B.VL_COALESCED, B.VL_PER_SWEEP])
def test_every_replay_equals_ordinary_steps(sparse_small, mode):
    w = sparse_small
    print_case("graph replays, mode %d" % mode)
    a = gpu_partition(w)
    g = gpu_partition(w)
    for k in range(5):
        run_gpu(a, w.dt, 1, mode)
        g.graph_step(w.dt, mode)
        g.moments()                 # ordinary launches and a synchronisation between replays
        assert same(a, g), "replay %d" % k
    # an ordinary step in between moves the list region; the next replays
    # take the other recorded graph
    run_gpu(a, w.dt, 1, mode)
    run_gpu(g, w.dt, 1, mode)
    run_gpu(a, w.dt, 2, mode)
    g.graph_step(w.dt, mode, nsteps=2)
    assert same(a, g)


def test_graph_steps_match_the_oracle(sparse_small):
    w = sparse_small
    print_case("graph replays against the oracle")
    g = gpu_partition(w)
    g.graph_step(w.dt, B.VL_COALESCED, nsteps=3)
    o, _ = run_oracle(w, 3)
    compare_states(g.export(), o.export_local(), 1e-12)


@pytest.mark.parametrize("storage", [B.VL_F32, B.VL_BF16])
def test_reduced_storage_replays(sparse_small, storage):
    """The per-line ledger stores rotate with a period of four steps and the
    list regions with two: replays through two rotations, then an ordinary
    step between replays (which shifts the recorded graph each replay takes),
    equal ordinary steps bit for bit, mass balance included."""
    w = sparse_small
    print_case("graph replays, storage %d" % storage)
    a = gpu_partition(w, storage=storage)
    g = gpu_partition(w, storage=storage)
    for k in range(8):
        run_gpu(a, w.dt, 1)
        g.graph_step(w.dt)
        assert same(a, g), "replay %d" % k
    run_gpu(a, w.dt, 1)
    run_gpu(g, w.dt, 1)
    run_gpu(a, w.dt, 5)
    g.graph_step(w.dt, nsteps=5)
    assert same(a, g)
    sa = run_gpu(a, w.dt, 1, stats=True)[-1]
    sg = run_gpu(g, w.dt, 1, stats=True)[-1]
    assert sa == sg


def test_recording_follows_dt_variant_and_courant_changes(sparse_small):
    w = sparse_small
    print_case("graph re-recording")
    a = gpu_partition(w)
    g = gpu_partition(w)
    dts = [w.dt, 0.5 * w.dt, 0.5 * w.dt, w.dt]
    for dt in dts:
        run_gpu(a, dt, 1)
        g.graph_step(dt)
    assert same(a, g)
    g.set_variant(1)
    a.set_variant(0)
    run_gpu(a, w.dt, 1)
    g.graph_step(w.dt)
    assert same(a, g)
    g.set_variant((4, 6, 2))  # per-shear choices are part of the recording
    run_gpu(a, w.dt, 1)
    g.graph_step(w.dt)
    assert same(a, g)
    table = np.zeros((3, 4 * max(w.nblk)))
    table[0] = 1.0
    table[1] = -1.0
    for p in (a, g):
        p.set_courant_override(table)
    run_gpu(a, 1.0, 1)
    g.graph_step(1.0)
    assert same(a, g)


def test_graph_step_errors(sparse_small):
    w = sparse_small
    g = gpu_partition(w)
    assert g.lib.vl_graph_step(g.h, w.dt * 2.1, B.VL_COALESCED, 1) == B.VL_ERR_CFL
    assert g.lib.vl_graph_step(g.h, w.dt, 7, 1) == B.VL_ERR_ARG
    assert g.lib.vl_graph_step(g.h, -w.dt, B.VL_COALESCED, 1) == B.VL_ERR_ARG
    assert g.lib.vl_graph_step(g.h, w.dt, B.VL_COALESCED, -1) == B.VL_ERR_ARG
    assert g.lib.vl_graph_step(g.h, w.dt, B.VL_COALESCED, 0) == B.VL_OK
    g.sync()

"""A partition at a simulation edge on the GPU: the boundary cells beyond
its x faces come from two partitions that are never stepped (their cells hold
the boundary contents), no Ghost Translation layers are computed beyond the
edge, and the result matches the oracle, the classical refresh and graph
replays."""
import numpy as np
import pytest

import oracle
from oracle import COALESCED, OraclePartition
from paper_2504_21450_amd import binding as B
from edgehelp import padded_with_boundaries
from gpuhelp import compare_states, need_gpu, print_case
from statehelp import random_state

pytestmark = pytest.mark.gpu
EDGES_X = 0b11
N, NBLK = (7, 5, 6), (3, 2, 3)
GEOM = dict(dx=(6.0, 5.0, 7.0), vmin=(-6.0, -4.0, -6.0), dv=(1.0, 1.0, 1.0))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.fixture(scope="module")
def states():
    return (random_state(N, NBLK, 41, density=0.4, zero_frac=0.1), random_state(N, NBLK, 42, density=0.4),
            random_state(N, NBLK, 43, density=0.4))


def part(st, edges, order=(0, 1, 2)):
    return B.Partition(N, NBLK, GEOM["dx"], GEOM["vmin"], GEOM["dv"], *st, order=order, sparse_min=2.5e-10,
                       vbuffer=6, edges=edges)


def table(p, lo, hi):
    out = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                out.append(lo if dx < 0 else hi if dx > 0 else p)
    return out


@pytest.mark.parametrize("order", [(0, 1, 2), (2, 0, 1)])
def test_edges_match_oracle_and_classical(states, order):
    st, lo_st, hi_st = states
    print_case("simulation edges on x, order %s" % (order,))
    lo, hi = part(lo_st, 0, order), part(hi_st, 0, order)
    a = part(st, EDGES_X, order)
    b = part(st, EDGES_X, order)
    assert a.lib.vl_fill_ghosts(a.h) == B.VL_ERR_ARG   # boundary cells need their sources
    assert b.step_rc(1.0, B.VL_PER_SWEEP) == B.VL_ERR_STALE_GHOSTS
    b.fill_ghosts_from(table(b, lo, hi))               # registers the sources
    for _ in range(3):
        a.fill_ghosts_from(table(a, lo, hi))
        a.step(1.0, B.VL_COALESCED)
        b.step(1.0, B.VL_PER_SWEEP)
    o = OraclePartition(N, NBLK, GEOM["dx"], GEOM["vmin"], GEOM["dv"], order, 2.5e-10, 6)
    o.set_edges(EDGES_X)
    o.load_padded(*padded_with_boundaries(N, st, lo_st, hi_st, NBLK))
    oracle.lib().vlo_mark_ghosts_valid(o._h)
    for k in range(3):
        if k:
            o.fill_ghosts()
        o.step(1.0, COALESCED)
    compare_states(a.export(), o.export_local(), 1e-12)
    assert all(np.array_equal(x, y) for x, y in zip(a.export(), b.export()))


def test_edge_graph_replays_equal_ordinary_steps(states):
    st, lo_st, hi_st = states
    lo, hi = part(lo_st, 0), part(hi_st, 0)
    a = part(st, EDGES_X)
    g = part(st, EDGES_X)
    assert g.lib.vl_graph_step(g.h, 1.0, B.VL_COALESCED, 1) == B.VL_ERR_STALE_GHOSTS
    g.fill_ghosts_from(table(g, lo, hi))
    g.step(1.0, B.VL_COALESCED)
    a.fill_ghosts_from(table(a, lo, hi))
    a.step(1.0, B.VL_COALESCED)
    for k in range(3):
        a.fill_ghosts_from(table(a, lo, hi))
        a.step(1.0, B.VL_COALESCED)
        g.graph_step(1.0, B.VL_COALESCED)
        assert all(np.array_equal(x, y) for x, y in zip(a.export(), g.export())), k


def test_autotune_at_a_simulation_edge_equals_ordinary_steps(states):
    """The autotuner needs the boundary cells' sources and then steps exactly
    as ordinary steps with those sources do."""
    st, lo_st, hi_st = states
    lo, hi = part(lo_st, 0), part(hi_st, 0)
    a = part(st, EDGES_X)
    b = part(st, EDGES_X)
    best = np.zeros(3, np.int32)
    assert a.lib.vl_autotune(a.h, 1.0, B.VL_COALESCED, 1, best.ctypes.data, None, 0) == B.VL_ERR_STALE_GHOSTS
    a.fill_ghosts_from(table(a, lo, hi))
    a.step(1.0, B.VL_COALESCED)
    _, ms = a.autotune(1.0, B.VL_COALESCED, steps_per_variant=1)
    for _ in range(1 + len(ms)):
        b.fill_ghosts_from(table(b, lo, hi))
        b.step(1.0, B.VL_COALESCED)
    assert all(np.array_equal(x, y) for x, y in zip(a.export(), b.export()))

"""Partitions at a simulation edge (Section 2.1: boundary cells feed the
stencils but are not translated; Section 3.3: a domain at the simulation edge
needs no Ghost Translation layers there), in the oracle: the boundary cells
keep their contents, flow enters from them, and Ghost Translation still gives
the classical result bit for bit."""
import numpy as np
import pytest

import oracle
from oracle import COALESCED, PER_SWEEP, OraclePartition
from edgehelp import padded_with_boundaries
from statehelp import random_state, to_dense

EDGES_X = 0b11  # both x faces
KW = dict(nblk=(2, 2, 2), dx=(4.0, 5.0, 7.0), vmin=(-4.0, -4.0, -4.0), dv=(1.0, 1.0, 1.0))


def make(n, order=(0, 1, 2), edges=EDGES_X, sparse_min=0.0, vbuffer=0, nblk=KW["nblk"]):
    p = OraclePartition(n, nblk, KW["dx"], KW["vmin"], KW["dv"], order, sparse_min, vbuffer)
    p.set_edges(edges)
    return p


def load(p, n, local, lo, hi, nblk=KW["nblk"]):
    p.load_padded(*padded_with_boundaries(n, local, lo, hi, nblk))
    oracle.lib().vlo_mark_ghosts_valid(p._h)


def run(p, steps, mode, dt=1.0):
    for k in range(steps):
        if mode == COALESCED and k > 0:
            p.fill_ghosts()      # refreshes the periodic ghost cells only
        p.step(dt, mode)


def dense_state(n, nblk, value):
    NB = int(np.prod(nblk))
    nc = int(np.prod(n))
    off = np.arange(nc + 1, dtype=np.int64) * NB
    ids = np.tile(np.arange(NB, dtype=np.int32), nc)
    f = value if np.ndim(value) else np.full(nc * NB * 64, float(value))
    return off, ids, f


@pytest.mark.parametrize("mode", [COALESCED, PER_SWEEP])
def test_constant_state_with_matching_boundary_is_unchanged(mode):
    n = (6, 4, 5)
    st = dense_state(n, KW["nblk"], 0.375)
    p = make(n)
    load(p, n, st, st, st)
    run(p, 3, mode)
    o, i, f = p.export_local()
    assert np.array_equal(o, st[0]) and np.array_equal(i, st[1])
    assert np.all(f == 0.375)


def test_integer_shift_brings_in_the_low_boundary():
    """c = +1 along x for every velocity cell: each local cell takes its
    left neighbour's value, the first one the boundary cell's, and the last
    one's content leaves through the high face."""
    n = (6, 3, 3)
    nblk = KW["nblk"]
    rng = np.random.default_rng(3)
    NB = int(np.prod(nblk))
    nc = int(np.prod(n))
    local = dense_state(n, nblk, rng.uniform(0.5, 1.5, nc * NB * 64))
    lo = dense_state(n, nblk, rng.uniform(2.0, 3.0, nc * NB * 64))
    hi = dense_state(n, nblk, rng.uniform(4.0, 5.0, nc * NB * 64))
    p = make(n)
    load(p, n, local, lo, hi)
    table = np.zeros((3, 8))
    table[0] = 1.0
    p.set_courant_override(table)
    p.step(1.0, COALESCED)
    got = to_dense(*p.export_local(), NB).reshape(n[2], n[1], n[0], NB * 64)
    a = to_dense(*local, NB).reshape(n[2], n[1], n[0], NB * 64)
    b = to_dense(*lo, NB).reshape(n[2], n[1], n[0], NB * 64)
    want = np.concatenate([b[:, :, -1:], a[:, :, :-1]], axis=2)
    assert np.max(np.abs(got - want)) <= 2 * np.finfo(float).eps * 5.0


@pytest.mark.parametrize("order", [(0, 1, 2), (2, 0, 1), (1, 2, 0)])
def test_ghost_translation_equals_classical_at_edges(order):
    n = (7, 5, 6)
    nblk = (3, 2, 3)
    st = random_state(n, nblk, 41, density=0.4, zero_frac=0.1)
    lo = random_state(n, nblk, 42, density=0.4)
    hi = random_state(n, nblk, 43, density=0.4)
    a = OraclePartition(n, nblk, (6.0, 5.0, 7.0), (-6.0, -4.0, -6.0), (1.0,) * 3, order, 2.5e-10, 6)
    b = OraclePartition(n, nblk, (6.0, 5.0, 7.0), (-6.0, -4.0, -6.0), (1.0,) * 3, order, 2.5e-10, 6)
    for p in (a, b):
        p.set_edges(EDGES_X)
        load(p, n, st, lo, hi, nblk)
    run(a, 3, COALESCED)
    run(b, 3, PER_SWEEP)
    ra, rb = a.export_local(), b.export_local()
    assert all(np.array_equal(x, y) for x, y in zip(ra, rb))
    # the boundary cells are as loaded (never translated, never refreshed)
    padded = padded_with_boundaries(n, st, lo, hi, nblk)
    P = tuple(v + 6 for v in n)
    for p in (a, b):
        for (x, y, z) in [(0, 0, 0), (2, 4, 7), (P[0] - 1, 3, 2), (P[0] - 3, P[1] - 1, P[2] - 1)]:
            q = x + P[0] * (y + P[1] * z)
            i, f = p.get_cell(x, y, z)
            o0, o1 = padded[0][q], padded[0][q + 1]
            assert np.array_equal(i, padded[1][o0:o1]) and np.array_equal(f, padded[2][o0 * 64:o1 * 64])


def test_no_ghost_layers_beyond_an_edge():
    n = (5, 6, 4)
    p = make(n, order=(2, 0, 1), edges=0b001101)   # low x, low y, high y
    boxes = [p.update_box(COALESCED, s) for s in range(3)]
    # first shear (z): later axes x and y, x only beyond the high face
    assert boxes[0] == ((3, 3, 3), (3 + 5 + 3, 3 + 6, 3 + 4))
    # second shear (x): later axis y, both faces at the edge
    assert boxes[1] == ((3, 3, 3), (3 + 5, 3 + 6, 3 + 4))
    assert boxes[2] == ((3, 3, 3), (3 + 5, 3 + 6, 3 + 4))
    with pytest.raises(ValueError):
        p.set_edges(64)

"""Pins of the oracle's 3D translation step: conservation, exact shifts,
symmetry, Ghost Translation against the classical per-direction ghost refresh
(Sections 2.1, 3, 3.1), domain decomposition, sparse-versus-dense equivalence
and the block pruning ledger."""
import numpy as np
import pytest

import oracle
from oracle import COALESCED, PER_SWEEP, OraclePartition
from oracle import gt_sets
from statehelp import (block_perm, dense_to_csr, lists_of, random_state, roll_cells, to_dense)

EPS = np.finfo(np.float64).eps

# small velocity mesh: nv = 8 per axis, v in +-3.5 (dv = 1, vmin = -4);
# dx chosen so every |c| <= 1 at dt = 1
SMALL = dict(nblk=(2, 2, 2), dx=(4.0, 5.0, 7.0), vmin=(-4.0, -4.0, -4.0), dv=(1.0, 1.0, 1.0))


def make(n, order=(0, 1, 2), sparse_min=0.0, vbuffer=0, **kw):
    g = dict(SMALL)
    g.update(kw)
    return OraclePartition(n, g["nblk"], g["dx"], g["vmin"], g["dv"], order, sparse_min, vbuffer)


def run(p, steps, dt=1.0, mode=COALESCED):
    st = None
    for _ in range(steps):
        if mode == COALESCED:
            p.fill_ghosts()
        st = p.step(dt, mode)
    return st


def test_spatially_constant_state_is_unchanged_bitwise():
    n = (4, 3, 5)
    NB = 8
    rng = np.random.default_rng(10)
    g = rng.uniform(0.1, 1.0, (NB, 64))
    dense = np.broadcast_to(g, (int(np.prod(n)), NB, 64)).copy()
    p = make(n)
    p.load_local(*dense_to_csr(dense))
    run(p, 2)
    o, i, f = p.export_local()
    assert np.array_equal(to_dense(o, i, f, NB), dense)


def test_mass_per_velocity_cell_is_conserved():
    """Translation moves mass only in space: the spatial sum of every velocity
    cell (hence mass, momentum and energy) is conserved."""
    n = (5, 4, 6)
    NB = 8
    st0 = random_state(n, SMALL["nblk"], 11, density=0.5)
    p = make(n)
    p.load_local(*st0)
    run(p, 3)
    s0 = to_dense(*st0, NB).sum(axis=0)
    s1 = to_dense(*p.export_local(), NB).sum(axis=0)
    assert np.max(np.abs(s1 - s0)) <= 1e-13 * np.max(s0)


@pytest.mark.parametrize("shift", [(1, 0, -1), (-1, 1, 0), (0, -1, 1)])
def test_integer_courant_gives_exact_periodic_shift(shift):
    n = (5, 4, 6)
    NB = 8
    st0 = random_state(n, SMALL["nblk"], 12, density=0.4)
    p = make(n)
    p.load_local(*st0)
    table = np.zeros((3, 8))
    for d in range(3):
        table[d, :] = shift[d]
    p.set_courant_override(table)
    run(p, 1)
    d0 = to_dense(*st0, NB)
    d1 = to_dense(*p.export_local(), NB)
    want = roll_cells(d0, n, shift)
    assert np.max(np.abs(d1 - want)) <= 4 * EPS * np.max(d0)


def test_axis_permutation_is_exact():
    """Relabelling the axes of space, velocity space and the sweep order
    together gives the relabelled result bit for bit."""
    n = (4, 5, 3)
    nblk = (3, 2, 2)
    kw = dict(nblk=nblk, dx=(6.0, 5.0, 7.0), vmin=(-6.0, -4.0, -4.0), dv=(1.0, 1.0, 1.0))
    st0 = random_state(n, nblk, 13, density=0.5)
    a = make(n, order=(0, 1, 2), sparse_min=3e-10, vbuffer=6, **kw)
    a.load_local(*st0)
    run(a, 2)
    ra = a.export_local()

    perm = (1, 2, 0)  # new axis k is old axis perm[k]
    inv = [perm.index(d) for d in range(3)]
    n2 = tuple(n[perm[k]] for k in range(3))
    newb, newl, nblk2 = block_perm(nblk, perm)
    kw2 = dict(nblk=nblk2, dx=tuple(kw["dx"][perm[k]] for k in range(3)),
               vmin=tuple(kw["vmin"][perm[k]] for k in range(3)), dv=(1.0, 1.0, 1.0))
    NB = int(np.prod(nblk))

    def relabel(state, nn, cell_map_src_dims):
        d = to_dense(*state, NB)
        # dense[cell, block, lane] -> new labels
        g = d.reshape(nn[2], nn[1], nn[0], NB, 64).transpose(2, 1, 0, 3, 4)  # [x,y,z,b,l]
        g = g.transpose(perm[0], perm[1], perm[2], 3, 4)  # new spatial axes
        out = np.zeros_like(g)
        out[:, :, :, newb[:, None], newl[None, :]] = g
        return out.transpose(2, 1, 0, 3, 4).reshape(-1, NB, 64)

    def present(state, nn):
        o, i, _ = state
        m = np.zeros((int(np.prod(nn)), NB), bool)
        for c in range(o.size - 1):
            m[c, i[o[c]:o[c + 1]]] = True
        g = m.reshape(nn[2], nn[1], nn[0], NB).transpose(2, 1, 0, 3).transpose(perm[0], perm[1], perm[2], 3)
        out = np.zeros_like(g)
        out[:, :, :, newb] = g
        return out.transpose(2, 1, 0, 3).reshape(-1, NB)

    d2 = relabel(st0, n, None)
    pres = present(st0, n)
    nc = d2.shape[0]
    cnt = pres.sum(axis=1)
    off = np.zeros(nc + 1, np.int64)
    np.cumsum(cnt, out=off[1:])
    ids2 = np.concatenate([np.nonzero(pres[c])[0] for c in range(nc)]).astype(np.int32)
    f2 = np.concatenate([d2[c, np.nonzero(pres[c])[0]].reshape(-1) for c in range(nc)])
    b = make(n2, order=tuple(inv[d] for d in (0, 1, 2)), sparse_min=3e-10, vbuffer=6, **kw2)
    b.load_local(off, ids2, f2)
    run(b, 2)
    rb = b.export_local()
    assert np.array_equal(relabel(ra, n, None), to_dense(*rb, NB))
    assert np.array_equal(present(ra, n), np.stack([np.isin(np.arange(NB), rb[1][rb[0][c]:rb[0][c + 1]])
                                                     for c in range(rb[0].size - 1)]))


@pytest.mark.parametrize("order", [(0, 1, 2), (2, 0, 1)])
def test_ghost_translation_equals_per_direction_refresh_bitwise(order):
    """GT3 (one ghost update per step, shears also on ghost cells) gives the
    classical result (ghost refresh before every shear) bit for bit, lists
    included (Section 3.2: the full variant needs no approximation)."""
    n = (5, 4, 6)
    nblk = (3, 2, 3)
    kw = dict(nblk=nblk, dx=(6.0, 5.0, 7.0), vmin=(-6.0, -4.0, -6.0), dv=(1.0, 1.0, 1.0))
    st0 = random_state(n, nblk, 14, density=0.35, zero_frac=0.1)
    a = make(n, order, sparse_min=2.5e-10, vbuffer=6, **kw)
    b = make(n, order, sparse_min=2.5e-10, vbuffer=6, **kw)
    a.load_local(*st0)
    b.load_local(*st0)
    for _ in range(3):
        a.fill_ghosts()
        sa = a.step(1.0, COALESCED)
        sb = b.step(1.0, PER_SWEEP)
        assert sa["blocks"] == sb["blocks"]
    ra, rb = a.export_local(), b.export_local()
    assert np.array_equal(ra[0], rb[0]) and np.array_equal(ra[1], rb[1])
    assert np.array_equal(ra[2], rb[2])


def test_ghost_translation_on_sparse_maxwellians_equals_refresh():
    w = oracle_small_sparse()
    a = OraclePartition.from_workload(w)
    b = OraclePartition.from_workload(w)
    for _ in range(2):
        a.fill_ghosts()
        a.step(w.dt, COALESCED)
        b.step(w.dt, PER_SWEEP)
    ra, rb = a.export_local(), b.export_local()
    assert all(np.array_equal(x, y) for x, y in zip(ra, rb))


def oracle_small_sparse():
    from paper_2504_21450_amd import workloads as W
    return W.maxwellian_sparse(n=(4, 3, 3), threads=1)


def test_domain_decomposition_2x2x2_is_exact():
    """Eight sub-partitions whose ghost domains are filled from their
    neighbours' local cells (one exchange per step, as in Fig. 3a) reproduce
    the single periodic partition bit for bit."""
    n = (6, 4, 8)
    sub = (3, 2, 4)
    nblk = (2, 2, 2)
    NB = 8
    st = random_state(n, nblk, 15, density=0.5)
    full = make(n, sparse_min=2e-10, vbuffer=6)
    full.load_local(*st)
    cur = st
    for _ in range(2):
        full.fill_ghosts()
        full.step(1.0, COALESCED)
        dense = to_dense(*cur, NB)
        pres = np.zeros((dense.shape[0], NB), bool)
        for c in range(cur[0].size - 1):
            pres[c, cur[1][cur[0][c]:cur[0][c + 1]]] = True
        new_dense = np.zeros_like(dense)
        new_pres = np.zeros_like(pres)
        for sz in range(2):
            for sy in range(2):
                for sx in range(2):
                    lo = (sx * sub[0], sy * sub[1], sz * sub[2])
                    p = make(sub, sparse_min=2e-10, vbuffer=6)
                    P = p.P
                    for z in range(P[2]):
                        for y in range(P[1]):
                            for x in range(P[0]):
                                gx = (lo[0] + x - 3) % n[0]
                                gy = (lo[1] + y - 3) % n[1]
                                gz = (lo[2] + z - 3) % n[2]
                                c = gx + n[0] * (gy + n[1] * gz)
                                ids = np.nonzero(pres[c])[0]
                                p.set_cell(x, y, z, ids, dense[c, ids].reshape(-1))
                    # set_cell is not a ghost update; an explicit halo is declared so
                    assert p.step_rc(1.0, COALESCED) == -4
                    mark_ghosts_valid(p)
                    p.step(1.0, COALESCED)
                    o, i, f = p.export_local()
                    for q in range(o.size - 1):
                        x, y, z = q % sub[0], (q // sub[0]) % sub[1], q // (sub[0] * sub[1])
                        c = (lo[0] + x) + n[0] * ((lo[1] + y) + n[1] * (lo[2] + z))
                        ids = i[o[q]:o[q + 1]]
                        new_pres[c, ids] = True
                        new_dense[c, ids] = f[o[q] * 64:o[q + 1] * 64].reshape(-1, 64)
        cnt = new_pres.sum(axis=1)
        off = np.zeros(cnt.size + 1, np.int64)
        np.cumsum(cnt, out=off[1:])
        ids = np.concatenate([np.nonzero(new_pres[c])[0] for c in range(cnt.size)]).astype(np.int32)
        f = np.concatenate([new_dense[c, np.nonzero(new_pres[c])[0]].reshape(-1) for c in range(cnt.size)])
        cur = (off, ids, f)
    rf = full.export_local()
    assert all(np.array_equal(x, y) for x, y in zip(rf, cur))


def mark_ghosts_valid(p):
    """An explicitly supplied ghost domain counts as a ghost update."""
    oracle.lib().vlo_mark_ghosts_valid(p._h)


def test_sparse_equals_dense_on_nonnegative_data():
    """With absent blocks read as zero and the sign-aware block growth, the
    sparse store gives exactly the dense result: equal values on the sparse
    lists and exact zeros elsewhere."""
    n = (5, 4, 3)
    NB = 8
    st = random_state(n, SMALL["nblk"], 16, density=0.3, zero_frac=0.2)
    s = make(n)
    s.load_local(*st)
    d = make(n)
    d.load_local(*dense_to_csr(to_dense(*st, NB)))
    run(s, 3)
    run(d, 3)
    ds = to_dense(*s.export_local(), NB)
    dd = to_dense(*d.export_local(), NB)
    assert np.array_equal(ds, dd)


def test_pruning_ledger_and_rule():
    n = (5, 4, 3)
    nblk = (3, 3, 2)
    NB = 18
    T = 6e-10
    kw = dict(nblk=nblk, dx=(6.0, 6.0, 7.0), vmin=(-6.0, -6.0, -4.0), dv=(1.0, 1.0, 1.0))
    st = random_state(n, nblk, 17, density=0.4, zero_frac=0.3)
    p = make(n, sparse_min=T, vbuffer=6, **kw)
    p.load_local(*st)
    p.fill_ghosts()
    s = p.step(1.0)
    assert s["pruned_mass"] > 0
    assert abs(s["mass_after"] + s["pruned_mass"] - s["mass_before"]) <= 1e-13 * s["mass_before"]
    o, i, f = p.export_local()
    f2 = f.reshape(-1, 64)
    for c in range(o.size - 1):
        ids = i[o[c]:o[c + 1]]
        content = {int(b) for b, v in zip(ids, f2[o[c]:o[c + 1]]) if np.any(v >= T)}
        want = set()
        for b in content:
            bx, by, bz = b % 3, (b // 3) % 3, b // 9
            want.add(b)
            for ox, oy, oz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                x, y, z = bx + ox, by + oy, bz + oz
                if 0 <= x < 3 and 0 <= y < 3 and 0 <= z < 2:
                    want.add(x + 3 * (y + 3 * z))
        assert set(int(b) for b in ids) == want


@pytest.mark.parametrize("order", [(0, 1, 2), (2, 0, 1), (1, 2, 0)])
def test_update_boxes_follow_the_papers_set_construction(order):
    """The oracle's per-shear update boxes are the paper's GT3 active sets
    (reverse-order construction of Section 3.1) in flux form."""
    n = 5
    p = make((n, n, n), order)
    want = gt_sets.pull_update_boxes(n, order)
    for s in range(3):
        lo, hi = p.update_box(COALESCED, s)
        assert tuple(v - 3 for v in lo) == want[s][0]
        assert tuple(v - 3 for v in hi) == want[s][1]
        lo, hi = p.update_box(PER_SWEEP, s)
        assert lo == (3, 3, 3) and hi == (3 + n,) * 3


def test_error_codes():
    n = (3, 3, 3)
    p = make(n)
    p.load_local(*random_state(n, SMALL["nblk"], 18))
    assert p.step_rc(1.0, COALESCED) == -4      # no ghost update since load
    p.fill_ghosts()
    assert p.step_rc(2.0, COALESCED) == -2      # |v dt/dx| = 3.5*2/4 > 1
    assert p.step_rc(1.0, COALESCED) == 0
    assert p.step_rc(1.0, COALESCED) == -4      # ghosts consumed by the step
    assert p.step_rc(1.0, PER_SWEEP) == 0       # the classical mode refreshes its own faces


def test_cell_centre_velocity_sets_the_courant_number():
    """Only the velocity cells with centre v_x = 3.5 (dv = 1, vmin = -4) hold
    mass and f varies along x only; with dx = 3.5 and dt = 1 their Courant
    number is exactly 1, so the step is an exact shift by one cell along x
    (the y and z shears see spatially constant data)."""
    n = (6, 3, 4)
    NB = 8
    kw = dict(dx=(3.5, 5.0, 7.0))
    rng = np.random.default_rng(19)
    prof = rng.uniform(0.1, 1.0, n[0])
    dense = np.zeros((int(np.prod(n)), NB, 64))
    lanes = [l for l in range(64) if (l & 3) == 3]       # ix = 3 within the block
    blocks = [b for b in range(NB) if b % 2 == 1]        # bx = 1 -> j_x = 7
    for c in range(dense.shape[0]):
        for b in blocks:
            dense[c, b, lanes] = prof[c % n[0]]
    p = make(n, **kw)
    p.load_local(*dense_to_csr(dense))
    run(p, 1)
    got = to_dense(*p.export_local(), NB)
    want = roll_cells(dense, n, (1, 0, 0))
    assert np.max(np.abs(got - want)) <= 4 * EPS


def test_pruning_threshold_is_inclusive():
    """dt = 0 moves nothing, so the step reduces to the end-of-step pruning of
    the input: a block survives iff one value is >= sparse_min or it is a face
    neighbour (in velocity space) of such a block."""
    n = (2, 2, 1)
    nblk = (4, 3, 2)
    NB = 24
    T = 1e-3
    dense = np.zeros((4, NB, 64))
    rng = np.random.default_rng(20)
    dense[:] = rng.uniform(0, 0.5 * T, dense.shape)
    dense[0, 5, 17] = T                       # exactly at the threshold: kept
    dense[1, 10, 3] = T * (1 - 1e-15)         # just below: not content
    dense[2, 0, 0] = 2 * T
    dense[3, 23, 63] = 1.5 * T
    p = make(n, sparse_min=T, vbuffer=6, nblk=nblk, vmin=(-8.0, -6.0, -4.0), dx=(10.0, 10.0, 10.0))
    p.load_local(*dense_to_csr(dense))
    p.fill_ghosts()
    s = p.step(0.0)
    o, i, f = p.export_local()

    def face_nb(b):
        bx, by, bz = b % 4, (b // 4) % 3, b // 12
        out = {b}
        for ox, oy, oz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            x, y, z = bx + ox, by + oy, bz + oz
            if 0 <= x < 4 and 0 <= y < 3 and 0 <= z < 2:
                out.add(x + 4 * (y + 3 * z))
        return out
    want = [face_nb(5), set(), face_nb(0), face_nb(23)]
    for c in range(4):
        assert set(int(b) for b in i[o[c]:o[c + 1]]) == want[c]
        for k, b in enumerate(i[o[c]:o[c + 1]]):
            assert np.array_equal(f[(o[c] + k) * 64:(o[c] + k + 1) * 64], dense[c, b])
    kept = sum(dense[c, list(want[c])].sum() for c in range(4))
    assert s["pruned_mass"] == pytest.approx((dense.sum() - kept) * 1000.0, rel=1e-12)


def _prune_only(dense, nblk, T, vbuffer):
    """dt = 0: the step reduces to the end-of-step pruning of the input."""
    n = (dense.shape[0], 1, 1)
    p = make(n, sparse_min=T, vbuffer=vbuffer, nblk=nblk, vmin=(-8.0, -6.0, -6.0),
             dx=(10.0, 10.0, 10.0))
    p.load_local(*dense_to_csr(dense))
    p.fill_ghosts()
    s = p.step(0.0)
    o, i, f = p.export_local()
    return s, [set(int(b) for b in i[o[c]:o[c + 1]]) for c in range(dense.shape[0])], (o, i, f)


def test_pruning_with_the_26_neighbour_buffer_hand_worked():
    """The velocity-space buffer of all 26 neighbours (Section 2's 'one
    neighbour-block buffer' read as every block touching a content block),
    clipped at the edges and corners of the mesh.  Mesh 4 x 3 x 3 blocks, id =
    bx + 4 (by + 3 bz).  The expected sets below were enumerated by hand.
      cell 0: content (1,1,1) = 17, inside the mesh: the 3x3x3 cube around it
      cell 1: content (3,2,2) = 35, the far corner: a 2x2x2 cube
      cell 2: content (0,0,1) = 12, on an edge of the mesh: 2x2x3 blocks
      cell 3: content (0,0,0) = 0 and (2,2,2) = 34; block 17 = (1,1,1) is
              held (below the threshold) and touches both only through a
              corner: kept with 26 neighbours, removed with 6."""
    nblk = (4, 3, 3)
    NB = 36
    T = 1e-3
    rng = np.random.default_rng(23)
    dense = rng.uniform(0.0, 0.5 * T, (4, NB, 64))
    for c in range(4):   # only the listed content blocks reach the threshold
        assert np.all(dense[c] < T)
    dense[0, 17, 40] = T
    dense[1, 35, 0] = 3 * T
    dense[2, 12, 63] = 2 * T
    dense[3, 0, 5] = 2 * T
    dense[3, 34, 21] = T
    want26 = [
        {0, 1, 2, 4, 5, 6, 8, 9, 10, 12, 13, 14, 16, 17, 18, 20, 21, 22,
         24, 25, 26, 28, 29, 30, 32, 33, 34},
        {18, 19, 22, 23, 30, 31, 34, 35},
        {0, 1, 4, 5, 12, 13, 16, 17, 24, 25, 28, 29},
        {0, 1, 4, 5, 12, 13, 16, 17, 18, 19, 21, 22, 23, 29, 30, 31, 33, 34, 35},
    ]
    want6 = [
        {17, 16, 18, 13, 21, 5, 29},
        {35, 34, 31, 23},
        {12, 13, 16, 0, 24},
        {0, 1, 4, 12, 34, 33, 35, 30, 22},
    ]
    assert len(want26[0]) == 27 and len(want26[1]) == 8 and len(want26[2]) == 12
    for vb, want in ((26, want26), (6, want6)):
        s, got, (o, i, f) = _prune_only(dense, nblk, T, vb)
        assert got == want, vb
        for c in range(4):
            for k, b in enumerate(i[o[c]:o[c + 1]]):
                assert np.array_equal(f[(o[c] + k) * 64:(o[c] + k + 1) * 64], dense[c, b])
        kept = sum(dense[c, sorted(want[c])].sum() for c in range(4))
        assert s["pruned_mass"] == pytest.approx((dense.sum() - kept) * 1000.0, rel=1e-12)
    # the corner-only neighbour is what tells the two buffers apart
    assert 17 in want26[3] and 17 not in want6[3]
    # without a buffer only the content blocks stay
    _, got0, _ = _prune_only(dense, nblk, T, 0)
    assert got0 == [{17}, {35}, {12}, {0, 34}]


def test_pruning_creates_zero_blocks_in_the_26_neighbour_buffer():
    """A content block whose diagonal neighbours are absent gets them as new,
    zero blocks (the list is the dilated set, not the old list)."""
    nblk = (3, 3, 3)
    NB = 27
    T = 1.0
    n = (1, 1, 1)
    p = make(n, sparse_min=T, vbuffer=26, nblk=nblk, vmin=(-6.0, -6.0, -6.0), dx=(10.0, 10.0, 10.0))
    f = np.full(64, 0.25)
    f[7] = 2.0
    p.load_local(np.array([0, 1], np.int64), np.array([13], np.int32), f)   # the centre block only
    p.fill_ghosts()
    p.step(0.0)
    o, i, g = p.export_local()
    assert list(i) == list(range(27))
    g = g.reshape(27, 64)
    assert np.array_equal(g[13], f)
    assert not np.any(np.delete(g, 13, axis=0))

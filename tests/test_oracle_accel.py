"""Pins of the oracle's acceleration step: the Lorentz-force term of the
Vlasov equation (Section 2, eq. 1) over one time step, split into three
velocity-axis shears by SLICE-3D (the method Section 2 names), each a
conservative 1D remap with the CW84 parabolas.

Pinned against the mathematics, not the code: the velocity map against a
numerical integration of the characteristics dv/dt = (q/m)(E + v x B); the
three one-coordinate maps composed back into the affine map; the column remap
against identity, exact integer shifts, closed-form integrals of quadratics
and mass conservation; the whole step against exact shifts (E only), per-cell
mass conservation, a Maxwellian rotated about B, a Maxwellian at rest in the
E x B frame, and the dense velocity space (the sparse lists lose nothing)."""
import numpy as np
import pytest

import oracle
from oracle import OraclePartition
from statehelp import dense_to_csr, random_state, to_dense

QM = 9.58e7   # proton charge-to-mass ratio [C/kg]


def rk4(E, B, qm, dt, v, n=20000):
    E, B, v = np.asarray(E, float), np.asarray(B, float), np.asarray(v, float)
    h = dt / n
    f = lambda u: qm * (E + np.cross(u, B))
    for _ in range(n):
        k1 = f(v)
        k2 = f(v + 0.5 * h * k1)
        k3 = f(v + 0.5 * h * k2)
        k4 = f(v + h * k3)
        v = v + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return v


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_velocity_map_follows_the_characteristics(seed):
    rng = np.random.default_rng(seed)
    E = rng.normal(0, 1e-3, 3)           # V/m
    B = rng.normal(0, 1e-8, 3)           # T
    dt = 0.4 / (QM * np.linalg.norm(B))  # gyration angle 0.4 rad
    A, c = oracle.accel_map(E, B, QM, dt)
    for _ in range(3):
        v = rng.normal(0, 3e5, 3)
        want = rk4(E, B, QM, dt, v)
        assert np.max(np.abs(A @ v + c - want)) <= 1e-9 * np.max(np.abs(want))
    # B = 0: a uniform acceleration
    A, c = oracle.accel_map(E, [0.0, 0.0, 0.0], QM, 0.5)
    assert np.array_equal(A, np.eye(3))
    assert np.allclose(c, QM * E * 0.5, rtol=1e-15, atol=0)


def test_gyration_is_a_rotation_about_b():
    B = np.array([1.0, 2.0, -2.0]) * 1e-9
    A, _ = oracle.accel_map([0, 0, 0], B, QM, 0.3)
    assert np.max(np.abs(A @ A.T - np.eye(3))) <= 1e-15
    assert abs(np.linalg.det(A) - 1.0) <= 1e-15
    b = B / np.linalg.norm(B)
    assert np.max(np.abs(A @ b - b)) <= 1e-15
    # the rotation angle is -(q/m)|B| dt (left-handed about B for q > 0)
    th = -QM * np.linalg.norm(B) * 0.3
    assert abs(np.arccos((np.trace(A) - 1.0) / 2.0) - abs(th)) <= 1e-12
    e = np.cross(b, [1.0, 0.0, 0.0])
    e /= np.linalg.norm(e)
    assert np.dot(np.cross(e, A @ e), b) * np.sign(th) > 0


@pytest.mark.parametrize("order", [(0, 1, 2), (2, 0, 1), (1, 2, 0)])
def test_three_one_coordinate_maps_compose_to_the_map(order):
    rng = np.random.default_rng(7)
    for _ in range(5):
        E = rng.normal(0, 1e-3, 3)
        B = rng.normal(0, 1e-8, 3)
        dt = rng.uniform(0.05, 0.5) / (QM * np.linalg.norm(B))
        A, c = oracle.accel_map(E, B, QM, dt)
        M = oracle.slice_factors(A, c, order)
        assert M is not None
        # each map changes only its own coordinate; the product of their own
        # coefficients is the volume change det A = 1
        assert abs(np.prod([M[k, order[k]] for k in range(3)]) - 1.0) <= 1e-14
        for _ in range(4):
            v = rng.normal(0, 3e5, 3)
            u = v.copy()
            for k in range(3):
                u[order[k]] = M[k, :3] @ u + M[k, 3]
            assert np.max(np.abs(u - (A @ v + c))) <= 1e-9 * np.max(np.abs(v))
    # a half turn cannot be split into order-preserving shears
    A, c = oracle.accel_map([0, 0, 0], [0, 0, 1e-8], QM, np.pi / (QM * 1e-8))
    assert oracle.slice_factors(A, c, (0, 1, 2)) is None


def test_column_remap_identity_and_integer_shifts():
    rng = np.random.default_rng(11)
    a = np.zeros(40)
    a[8:30] = rng.uniform(0.1, 1.0, 22)
    assert np.array_equal(oracle.remap_column(a, 1.0, 0.0), a)
    for k in (1, 3, -5):
        want = np.zeros(40)
        want[8 + k:30 + k] = a[8:30]
        assert np.array_equal(oracle.remap_column(a, 1.0, float(k)), want)


@pytest.mark.parametrize("alpha,sigma", [(1.0, 0.37), (0.97, 2.3), (1.02, -1.7), (1.0, -2.75)])
def test_column_remap_integrates_quadratics_exactly(alpha, sigma):
    """Cell averages of an increasing quadratic: the parabolas reproduce it
    (the limiter stays inactive away from the column's ends), so each new
    cell is the closed-form integral over its source interval."""
    N = 60
    Q = lambda u: (u ** 3) / 3.0 + 5.0 * u ** 2 + 26.0 * u   # antiderivative of (u + 5)^2 + 1
    i = np.arange(N, dtype=float)
    a = Q(i + 1.0) - Q(i)
    out = oracle.remap_column(a, alpha, sigma)
    for t in range(12, 48):
        lo, hi = (t - sigma) / alpha, (t + 1 - sigma) / alpha
        want = Q(hi) - Q(lo)
        assert abs(out[t] - want) <= 1e-12 * want, t


@pytest.mark.parametrize("alpha,sigma", [(1.0, 0.4), (0.95, 1.3), (1.05, -2.2)])
def test_column_remap_conserves_mass(alpha, sigma):
    rng = np.random.default_rng(13)
    a = np.zeros(64)
    a[15:45] = rng.uniform(0.0, 1.0, 30)
    a[20] = 0.0
    out = oracle.remap_column(a, alpha, sigma)
    assert abs(out.sum() - a.sum()) <= 1e-14 * a.sum()
    assert np.min(out) >= 0.0


def geom(nblk=(4, 4, 4)):
    return dict(nblk=nblk, dx=(1e5, 1e5, 1e5), vmin=tuple(-2.0 * b * 1e4 for b in nblk), dv=(1e4, 1e4, 1e4))


def partition(n, st, g, sparse_min=0.0, vbuffer=0):
    o = OraclePartition(n, g["nblk"], g["dx"], g["vmin"], g["dv"], (0, 1, 2), sparse_min, vbuffer)
    o.load_local(*st)
    return o


def inner_state(n, nblk, seed, margin=1):
    """Random nonnegative values on the blocks at least `margin` blocks from
    the velocity mesh's faces, dense there."""
    rng = np.random.default_rng(seed)
    NB = int(np.prod(nblk))
    nc = int(np.prod(n))
    b = np.arange(NB)
    bc = np.stack([b % nblk[0], (b // nblk[0]) % nblk[1], b // (nblk[0] * nblk[1])], 1)
    inner = np.all((bc >= margin) & (bc < np.array(nblk) - margin), 1)
    dense = np.zeros((nc, NB, 64))
    dense[:, inner] = rng.uniform(0.1, 1.0, (nc, int(inner.sum()), 64)) * 1e-12
    return dense


def test_electric_acceleration_by_whole_cells_is_an_exact_shift():
    """B = 0 and (q/m) E dt a whole number of velocity cells per axis: every
    column moves by whole cells, so the step is an exact shift of f."""
    n, g = (2, 1, 2), geom((5, 5, 5))
    dense = inner_state(n, g["nblk"], 21, margin=2)
    shift = np.array([2, -3, 1])
    dt = 0.5
    E = shift * g["dv"][0] / (QM * dt)
    EB = np.tile(np.concatenate([E, [0.0, 0.0, 0.0]]), (int(np.prod(n)), 1))
    o = partition(n, dense_to_csr(dense), g)
    o.accelerate(dt, QM, EB)
    got = to_dense(*o.export_local(), 125)
    nv = 20
    want = np.zeros_like(dense)
    for c in range(dense.shape[0]):
        fv = np.zeros((nv, nv, nv))   # (z, y, x) velocity cells
        for bid in range(125):
            bx, by, bz = bid % 5, (bid // 5) % 5, bid // 25
            fv[4 * bz:4 * bz + 4, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4] = dense[c, bid].reshape(4, 4, 4)
        fv = np.roll(fv, tuple(shift[::-1]), axis=(0, 1, 2))
        for bid in range(125):
            bx, by, bz = bid % 5, (bid // 5) % 5, bid // 25
            want[c, bid] = fv[4 * bz:4 * bz + 4, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4].reshape(-1)
    assert np.array_equal(got, want)


def test_acceleration_conserves_mass_cell_by_cell():
    n, g = (3, 2, 2), geom((6, 6, 6))
    dense = inner_state(n, g["nblk"], 22, margin=2)
    rng = np.random.default_rng(23)
    nc = int(np.prod(n))
    # drift |E|/|B| ~ 1e4 m/s (one velocity cell): the distribution stays on the mesh
    EB = np.concatenate([rng.normal(0, 1e-4, (nc, 3)), rng.normal(0, 1e-8, (nc, 3))], 1)
    o = partition(n, dense_to_csr(dense), g)
    s = o.accelerate(0.3 / (QM * 1.5e-8), QM, EB)
    got = to_dense(*o.export_local(), 216)
    per0 = dense.sum(axis=(1, 2))
    per1 = got.sum(axis=(1, 2))
    assert np.max(np.abs(per1 - per0) / per0) <= 1e-13
    assert abs(s["mass_after"] - s["mass_before"]) <= 1e-13 * s["mass_before"]
    assert np.min(got) >= 0.0


def maxwellian_cell(g, V, vth):
    nblk, dv, vmin = g["nblk"], g["dv"][0], g["vmin"]
    NB = int(np.prod(nblk))
    out = np.zeros((NB, 64))
    for bid in range(NB):
        bx, by, bz = bid % nblk[0], (bid // nblk[0]) % nblk[1], bid // (nblk[0] * nblk[1])
        for l in range(64):
            v = np.array([vmin[0] + (4 * bx + (l & 3) + 0.5) * dv, vmin[1] + (4 * by + ((l >> 2) & 3) + 0.5) * dv,
                          vmin[2] + (4 * bz + (l >> 4) + 0.5) * dv])
            out[bid, l] = np.exp(-np.sum((v - V) ** 2) / (2 * vth ** 2))
    return out * 1e-9


def test_maxwellian_gyrates_about_the_magnetic_field():
    """A drifting Maxwellian in B = B z: its density is unchanged, its bulk
    velocity rotates by -(q/m)|B| dt about z, its speed and temperature stay."""
    g = geom((8, 8, 8))
    V0 = np.array([6e4, 0.0, 1e4])
    f = maxwellian_cell(g, V0, 1.6e4)
    B = np.array([0.0, 0.0, 1e-8])
    th = -0.35
    dt = -th / (QM * 1e-8)
    o = partition((1, 1, 1), dense_to_csr(f[None]), g)
    n0, Vb, P0, _ = o.moments()
    o.accelerate(dt, QM, np.concatenate([[0.0, 0.0, 0.0], B])[None])
    n1, V1, P1, _ = o.moments()
    # the tail beyond 6 thermal speeds (~1e-9 of the mass) reaches the mesh's
    # edge and part of it turns off the mesh
    assert abs(n1[0] - n0[0]) <= 1e-9 * n0[0]
    R = np.array([[np.cos(th), -np.sin(th), 0.0], [np.sin(th), np.cos(th), 0.0], [0.0, 0.0, 1.0]])
    want = R @ Vb[0]
    assert np.linalg.norm(V1[0] - want) <= 2e-3 * np.linalg.norm(Vb[0])
    assert abs(np.sum(P1[0, :3]) - np.sum(P0[0, :3])) <= 0.02 * np.sum(P0[0, :3])   # temperature


def test_maxwellian_at_rest_in_the_e_cross_b_frame_stays():
    """E = -V0 x B: the drift velocity is V0 (perpendicular to B), so a
    Maxwellian centred there only gyrates about its own centre: the step
    leaves its moments and values (to the remap's resolution) in place."""
    g = geom((8, 8, 8))
    V0 = np.array([4e4, -3e4, 0.0])
    f = maxwellian_cell(g, V0, 1.6e4)
    B = np.array([0.0, 0.0, 1e-8])
    E = -np.cross(V0, B)
    dt = 0.3 / (QM * 1e-8)
    o = partition((1, 1, 1), dense_to_csr(f[None]), g)
    n0, Vb, P0, _ = o.moments()
    o.accelerate(dt, QM, np.concatenate([E, B])[None])
    n1, V1, P1, _ = o.moments()
    assert abs(n1[0] - n0[0]) <= 1e-13 * n0[0]
    assert np.linalg.norm(V1[0] - Vb[0]) <= 2e-3 * 1.6e4
    got = to_dense(*o.export_local(), 512)[0]
    assert np.max(np.abs(got - f)) <= 0.05 * np.max(f)


def test_sparse_lists_equal_the_dense_velocity_space():
    """Absent blocks read as zero and every block that receives mass joins
    the list, so the sparse step gives the dense one's values exactly; the
    list is the old list plus the blocks holding a nonzero value."""
    n, g = (2, 2, 1), geom((5, 5, 5))
    st = random_state(n, g["nblk"], 31, density=0.25, scale=1e-12)
    dense = to_dense(*st, 125)
    b = np.arange(125)
    bc = np.stack([b % 5, (b // 5) % 5, b // 25], 1)
    edge = np.any((bc == 0) | (bc == 4), 1)
    dense[:, edge] = 0.0     # nothing at the mesh's faces, so nothing leaves it
    keep = [np.nonzero(np.any(dense[c] != 0, axis=1))[0] for c in range(dense.shape[0])]
    off = np.zeros(len(keep) + 1, np.int64)
    off[1:] = np.cumsum([k.size for k in keep])
    ids = np.concatenate(keep).astype(np.int32)
    vals = np.concatenate([dense[c, k].reshape(-1) for c, k in enumerate(keep)])
    rng = np.random.default_rng(32)
    nc = int(np.prod(n))
    EB = np.concatenate([rng.normal(0, 1e-4, (nc, 3)), rng.normal(0, 1e-8, (nc, 3))], 1)
    dt = 0.25 / (QM * 1.5e-8)
    s = partition(n, (off, ids, vals), g)
    d = partition(n, dense_to_csr(dense), g)
    s.accelerate(dt, QM, EB)
    d.accelerate(dt, QM, EB)
    so, si, sf = s.export_local()
    ds = to_dense(so, si, sf, 125)
    dd = to_dense(*d.export_local(), 125)
    assert np.array_equal(ds, dd)
    for c in range(nc):
        lst = set(si[so[c]:so[c + 1]].tolist())
        want = set(keep[c].tolist()) | set(np.nonzero(np.any(dd[c] != 0, axis=1))[0].tolist())
        assert lst == want

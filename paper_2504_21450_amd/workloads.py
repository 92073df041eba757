"""Seeded synthetic plasma states for the Vlasov translation path.

This module only *samples* initial distribution functions f(x, v) on a sparse
velocity mesh; it contains no part of the translation method (no
reconstruction, flux, remap or pruning step).  Both the CPU oracle and the HIP
library are fed from here, so neither side's arithmetic ever produces the
other's input.

State layout (local cells only, x fastest):
  offsets : int64[ncell + 1]   CSR row pointers, in blocks
  ids     : int32[nblocks]     global velocity-block ids, ascending per cell
  f       : float64[nblocks*64] 64 phase-space densities per block [s^3 m^-6]

Velocity mesh: nblk[d] blocks of 4 cells per axis; block id
  b = bx + nblk_x * (by + nblk_y * bz); lane within a block l = ix + 4 iy + 16 iz;
cell-centre velocity v_d(j) = vmin_d + (j + 1/2) dv_d with j = 4 b_d + i_d.

The workloads follow the physical setups of the paper's scaling runs
(Section 4.1: T = 1e5 K, n = 1e6 m^-3, V_x = 100 km/s, dv = 30 km/s; Section
2.2: cold solar wind at -750 km/s, dv = 40 km/s), since the paper's own
datasets are not public.  Initial f is a point sample of the analytic
distribution at velocity-cell centres times (1 + 0.01 u), u uniform in
[-1, 1) from a counter-based SplitMix64 stream (Steele, Lea & Flood 2014)
keyed by (seed, local cell, block id, lane), so any sub-box can be regenerated
independently of list selection and of the order of generation.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

M_P = 1.67262192e-27  # proton mass [kg]
K_B = 1.380649e-23    # Boltzmann constant [J/K]

VL_F64, VL_F32, VL_BF16 = 0, 1, 2


@dataclass
class Workload:
    name: str
    n: tuple            # local spatial cells per axis
    dx: tuple           # spatial cell size [m]
    nblk: tuple         # velocity blocks per axis
    vmin: tuple         # lower velocity-mesh edge [m/s]
    dv: tuple           # velocity cell size [m/s]
    dt: float           # time step [s]
    steps: int
    sparse_min: float   # block-content threshold [s^3 m^-6]; <= 0: no pruning
    vbuffer: int        # velocity-space buffer: 0, 6 (face) or 26 neighbours
    storage: int = VL_F64
    order: tuple = (0, 1, 2)
    offsets: np.ndarray = field(default=None, repr=False)
    ids: np.ndarray = field(default=None, repr=False)
    f: np.ndarray = field(default=None, repr=False)
    seed: int = 0
    # the physical fields the state was sampled from (per local cell)
    fields: dict = field(default=None, repr=False)

    @property
    def ncell(self):
        return int(np.prod(self.n))

    @property
    def nblocks(self):
        return int(self.offsets[-1])

    @property
    def nv(self):
        return tuple(4 * b for b in self.nblk)

    def max_courant(self):
        c = 0.0
        for d in range(3):
            nv = 4 * self.nblk[d]
            vlo = self.vmin[d] + 0.5 * self.dv[d]
            vhi = self.vmin[d] + (nv - 0.5) * self.dv[d]
            c = max(c, max(abs(vlo), abs(vhi)) * self.dt / self.dx[d])
        return c


# --------------------------------------------------------------------------
# counter-based uniform noise (SplitMix64 finaliser over a counter)
# --------------------------------------------------------------------------
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(counter: np.ndarray, seed: int) -> np.ndarray:
    """SplitMix64 output for state = seed + (counter + 1) * golden (uint64)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (counter.astype(np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(counter: np.ndarray, seed: int) -> np.ndarray:
    """u in [-1, 1) with 53 random bits."""
    z = splitmix64(counter, seed)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 / 9007199254740992.0) - 1.0


# --------------------------------------------------------------------------
# smooth periodic fields from seeded sine sums
# --------------------------------------------------------------------------
def sine_sum_field(rng, n, nmodes=3):
    """Normalised periodic field s(x) in [-1, 1] on an n-box of cell centres.

    s = sum_m a_m sin(2 pi k_m . x / L + phi_m) / sum_m |a_m|,
    k_m integer in {-2..2}^3 \\ {0}."""
    ks = []
    while len(ks) < nmodes:
        k = rng.integers(-2, 3, size=3)
        if np.any(k != 0):
            ks.append(k)
    amps = rng.uniform(0.5, 1.0, size=nmodes)
    phases = rng.uniform(0.0, 2 * np.pi, size=nmodes)
    x = [(np.arange(n[d]) + 0.5) / n[d] for d in range(3)]
    X, Y, Z = np.meshgrid(x[0], x[1], x[2], indexing="ij")
    s = np.zeros(X.shape)
    for k, a, ph in zip(ks, amps, phases):
        s += a * np.sin(2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)
    s /= amps.sum()
    # (x, y, z) -> flat x-fastest
    return np.ascontiguousarray(s.transpose(2, 1, 0)).reshape(-1)


# --------------------------------------------------------------------------
# velocity-space geometry
# --------------------------------------------------------------------------
def _lane_offsets():
    l = np.arange(64)
    return np.stack([l & 3, (l >> 2) & 3, l >> 4], axis=1)  # (64, 3)


def _block_coords(nblk):
    b = np.arange(nblk[0] * nblk[1] * nblk[2])
    return np.stack([b % nblk[0], (b // nblk[0]) % nblk[1], b // (nblk[0] * nblk[1])], axis=1)


def _dilate(mask, nblk, vbuffer):
    """mask: (m, NB) bool -> dilation by the face (6) or full (26) neighbours."""
    if vbuffer == 0:
        return mask.copy()
    m = mask.shape[0]
    g = mask.reshape(m, nblk[2], nblk[1], nblk[0])
    out = g.copy()
    if vbuffer == 6:
        shifts = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    else:
        shifts = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
                  if (a, b, c) != (0, 0, 0)]
    for sx, sy, sz in shifts:
        src = [slice(None)] * 4
        dst = [slice(None)] * 4
        for ax, s in ((3, sx), (2, sy), (1, sz)):
            if s == 1:
                dst[ax] = slice(1, None)
                src[ax] = slice(0, -1)
            elif s == -1:
                dst[ax] = slice(0, -1)
                src[ax] = slice(1, None)
        out[tuple(dst)] |= g[tuple(src)]
    return out.reshape(m, -1)


# --------------------------------------------------------------------------
# distribution-function models
# --------------------------------------------------------------------------
# A model maps an array of local-cell indices (m,) to a list of components;
# each component is a dict of per-cell arrays: n (m,) [m^-3], V (m, 3)
# [m/s], Tpar, Tperp (m,) [K] and bhat (m, 3) (unit vector of the parallel
# direction).  An isotropic Maxwellian has Tpar == Tperp; a component with
# n = 0 is absent for that cell.

def _component_f(v, n, V, Tpa, Tpe, bh):
    """(Bi-)Maxwellian at velocities v (p, 64, 3); parameters per pair (p,)."""
    u = v - V[:, None, :]
    upar = np.einsum("pli,pi->pl", u, bh)
    u2 = np.einsum("pli,pli->pl", u, u)
    uperp2 = np.maximum(u2 - upar * upar, 0.0)
    spa = (K_B / M_P) * Tpa
    spe = (K_B / M_P) * Tpe
    norm = n / ((2.0 * np.pi) ** 1.5 * spe * np.sqrt(spa))
    return norm[:, None] * np.exp(-0.5 * upar * upar / spa[:, None] - 0.5 * uperp2 / spe[:, None])


def _component_radius2(comp, thresh):
    """Squared radius beyond which 1.01 f_component < thresh / 2 (so a sum of
    <= 2 components stays below thresh); -1 where the peak is too low."""
    spa = (K_B / M_P) * comp["Tpar"]
    spe = (K_B / M_P) * comp["Tperp"]
    with np.errstate(divide="ignore", invalid="ignore"):   # absent components
        peak = comp["n"] / ((2.0 * np.pi) ** 1.5 * spe * np.sqrt(spa))
        r = 1.01 * peak / (0.5 * thresh)
    out = np.full(r.shape, -1.0)
    ok = r > 1.0
    out[ok] = 2.0 * np.maximum(spa, spe)[ok] * np.log(r[ok])
    return out


def sample_cells(models, nblk, vmin, dv, sparse_min, vbuffer, seed, cell_ids,
                 threads=None, batch=256):
    """Sample the sparse state of the cells whose global local-cell indices are
    `cell_ids` (x-fastest numbering of the full local box).

    Block selection: with sparse_min > 0, a block is kept if any of its 64
    sampled values is >= sparse_min, plus the `vbuffer` velocity neighbours of
    such blocks (clipped to the mesh).  With sparse_min <= 0 every block is
    kept (dense mesh)."""
    NB = nblk[0] * nblk[1] * nblk[2]
    bc = _block_coords(nblk)                      # (NB, 3)
    lo = _lane_offsets()                          # (64, 3)
    vmin = np.asarray(vmin, dtype=np.float64)
    dv = np.asarray(dv, dtype=np.float64)
    # block centre-grid bounding boxes of the velocity-cell centres
    blo = vmin + (4 * bc + 0.5) * dv
    bhi = vmin + (4 * bc + 3.5) * dv

    def values(cells_global, comps, pc, pb):
        v = vmin + (4 * bc[pb][:, None, :] + lo[None, :, :] + 0.5) * dv  # (p, 64, 3)
        fv = np.zeros(v.shape[:2])
        for comp in comps:
            n = comp["n"][pc]
            sel = n > 0
            if not np.any(sel):
                continue
            fv[sel] += _component_f(v[sel], n[sel], comp["V"][pc][sel], comp["Tpar"][pc][sel],
                                    comp["Tperp"][pc][sel], comp["bhat"][pc][sel])
        counter = ((cells_global[pc].astype(np.int64) * NB + pb)[:, None] * 64
                   + np.arange(64)[None, :])
        u = uniform_pm1(counter, seed)
        return fv * (1.0 + 0.01 * u)

    def do_batch(cb):
        cells_global = np.asarray(cb, dtype=np.int64)
        m = cells_global.size
        comps = models(cells_global)
        if sparse_min > 0:
            cand = np.zeros((m, NB), dtype=bool)
            for comp in comps:
                r2 = _component_radius2(comp, sparse_min)
                V = comp["V"]
                near = np.clip(V[:, None, :], blo[None], bhi[None])
                d2 = np.sum((near - V[:, None, :]) ** 2, axis=2)
                cand |= (d2 <= r2[:, None]) & (comp["n"] > 0)[:, None]
            union = cand | _dilate(cand, nblk, vbuffer)
            pc, pb = np.nonzero(union)
            fv = values(cells_global, comps, pc, pb)
            content = np.zeros((m, NB), dtype=bool)
            content[pc, pb] = np.any(fv >= sparse_min, axis=1)
            final = _dilate(content, nblk, vbuffer)
            keep = final[pc, pb]
            pc, pb, fv = pc[keep], pb[keep], fv[keep]
        else:
            pc = np.repeat(np.arange(m), NB)
            pb = np.tile(np.arange(NB), m)
            fv = values(cells_global, comps, pc, pb)
        counts = np.bincount(pc, minlength=m)
        return counts, pb.astype(np.int32), fv.reshape(-1)

    cell_ids = np.asarray(cell_ids, dtype=np.int64)
    batches = [cell_ids[i:i + batch] for i in range(0, cell_ids.size, batch)]
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    if threads > 1 and len(batches) > 1:
        with ThreadPoolExecutor(threads) as ex:
            res = list(ex.map(do_batch, batches))
    else:
        res = [do_batch(b) for b in batches]
    counts = np.concatenate([r[0] for r in res]) if res else np.zeros(0, np.int64)
    offsets = np.zeros(cell_ids.size + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    ids = np.concatenate([r[1] for r in res]) if res else np.zeros(0, np.int32)
    f = np.concatenate([r[2] for r in res]) if res else np.zeros(0)
    return offsets, ids, f


def _iso(n, V, T):
    """Isotropic Maxwellian component from per-cell arrays n (m,), V (m, 3), T (m,)."""
    n = np.asarray(n, dtype=np.float64)
    m = n.size
    return {"n": n, "V": np.broadcast_to(np.asarray(V, dtype=np.float64), (m, 3)),
            "Tpar": np.broadcast_to(np.asarray(T, dtype=np.float64), (m,)),
            "Tperp": np.broadcast_to(np.asarray(T, dtype=np.float64), (m,)),
            "bhat": np.broadcast_to(np.array([1.0, 0.0, 0.0]), (m, 3))}


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------
def maxwellian_small(seed=21451, n=(8, 8, 8)):
    """Dense FP64 case: 8^3 periodic cells, dx = 300 km, 16^3 velocity cells
    (4^3 blocks) with dv = 40 km/s over +-320 km/s; proton Maxwellian with
    n(x) = 1e6 (1 + 0.2 sin(2 pi x / L)), V = (100, 0, 0) km/s, T = 1e5 K,
    +-1 % noise; dt such that the largest cell-centre |v| dt / dx = 0.5."""
    dx = (300e3,) * 3
    nblk = (4, 4, 4)
    dv = (40e3,) * 3
    vmin = (-320e3,) * 3
    Lx = n[0] * dx[0]

    def model(c):
        xc = (c % n[0] + 0.5) * dx[0]
        return [_iso(1e6 * (1.0 + 0.2 * np.sin(2 * np.pi * xc / Lx)), (100e3, 0.0, 0.0), 1e5)]

    offsets, ids, f = sample_cells(model, nblk, vmin, dv, 0.0, 0, seed,
                                   np.arange(n[0] * n[1] * n[2]))
    vmax_c = 320e3 - 20e3
    dt = 0.5 * dx[0] / vmax_c
    return Workload("maxwellian-8x8x8-dense-v16", tuple(n), dx, nblk, vmin, dv, dt, 10,
                    0.0, 0, VL_F64, (0, 1, 2), offsets, ids, f, seed)


def _smooth_fields(seed, n):
    rng = np.random.default_rng(seed)
    sn = sine_sum_field(rng, n)
    sT = sine_sum_field(rng, n)
    sV = [sine_sum_field(rng, n) for _ in range(3)]
    dens = 1e6 + 3e6 * 0.5 * (sn + 1.0)
    temp = 10.0 ** (5.0 + 0.5 * (sT + 1.0))
    vel = np.stack([600e3 / math.sqrt(3.0) * s for s in sV], axis=1)
    return dens, temp, vel


def maxwellian_sparse(seed=21452, n=(64, 64, 32), cells=None, threads=None, steps=20,
                      storage=VL_F64):
    """Sparse FP64 case on a coalesced-ghost partition: 64 x 64 x 32 periodic
    cells, dx = 300 km, 100^3 velocity cells (25^3 blocks), dv = 30 km/s over
    +-1500 km/s; one Maxwellian per cell with n in [1e6, 4e6] m^-3 (linear),
    T in [1e5, 1e6] K (logarithmic) and each bulk-velocity component in
    +-600/sqrt(3) km/s, all from seeded periodic sine sums; blocks kept where
    max f >= 1e-15 s^3 m^-6 plus the 6 face-neighbour blocks.  dt gives a
    largest Courant number of 1/2 (dx = 300 km is assumed; only v dt / dx
    matters).  `cells` restricts sampling to a subset of local cells (the
    fields stay those of the full box)."""
    dx = (300e3,) * 3
    nblk = (25, 25, 25)
    dv = (30e3,) * 3
    vmin = (-1500e3,) * 3
    dens, temp, vel = _smooth_fields(seed, n)

    def model(c):
        return [_iso(dens[c], vel[c], temp[c])]

    if cells is None:
        cells = np.arange(n[0] * n[1] * n[2])
    offsets, ids, f = sample_cells(model, nblk, vmin, dv, 1e-15, 6, seed, cells,
                                   threads=threads)
    dt = 0.5 * dx[0] / 1485e3
    name = "maxwellian-sparse-%dx%dx%d-v100" % tuple(n)
    w = Workload(name, tuple(n), dx, nblk, vmin, dv, dt, steps, 1e-15, 6, storage, (0, 1, 2),
                 offsets, ids, f, seed)
    w.fields = {"n": dens, "T": temp, "V": vel}
    return w


# --------------------------------------------------------------------------
# uneven batched cells: cold solar wind and hot magnetosheath-like mixtures
# --------------------------------------------------------------------------
# per-cell component table: (ncell, 2, 10) float64 rows
#   [n, Vx, Vy, Vz, Tpar, Tperp, bx, by, bz, 0]; n = 0 marks an absent component
NCOMP, NPAR = 2, 10
BHAT = np.array([1.0, 1.0, 1.0]) / math.sqrt(3.0)   # parallel direction (Section 4.1's B)


def blob_field(rng, n, nblobs=16, rmin=3.0, rmax=8.0):
    """Sum of `nblobs` periodic Gaussians exp(-|x - c|^2 / (2 r^2)) over the
    cell centres of an n-box (minimum-image distances, in cells), centres
    uniform in the box and radii uniform in [rmin, rmax]; flat x-fastest."""
    c = rng.uniform(0.0, 1.0, size=(nblobs, 3)) * np.asarray(n, dtype=np.float64)
    r = rng.uniform(rmin, rmax, size=nblobs)
    x = [np.arange(n[d]) + 0.5 for d in range(3)]
    out = np.zeros((n[2], n[1], n[0]))
    for k in range(nblobs):
        d2 = []
        for d in range(3):
            t = np.abs(x[d] - c[k, d])
            t = np.minimum(t, n[d] - t)
            d2.append(t * t)
        out += np.exp(-(d2[2][:, None, None] + d2[1][None, :, None] + d2[0][None, None, :])
                      / (2.0 * r[k] * r[k]))
    return out.reshape(-1)


def mixture_params(seed, n, hot_fraction):
    """Component table of the blob mixture.  Cells whose blob field lies in the
    top `hot_fraction` are hot: a bi-Maxwellian core (0.9 n_h, T_par = 5e6 K,
    T_perp = 1e7 K, V = 0) plus a beam (0.1 n_h, 800 km/s along bhat,
    T = 1e6 K), n_h = 1e6 m^-3; the others are cold solar wind (1e6 m^-3,
    T = 1e5 K, V = (-750, 0, 0) km/s, Section 2.2)."""
    rng = np.random.default_rng(seed)
    B = blob_field(rng, n)
    ncell = B.size
    hot = np.zeros(ncell, dtype=bool)
    nh = int(round(hot_fraction * ncell))
    if nh > 0:
        hot[np.argsort(-B, kind="stable")[:nh]] = True
    P = np.zeros((ncell, NCOMP, NPAR))
    cold = ~hot
    P[cold, 0, 0] = 1e6
    P[cold, 0, 1:4] = (-750e3, 0.0, 0.0)
    P[cold, 0, 4:6] = 1e5
    P[cold, 0, 6:9] = (1.0, 0.0, 0.0)
    P[hot, 0, 0] = 0.9e6
    P[hot, 0, 4] = 5e6
    P[hot, 0, 5] = 1e7
    P[hot, 0, 6:9] = BHAT
    P[hot, 1, 0] = 0.1e6
    P[hot, 1, 1:4] = 800e3 * BHAT
    P[hot, 1, 4:6] = 1e6
    P[hot, 1, 6:9] = BHAT
    return P, hot


def table_model(P):
    """A sample_cells model reading the component table P."""
    def model(c):
        comps = []
        for k in range(P.shape[1]):
            q = P[c, k]
            comps.append({"n": q[:, 0], "V": q[:, 1:4], "Tpar": q[:, 4], "Tperp": q[:, 5],
                          "bhat": q[:, 6:9]})
        return comps
    return model


def blob_mixture(seed=21454, n=(96, 96, 48), hot_fraction=0.4, cells=None, threads=None,
                 steps=20, storage=VL_F32, sample=True):
    """Uneven batched cells: the blob mixture on an n-box with the velocity mesh
    of the sparse Maxwellian case (100^3 cells, dv = 30 km/s, +-1500 km/s),
    blocks kept where max f >= 1e-15 s^3 m^-6 plus the 6 face neighbours
    (about 80 blocks per cold cell, about 4000 per hot one).  The hot cells
    are the top `hot_fraction` of a field of 16 periodic Gaussian blobs of
    radius 3..8 cells (0.4: the uneven case; about 0.1: a mean near 500
    blocks).  With sample=False only the component table is built (for
    device-side sampling); `cells` restricts host sampling to a subset."""
    dx = (300e3,) * 3
    nblk = (25, 25, 25)
    dv = (30e3,) * 3
    vmin = (-1500e3,) * 3
    P, hot = mixture_params(seed, n, hot_fraction)
    offsets = ids = f = None
    if sample:
        if cells is None:
            cells = np.arange(n[0] * n[1] * n[2])
        offsets, ids, f = sample_cells(table_model(P), nblk, vmin, dv, 1e-15, 6, seed, cells,
                                       threads=threads, batch=16)
    dt = 0.5 * dx[0] / 1485e3
    name = "blob-mixture-%dx%dx%d-hot%g-v100" % (tuple(n) + (hot_fraction,))
    w = Workload(name, tuple(n), dx, nblk, vmin, dv, dt, steps, 1e-15, 6, storage, (0, 1, 2),
                 offsets, ids, f, seed)
    w.fields = {"params": P, "hot": hot}
    return w


def lorentz_fields(ncell, seed=21455, B0=1e-8, vdrift=1e5, vpar=6e4, dt=None, qm=9.58e7):
    """Seeded per-cell fields for an acceleration step: (ncell, 6) as Ex, Ey,
    Ez [V/m], Bx, By, Bz [T], x fastest.  B of random direction and
    0.5-1.5 B0; E = -Vd x B + E_par b with Vd perpendicular to B (normal
    components of rms vdrift / sqrt(3)) and E_par moving a velocity by up to
    vpar over dt (default dt: a gyration angle of 0.3 rad at B0)."""
    if dt is None:
        dt = 0.3 / (qm * B0)
    rng = np.random.default_rng(seed)
    b = rng.normal(size=(ncell, 3))
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    B = b * (B0 * rng.uniform(0.5, 1.5, ncell))[:, None]
    Vd = rng.normal(size=(ncell, 3)) * vdrift / math.sqrt(3.0)
    Vd -= np.sum(Vd * b, axis=1, keepdims=True) * b
    Epar = rng.uniform(-1.0, 1.0, ncell) * vpar / (qm * dt)
    E = -np.cross(Vd, B) + Epar[:, None] * b
    return np.concatenate([E, B], 1), dt


def subbox_cells(n, lo, size, halo):
    """Local-cell indices (x-fastest, periodic wrap) of the box
    [lo - halo, lo + size + halo) of an n-box, in x-fastest order of the
    padded sub-box."""
    rng = [np.arange(lo[d] - halo, lo[d] + size[d] + halo) % n[d] for d in range(3)]
    z, y, x = np.meshgrid(rng[2], rng[1], rng[0], indexing="ij")
    return (x + n[0] * (y + n[1] * z)).reshape(-1)


def take_cells(offsets, ids, f, cells):
    """Gather the CSR rows `cells` of a state into a new CSR state."""
    cells = np.asarray(cells, dtype=np.int64)
    counts = offsets[cells + 1] - offsets[cells]
    no = np.zeros(cells.size + 1, dtype=np.int64)
    np.cumsum(counts, out=no[1:])
    if no[-1] == 0:
        return no, np.zeros(0, np.int32), np.zeros(0)
    starts = np.repeat(offsets[cells] - no[:-1], counts)
    blk = np.arange(no[-1]) + starts
    ni = ids[blk]
    nf = f.reshape(-1, 64)[blk].reshape(-1)
    return no, ni, nf

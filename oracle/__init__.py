"""FP64 CPU oracle for the Vlasov translation step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the slow reference the HIP library is checked
against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
may import this package; the product path never does, and this package imports
nothing from the product package.

The C source (vlasov_oracle.c) documents what is computed and which part of the
paper each step follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vlasov_oracle.c")
_LIB = os.path.join(_HERE, "libvlasov_oracle.so")

COALESCED = 0
PER_SWEEP = 1

M_P = 1.67262192e-27


def build(force=True):
    """Compile the oracle with gcc (plain C11, OpenMP, no FMA contraction)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        L.vlo_create.restype = C.c_void_p
        L.vlo_create.argtypes = [i32p, i32p, f64p, f64p, f64p, i32p, C.c_double, C.c_int32]
        L.vlo_destroy.argtypes = [C.c_void_p]
        L.vlo_set_cell.restype = C.c_int
        L.vlo_set_cell.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, i32p, f64p]
        L.vlo_cell_count.restype = C.c_int32
        L.vlo_cell_count.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]
        L.vlo_get_cell.restype = C.c_int
        L.vlo_get_cell.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, i32p, f64p]
        L.vlo_load_local.restype = C.c_int
        L.vlo_load_local.argtypes = [C.c_void_p, i64p, i32p, f64p]
        L.vlo_local_blocks.restype = C.c_int64
        L.vlo_local_blocks.argtypes = [C.c_void_p]
        L.vlo_export_local.argtypes = [C.c_void_p, i64p, i32p, f64p]
        L.vlo_set_courant_override.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
        L.vlo_fill_ghosts.argtypes = [C.c_void_p]
        L.vlo_mark_ghosts_valid.argtypes = [C.c_void_p]
        L.vlo_update_box.argtypes = [C.c_void_p, C.c_int32, C.c_int32, i32p, i32p]
        L.vlo_set_gt_level.restype = C.c_int32
        L.vlo_set_gt_level.argtypes = [C.c_void_p, C.c_int32]
        L.vlo_set_edges.restype = C.c_int32
        L.vlo_set_edges.argtypes = [C.c_void_p, C.c_int32]
        L.vlo_step.restype = C.c_int
        L.vlo_step.argtypes = [C.c_void_p, C.c_double, C.c_int32, f64p]
        L.vlo_local_mass.restype = C.c_double
        L.vlo_local_mass.argtypes = [C.c_void_p]
        L.vlo_moments.argtypes = [C.c_void_p, f64p, f64p, f64p, f64p]
        L.vlo_ppm_line.argtypes = [f64p, C.c_int, C.c_double, f64p, f64p, f64p, f64p, f64p, f64p]
        L.vlo_accel_map.argtypes = [f64p, f64p, C.c_double, C.c_double, f64p, f64p]
        L.vlo_slice_factors.restype = C.c_int
        L.vlo_slice_factors.argtypes = [f64p, f64p, i32p, f64p]
        L.vlo_remap_column.argtypes = [f64p, C.c_int, C.c_double, C.c_double, f64p]
        L.vlo_accelerate.restype = C.c_int
        L.vlo_accelerate.argtypes = [C.c_void_p, C.c_double, C.c_double, f64p, i32p, f64p]
        _lib = L
    return _lib


def ppm_line(a, c):
    """1D remap of a line a[0..L) with Courant number c.  Returns a dict with
    'out' (cells [3, L-3) updated, others copied from a), 'face' (a_{i+1/2}),
    'al', 'ar', 'a6' (limited profile per cell) and 'flux' (F_{i+1/2})."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    L = a.size
    out = a.copy()
    arrs = {k: np.full(L, np.nan) for k in ("face", "al", "ar", "a6", "flux")}
    lib().vlo_ppm_line(a, L, float(c), out, arrs["face"], arrs["al"], arrs["ar"], arrs["a6"],
                       arrs["flux"])
    arrs["out"] = out
    return arrs


def accel_map(E, B, qm, dt):
    """The exact velocity map of constant fields E, B over dt for charge-to-
    mass ratio qm: v' = A v + c.  Returns (A (3x3), c (3,))."""
    A = np.zeros(9)
    c = np.zeros(3)
    lib().vlo_accel_map(np.ascontiguousarray(E, np.float64), np.ascontiguousarray(B, np.float64),
                        float(qm), float(dt), A, c)
    return A.reshape(3, 3), c


def slice_factors(A, c, order=(0, 1, 2)):
    """The three one-coordinate maps of the SLICE-3D split of v' = A v + c in
    the given axis order: a (3, 4) array, row k = coefficients of coordinates
    0..2 and the constant of the map that sets coordinate order[k]; None if a
    step is not invertible and order-preserving."""
    M = np.zeros(12)
    rc = lib().vlo_slice_factors(np.ascontiguousarray(A, np.float64).reshape(-1),
                                 np.ascontiguousarray(c, np.float64), np.array(order, np.int32), M)
    return None if rc else M.reshape(3, 4)


def remap_column(a, alpha, sigma):
    """Conservative remap of a column of unit cells under u -> alpha u + sigma."""
    a = np.ascontiguousarray(a, np.float64)
    out = np.zeros_like(a)
    lib().vlo_remap_column(a, a.size, float(alpha), float(sigma), out)
    return out


class OraclePartition:
    """A periodic partition of n[0] x n[1] x n[2] cells padded by 3 ghost
    layers; the block store and every step run in the C oracle."""

    H = 3

    def __init__(self, n, nblk, dx, vmin, dv, order=(0, 1, 2), sparse_min=0.0, vbuffer=0):
        self.n = tuple(int(v) for v in n)
        self.P = tuple(v + 2 * self.H for v in self.n)
        self.nblk = tuple(int(v) for v in nblk)
        self.dx, self.vmin, self.dv = tuple(dx), tuple(vmin), tuple(dv)
        self.order = tuple(order)
        self._h = lib().vlo_create(np.array(self.n, np.int32), np.array(self.nblk, np.int32),
                                   np.array(dx, np.float64), np.array(vmin, np.float64),
                                   np.array(dv, np.float64), np.array(order, np.int32),
                                   float(sparse_min), int(vbuffer))

    @classmethod
    def from_workload(cls, w, order=None, gt_level=3):
        p = cls(w.n, w.nblk, w.dx, w.vmin, w.dv, order or w.order, w.sparse_min, w.vbuffer)
        p.load_local(w.offsets, w.ids, w.f)
        if gt_level != 3:
            p.set_gt_level(gt_level)
        return p

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().vlo_destroy(h)
            self._h = None

    # -- state ---------------------------------------------------------------
    def load_local(self, offsets, ids, f):
        rc = lib().vlo_load_local(self._h, np.ascontiguousarray(offsets, np.int64),
                                  np.ascontiguousarray(ids, np.int32),
                                  np.ascontiguousarray(f, np.float64))
        if rc:
            raise ValueError("vlo_load_local: %d" % rc)

    def set_cell(self, x, y, z, ids, f):
        ids = np.ascontiguousarray(ids, np.int32)
        f = np.ascontiguousarray(f, np.float64)
        if ids.size == 0:
            ids = np.zeros(1, np.int32)
            f = np.zeros(64)
            cnt = 0
        else:
            cnt = ids.size
        rc = lib().vlo_set_cell(self._h, x, y, z, cnt, ids, f)
        if rc:
            raise ValueError("vlo_set_cell: %d" % rc)

    def load_padded(self, offsets, ids, f):
        """Set every cell of the padded box (x fastest) from a CSR state —
        used to supply an explicit ghost domain instead of a periodic one."""
        P = self.P
        q = 0
        f2 = f.reshape(-1, 64)
        for z in range(P[2]):
            for y in range(P[1]):
                for x in range(P[0]):
                    b0, b1 = offsets[q], offsets[q + 1]
                    self.set_cell(x, y, z, ids[b0:b1], f2[b0:b1].reshape(-1))
                    q += 1

    def get_cell(self, x, y, z):
        n = lib().vlo_cell_count(self._h, x, y, z)
        ids = np.zeros(max(n, 1), np.int32)
        f = np.zeros(max(n, 1) * 64)
        lib().vlo_get_cell(self._h, x, y, z, ids, f)
        return ids[:n], f[:n * 64]

    def export_local(self):
        nb = lib().vlo_local_blocks(self._h)
        offsets = np.zeros(int(np.prod(self.n)) + 1, np.int64)
        ids = np.zeros(max(nb, 1), np.int32)
        f = np.zeros(max(nb, 1) * 64)
        lib().vlo_export_local(self._h, offsets, ids, f)
        return offsets, ids[:nb], f[:nb * 64]

    def set_courant_override(self, table):
        if table is None:
            lib().vlo_set_courant_override(self._h, None, 0)
            return
        t = np.ascontiguousarray(table, np.float64)
        self._cover = t
        lib().vlo_set_courant_override(self._h, t.ctypes.data, t.shape[1])

    # -- the method ----------------------------------------------------------
    def fill_ghosts(self):
        lib().vlo_fill_ghosts(self._h)

    def set_gt_level(self, k):
        """Ghost Translation level of the coalesced mode (Section 3.2): the
        later shears' ghost layers computed by each shear, 1..3."""
        if lib().vlo_set_gt_level(self._h, int(k)) != 0:
            raise ValueError("gt level must be 1, 2 or 3")

    def set_edges(self, mask):
        """Faces at the simulation edge (bit 2d low, 2d+1 high face of axis
        d): the padded cells beyond them are boundary cells, kept as loaded."""
        if lib().vlo_set_edges(self._h, int(mask)) != 0:
            raise ValueError("edge mask must be in 0..63")

    def update_box(self, mode, s):
        lo = np.zeros(3, np.int32)
        hi = np.zeros(3, np.int32)
        lib().vlo_update_box(self._h, mode, s, lo, hi)
        return tuple(lo), tuple(hi)

    def step(self, dt, mode=COALESCED):
        st = np.zeros(8)
        rc = lib().vlo_step(self._h, float(dt), int(mode), st)
        if rc:
            raise RuntimeError("vlo_step: %d" % rc)
        return {"mass_before": st[0], "mass_after": st[1], "pruned_mass": st[2],
                "updates": (int(st[3]), int(st[4]), int(st[5])), "blocks": int(st[6])}

    def accelerate(self, dt, qm, EB, order=(0, 1, 2)):
        """One acceleration step of the local cells (fields EB: (ncell, 6) as
        Ex, Ey, Ez, Bx, By, Bz per cell, x fastest)."""
        st = np.zeros(4)
        EB = np.ascontiguousarray(EB, np.float64).reshape(-1)
        rc = lib().vlo_accelerate(self._h, float(dt), float(qm), EB, np.array(order, np.int32), st)
        if rc:
            raise RuntimeError("vlo_accelerate: %d" % rc)
        return {"mass_before": st[0], "mass_after": st[1], "pruned_mass": st[2], "blocks": int(st[3])}

    def step_rc(self, dt, mode=COALESCED):
        st = np.zeros(8)
        return lib().vlo_step(self._h, float(dt), int(mode), st)

    def local_mass(self):
        return lib().vlo_local_mass(self._h)

    def moments(self):
        nc = int(np.prod(self.n))
        dens = np.zeros(nc)
        V = np.zeros(nc * 3)
        P = np.zeros(nc * 6)
        tot = np.zeros(1)
        lib().vlo_moments(self._h, dens, V, P, tot)
        return dens, V.reshape(nc, 3), P.reshape(nc, 6), float(tot[0])

"""ctypes binding of libvlasov.so (C ABI in include/vlasov.h).

Argument marshalling only: every step of the translation runs in the HIP
library.  PyTorch provides the device workspace and the stream.  There is no
fallback: if the library is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvlasov.so")

VL_F64, VL_F32, VL_BF16 = 0, 1, 2
VL_COALESCED, VL_PER_SWEEP = 0, 1
VL_OK, VL_ERR_ARG, VL_ERR_CFL, VL_ERR_CAPACITY, VL_ERR_STALE_GHOSTS, VL_ERR_HIP, VL_ERR_STATE = (
    0, -1, -2, -3, -4, -5, -6)
VL_ERR_SCRATCH = -7
VL_ERR_SPLIT = -8

EXPORTED = ("vl_workspace_bytes", "vl_init_partition", "vl_load_values", "vl_fill_ghosts", "vl_fill_ghosts_from", "vl_translate_step",
            "vl_moments", "vl_local_block_count", "vl_export_state", "vl_export_cells",
            "vl_set_courant_override", "vl_counters", "vl_profile_start", "vl_profile_stop",
            "vl_autotune", "vl_set_variant", "vl_set_shear_variants", "vl_get_shear_variants",
            "vl_graph_step", "vl_sync", "vl_destroy",
            "vl_status_string", "vl_moments_static", "vl_accelerate")


class VlDesc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("nblk", C.c_int32 * 3), ("order", C.c_int32 * 3),
                ("storage", C.c_int32), ("stencil", C.c_int32), ("gt_level", C.c_int32),
                ("vbuffer", C.c_int32), ("edges", C.c_int32),
                ("dx", C.c_double * 3), ("vmin", C.c_double * 3), ("dv", C.c_double * 3),
                ("sparse_min", C.c_double), ("block_capacity", C.c_int64),
                ("ghost_block_capacity", C.c_int64)]


class VlStepStats(C.Structure):
    _fields_ = [("mass_before", C.c_double), ("mass_after", C.c_double),
                ("pruned_mass", C.c_double), ("ledger_mass", C.c_double),
                ("local_blocks", C.c_int64), ("updated_ps", C.c_int64 * 3),
                ("read_ps", C.c_int64 * 3), ("items", C.c_int64 * 3),
                ("device_errors", C.c_uint64)]


class VlasovError(RuntimeError):
    def __init__(self, call, status):
        self.status = status
        super().__init__("%s: %s (%d)" % (call, status_string(status), status))


_lib = None


def load():
    """Load libvlasov.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libvlasov.so not built: run `python -m paper_2504_21450_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.vl_workspace_bytes.restype = C.c_size_t
    L.vl_workspace_bytes.argtypes = [C.POINTER(VlDesc)]
    L.vl_init_partition.restype = C.c_int
    L.vl_init_partition.argtypes = [C.POINTER(VlDesc), vp, C.c_size_t, vp, vp, vp, vp, C.POINTER(vp)]
    L.vl_load_values.restype = C.c_int
    L.vl_load_values.argtypes = [vp, i64, i64, vp]
    L.vl_fill_ghosts.restype = C.c_int
    L.vl_fill_ghosts_from.restype = C.c_int
    L.vl_fill_ghosts_from.argtypes = [vp, vp]
    L.vl_fill_ghosts.argtypes = [vp]
    L.vl_translate_step.restype = C.c_int
    L.vl_translate_step.argtypes = [vp, dbl, i32, C.POINTER(VlStepStats)]
    L.vl_moments.restype = C.c_int
    L.vl_moments.argtypes = [vp, vp, vp, vp, vp]
    L.vl_moments_static.restype = C.c_int
    L.vl_moments_static.argtypes = [vp, vp, vp, vp, vp]
    L.vl_accelerate.restype = C.c_int
    L.vl_accelerate.argtypes = [vp, dbl, dbl, vp, vp, C.POINTER(VlStepStats)]
    L.vl_local_block_count.restype = C.c_int
    L.vl_local_block_count.argtypes = [vp, C.POINTER(i64)]
    L.vl_export_state.restype = C.c_int
    L.vl_export_state.argtypes = [vp, vp, vp, vp, i64]
    L.vl_export_cells.restype = C.c_int
    L.vl_export_cells.argtypes = [vp, vp, i64, vp, vp, vp, i64]
    L.vl_set_courant_override.restype = C.c_int
    L.vl_set_courant_override.argtypes = [vp, vp, i32]
    L.vl_counters.restype = C.c_int
    L.vl_counters.argtypes = [vp, vp, i32]
    L.vl_profile_start.restype = C.c_int
    L.vl_profile_start.argtypes = [vp, i32]
    L.vl_profile_stop.restype = C.c_int
    L.vl_profile_stop.argtypes = [vp, vp, vp]
    L.vl_autotune.restype = C.c_int
    L.vl_autotune.argtypes = [vp, dbl, i32, i32, vp, vp, i32]
    L.vl_set_variant.restype = C.c_int
    L.vl_set_variant.argtypes = [vp, i32]
    L.vl_set_shear_variants.restype = C.c_int
    L.vl_set_shear_variants.argtypes = [vp, vp]
    L.vl_get_shear_variants.restype = C.c_int
    L.vl_get_shear_variants.argtypes = [vp, vp, vp]
    L.vl_graph_step.restype = C.c_int
    L.vl_graph_step.argtypes = [vp, dbl, i32, i32]
    L.vl_sync.restype = C.c_int
    L.vl_sync.argtypes = [vp]
    L.vl_destroy.restype = None
    L.vl_destroy.argtypes = [vp]
    L.vl_status_string.restype = C.c_char_p
    L.vl_status_string.argtypes = [C.c_int]
    _lib = L
    return L


def status_string(s):
    return load().vl_status_string(int(s)).decode()


def _check(call, rc):
    if rc != VL_OK:
        raise VlasovError(call, rc)


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None and a.size else C.c_void_p(0)


def make_desc(n, nblk, dx, vmin, dv, order=(0, 1, 2), storage=VL_F64, sparse_min=0.0, vbuffer=0,
              block_capacity=1, ghost_block_capacity=1, stencil=2, gt_level=3, edges=0):
    d = VlDesc()
    for k in range(3):
        d.n[k], d.nblk[k], d.order[k] = int(n[k]), int(nblk[k]), int(order[k])
        d.dx[k], d.vmin[k], d.dv[k] = float(dx[k]), float(vmin[k]), float(dv[k])
    d.storage, d.stencil, d.gt_level, d.vbuffer = int(storage), int(stencil), int(gt_level), int(vbuffer)
    d.edges = int(edges)
    d.sparse_min = float(sparse_min)
    d.block_capacity = int(block_capacity)
    d.ghost_block_capacity = int(ghost_block_capacity)
    return d


def workspace_bytes(desc):
    return int(load().vl_workspace_bytes(C.byref(desc)))


def ghost_blocks_estimate(n, offsets):
    """Blocks the ghost domain holds after a periodic ghost update."""
    counts = np.diff(np.asarray(offsets)).reshape(n[2], n[1], n[0])
    padded = np.pad(counts, 3, mode="wrap")
    return int(padded.sum() - counts.sum())


class Partition:
    """One partition on one GPU: the block store lives in a torch uint8
    workspace tensor; all work runs on the torch stream current at creation."""

    def __init__(self, n, nblk, dx, vmin, dv, offsets, ids, f, storage=VL_F64, order=(0, 1, 2),
                 sparse_min=0.0, vbuffer=0, block_capacity=None, ghost_block_capacity=None,
                 device="cuda:0", slack=2.5, gt_level=3, edges=0):
        import torch

        self.torch = torch
        self.lib = load()
        self.n = tuple(int(v) for v in n)
        self.ncell = int(np.prod(self.n))
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        f = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
        nb = int(offsets[-1])
        NB = int(np.prod(nblk))
        nghost = int(np.prod([v + 6 for v in self.n])) - self.ncell
        # small partitions get room for a dense velocity mesh (no overflow
        # possible); large ones a multiple of the current block count
        if block_capacity is None:
            block_capacity = int(nb * slack) + 8 * self.ncell + 1024
            if self.ncell * NB <= 4_000_000:
                block_capacity = max(block_capacity, self.ncell * NB + 1024)
        if ghost_block_capacity is None:
            ghost_block_capacity = int(ghost_blocks_estimate(self.n, offsets) * slack) + 1024
            if nghost * NB <= 20_000_000:
                ghost_block_capacity = max(ghost_block_capacity, nghost * NB + 1024)
        self.desc = make_desc(n, nblk, dx, vmin, dv, order, storage, sparse_min, vbuffer,
                              block_capacity, ghost_block_capacity, gt_level=gt_level, edges=edges)
        self.ws_bytes = workspace_bytes(self.desc)
        if self.ws_bytes == 0:
            raise VlasovError("vl_workspace_bytes", VL_ERR_ARG)
        self.device = torch.device(device)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = self.lib.vl_init_partition(C.byref(self.desc), C.c_void_p(self.ws_ptr), self.ws_bytes,
                                        C.c_void_p(self.stream.cuda_stream), _ptr(offsets), _ptr(ids),
                                        _ptr(f), C.byref(h))
        _check("vl_init_partition", rc)
        self.h = h

    @classmethod
    def from_workload(cls, w, storage=None, device="cuda:0", order=None, **kw):
        return cls(w.n, w.nblk, w.dx, w.vmin, w.dv, w.offsets, w.ids, w.f,
                   storage=w.storage if storage is None else storage,
                   order=w.order if order is None else order, sparse_min=w.sparse_min,
                   vbuffer=w.vbuffer, device=device, **kw)

    def close(self):
        if getattr(self, "h", None):
            self.lib.vl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the path ----------------------------------------------------------
    def fill_ghosts(self):
        _check("vl_fill_ghosts", self.lib.vl_fill_ghosts(self.h))

    def step(self, dt, mode=VL_COALESCED, stats=False):
        st = VlStepStats() if stats else None
        rc = self.lib.vl_translate_step(self.h, float(dt), int(mode), C.byref(st) if stats else None)
        if rc != VL_OK and stats and st.device_errors:
            raise VlasovError("vl_translate_step (device error bits %#x)" % st.device_errors, rc)
        _check("vl_translate_step", rc)
        if not stats:
            return None
        return {"mass_before": st.mass_before, "mass_after": st.mass_after,
                "pruned_mass": st.pruned_mass, "ledger_mass": st.ledger_mass,
                "blocks": st.local_blocks, "updated_ps": tuple(st.updated_ps),
                "read_ps": tuple(st.read_ps), "items": tuple(st.items)}

    def accelerate(self, dt, qm, fields, order=None, stats=False):
        """Acceleration step in per-cell fields: `fields` is a device FP64
        tensor of 6 values per local cell (Ex, Ey, Ez, Bx, By, Bz), x fastest;
        order: the slice order (default x, y, z)."""
        t = self.torch
        assert fields.device.type == "cuda" and fields.dtype == t.float64 and fields.is_contiguous()
        assert fields.numel() == 6 * self.ncell
        o = (C.c_int32 * 3)(*order) if order is not None else None
        st = VlStepStats() if stats else None
        rc = self.lib.vl_accelerate(self.h, float(dt), float(qm), C.c_void_p(fields.data_ptr()), o,
                                    C.byref(st) if stats else None)
        if rc != VL_OK and stats and st.device_errors:
            raise VlasovError("vl_accelerate (device error bits %#x)" % st.device_errors, rc)
        _check("vl_accelerate", rc)
        if not stats:
            return None
        return {"mass_before": st.mass_before, "mass_after": st.mass_after,
                "pruned_mass": st.pruned_mass, "blocks": st.local_blocks}

    def accelerate_rc(self, dt, qm, fields, order=None):
        o = (C.c_int32 * 3)(*order) if order is not None else None
        return self.lib.vl_accelerate(self.h, float(dt), float(qm), C.c_void_p(fields.data_ptr()), o, None)

    def fill_ghosts_from(self, nbr):
        """Ghost update from the 27 partitions around this one (nbr[13] is
        self), indexed (dx+1) + 3(dy+1) + 9(dz+1); asynchronous."""
        arr = (C.c_void_p * 27)(*[q.h.value if hasattr(q.h, "value") else q.h for q in nbr])
        _check("vl_fill_ghosts_from", self.lib.vl_fill_ghosts_from(self.h, arr))

    def load_values(self, first_block, nblocks, dev_f):
        """Values of initial blocks [first_block, first_block + nblocks) from a
        device FP64 tensor (before the first step; asynchronous)."""
        _check("vl_load_values", self.lib.vl_load_values(self.h, int(first_block), int(nblocks),
                                                         C.c_void_p(dev_f.data_ptr())))

    def step_rc(self, dt, mode=VL_COALESCED):
        return self.lib.vl_translate_step(self.h, float(dt), int(mode), None)

    def graph_step(self, dt, mode=VL_COALESCED, nsteps=1):
        """nsteps whole steps (ghost update included in coalesced mode) replayed
        from recorded HIP graphs; asynchronous."""
        _check("vl_graph_step", self.lib.vl_graph_step(self.h, float(dt), int(mode), int(nsteps)))

    def moments(self, total=True):
        t = self.torch
        dn = t.empty(self.ncell, dtype=t.float64, device=self.device)
        dV = t.empty(self.ncell * 3, dtype=t.float64, device=self.device)
        dP = t.empty(self.ncell * 6, dtype=t.float64, device=self.device)
        tot = C.c_double(0.0)
        rc = self.lib.vl_moments(self.h, C.c_void_p(dn.data_ptr()), C.c_void_p(dV.data_ptr()),
                                 C.c_void_p(dP.data_ptr()), C.byref(tot) if total else None)
        _check("vl_moments", rc)
        return dn, dV.view(self.ncell, 3), dP.view(self.ncell, 6), tot.value

    def moments_static(self):
        """vl_moments_static: the moments with their scratch in the library's
        fixed device array (no allocation in the library); asynchronous.
        Returns device tensors (n, V, P, total mass)."""
        t = self.torch
        dn = t.empty(self.ncell, dtype=t.float64, device=self.device)
        dV = t.empty(self.ncell * 3, dtype=t.float64, device=self.device)
        dP = t.empty(self.ncell * 6, dtype=t.float64, device=self.device)
        dt_ = t.empty(1, dtype=t.float64, device=self.device)
        rc = self.lib.vl_moments_static(self.h, C.c_void_p(dn.data_ptr()), C.c_void_p(dV.data_ptr()),
                                        C.c_void_p(dP.data_ptr()), C.c_void_p(dt_.data_ptr()))
        _check("vl_moments_static", rc)
        return dn, dV.view(self.ncell, 3), dP.view(self.ncell, 6), dt_

    COUNTER_NAMES = ("ring_head", "ring_tail", "ring_limit", "ghost_slots", "ghost_list",
                     "list0", "list1", "items", "rows", "work", "err", "upd0", "upd1", "upd2",
                     "read0", "read1", "read2", "items0", "items1", "items2", "cur",
                     "cum_upd", "cum_read")

    def counters(self):
        out = np.zeros(32, np.uint64)
        _check("vl_counters", self.lib.vl_counters(self.h, _ptr(out), 23))
        return {k: int(v) for k, v in zip(self.COUNTER_NAMES, out)}

    KERNEL_CLASSES = ("ghost_fill", "planner", "shear", "prune", "moments", "shear1", "shear2", "shear3",
                      "accel")

    def profile_start(self, max_launches=4096):
        _check("vl_profile_start", self.lib.vl_profile_start(self.h, int(max_launches)))

    def profile_stop(self):
        ms = np.zeros(len(self.KERNEL_CLASSES))
        n = np.zeros(len(self.KERNEL_CLASSES), np.int64)
        _check("vl_profile_stop", self.lib.vl_profile_stop(self.h, _ptr(ms), _ptr(n)))
        return {k: (float(a), int(c)) for k, a, c in zip(self.KERNEL_CLASSES, ms, n)}

    def autotune(self, dt, mode=VL_COALESCED, steps_per_variant=2):
        """Time every shear-kernel variant on real steps and keep the fastest
        for each shear of the order.  Returns (the three chosen variants,
        ms per step of all shears with each variant)."""
        best = np.zeros(3, np.int32)
        ms = np.full(32, np.nan)
        _check("vl_autotune", self.lib.vl_autotune(self.h, float(dt), int(mode), int(steps_per_variant),
                                                   _ptr(best), _ptr(ms), 32))
        return tuple(int(v) for v in best), [float(v) for v in ms if not np.isnan(v)]

    def set_variant(self, v):
        """One variant for all three shears, or a sequence of three."""
        if np.ndim(v) == 0:
            _check("vl_set_variant", self.lib.vl_set_variant(self.h, int(v)))
        else:
            a = np.ascontiguousarray(v, np.int32)
            if a.shape != (3,):
                raise ValueError("three shear variants expected")
            _check("vl_set_shear_variants", self.lib.vl_set_shear_variants(self.h, _ptr(a)))

    def variants(self):
        """(variants of the three shears, number of compiled variants)"""
        a = np.zeros(3, np.int32)
        n = np.zeros(1, np.int32)
        _check("vl_get_shear_variants", self.lib.vl_get_shear_variants(self.h, _ptr(a), _ptr(n)))
        return tuple(int(v) for v in a), int(n[0])

    def sync(self):
        _check("vl_sync", self.lib.vl_sync(self.h))

    def local_blocks(self):
        v = C.c_int64(0)
        _check("vl_local_block_count", self.lib.vl_local_block_count(self.h, C.byref(v)))
        return int(v.value)

    def export(self):
        nb = self.local_blocks()
        off = np.zeros(self.ncell + 1, np.int64)
        ids = np.zeros(max(nb, 1), np.int32)
        f = np.zeros(max(nb, 1) * 64)
        _check("vl_export_state", self.lib.vl_export_state(self.h, _ptr(off), _ptr(ids), _ptr(f), nb))
        nb = int(off[-1])
        return off, ids[:nb], f[:nb * 64]

    def export_cells(self, cells):
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        cap = 1
        off = np.zeros(cells.size + 1, np.int64)
        # first pass sizes the output
        rc = self.lib.vl_export_cells(self.h, _ptr(cells), cells.size, _ptr(off), None, None, 0)
        if rc not in (VL_OK, VL_ERR_ARG):
            _check("vl_export_cells", rc)
        cap = max(int(off[-1]), 1)
        ids = np.zeros(cap, np.int32)
        f = np.zeros(cap * 64)
        _check("vl_export_cells", self.lib.vl_export_cells(self.h, _ptr(cells), cells.size, _ptr(off),
                                                           _ptr(ids), _ptr(f), cap))
        nb = int(off[-1])
        return off, ids[:nb], f[:nb * 64]

    def set_courant_override(self, table):
        if table is None:
            _check("vl_set_courant_override", self.lib.vl_set_courant_override(self.h, None, 0))
            return
        t = np.ascontiguousarray(table, dtype=np.float64)
        _check("vl_set_courant_override",
               self.lib.vl_set_courant_override(self.h, _ptr(t), int(t.shape[1])))

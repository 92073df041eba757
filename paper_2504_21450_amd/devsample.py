"""Device-side sampling of the synthetic input states (libvlgen.so), for
partitions too large to sample on the host.

The definition is the host sampler's (workloads.sample_cells with a
component-table model): the same per-cell parameter table, block selection
and counter-based noise, evaluated by gen/vlgen.hip.  Values agree with the
host sampler to the last-place differences of exp; block lists are the same
unless a sampled value lies within those few ulps of the threshold.  The
state goes into the partition in pieces: block lists at creation, values
through vl_load_values from a device staging buffer.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import binding as B
from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
GEN_PATH = os.path.join(HERE, "libvlgen.so")
_gen = None


def load_gen():
    global _gen
    if _gen is not None:
        return _gen
    if not os.path.exists(GEN_PATH):
        raise RuntimeError("libvlgen.so not built: run `python -m paper_2504_21450_amd.build`")
    L = C.CDLL(GEN_PATH)
    vp, i32, i64, dbl, u64 = C.c_void_p, C.c_int32, C.c_longlong, C.c_double, C.c_ulonglong
    geom = [vp, vp, vp, dbl, i32, i32, dbl, dbl, u64, vp]
    L.vg_masks.restype = C.c_int
    L.vg_masks.argtypes = geom + [i64, i64, vp, vp, vp]
    L.vg_ids.restype = C.c_int
    L.vg_ids.argtypes = [vp, i32, vp, i64, i64, vp, vp]
    L.vg_values.restype = C.c_int
    L.vg_values.argtypes = geom + [vp, vp, i64, i64, i64, vp, vp]
    _gen = L
    return L


class _Geom:
    def __init__(self, w):
        self.nblk = np.asarray(w.nblk, dtype=np.int32)
        self.vmin = np.asarray(w.vmin, dtype=np.float64)
        self.dv = np.asarray(w.dv, dtype=np.float64)
        self.args = None

    def pack(self, w, ncomp, params):
        return [C.c_void_p(self.nblk.ctypes.data), C.c_void_p(self.vmin.ctypes.data),
                C.c_void_p(self.dv.ctypes.data), float(w.sparse_min), int(w.vbuffer), int(ncomp),
                W.K_B / W.M_P, (2.0 * np.pi) ** 1.5, int(w.seed), C.c_void_p(params.data_ptr())]


def _chk(name, rc):
    if rc != 0:
        raise RuntimeError("%s failed (%d)" % (name, rc))


def sample_lists(w, device="cuda:0"):
    """Block lists of every cell of workload w (w.fields["params"]) sampled on
    the device.  Returns host (offsets, ids) and the device tensors the value
    pass needs (params, offsets, ids)."""
    import torch

    L = load_gen()
    P = np.ascontiguousarray(w.fields["params"], dtype=np.float64)
    ncell, ncomp = P.shape[0], P.shape[1]
    assert ncell == w.ncell and P.shape[2] == W.NPAR
    NB = int(np.prod(w.nblk))
    Wd = (NB + 31) // 32
    stream = C.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    params = torch.from_numpy(P.reshape(-1)).to(device)
    masks = torch.empty(ncell * Wd, dtype=torch.int32, device=device)
    counts = torch.empty(ncell, dtype=torch.int32, device=device)
    g = _Geom(w)
    _chk("vg_masks", L.vg_masks(*g.pack(w, ncomp, params), 0, ncell, C.c_void_p(masks.data_ptr()),
                                C.c_void_p(counts.data_ptr()), stream))
    cnt = counts.cpu().numpy().astype(np.int64)
    offsets = np.zeros(ncell + 1, dtype=np.int64)
    np.cumsum(cnt, out=offsets[1:])
    off_d = torch.from_numpy(offsets).to(device)
    ids_d = torch.empty(max(int(offsets[-1]), 1), dtype=torch.int32, device=device)
    _chk("vg_ids", L.vg_ids(C.c_void_p(masks.data_ptr()), Wd, C.c_void_p(off_d.data_ptr()), 0, ncell,
                            C.c_void_p(ids_d.data_ptr()), stream))
    del masks
    ids = ids_d[:int(offsets[-1])].cpu().numpy()
    return offsets, ids, (params, off_d, ids_d, ncomp)


def sample_partition(w, storage=None, slack=2.5, chunk_blocks=1 << 22, device="cuda:0", **kw):
    """A Partition holding workload w's initial state, sampled on the device.
    Sets w.offsets and w.ids (host) as a side effect; w.f stays None."""
    import torch

    L = load_gen()
    offsets, ids, (params, off_d, ids_d, ncomp) = sample_lists(w, device)
    w.offsets, w.ids = offsets, ids
    p = B.Partition(w.n, w.nblk, w.dx, w.vmin, w.dv, offsets, ids, None,
                    storage=w.storage if storage is None else storage, order=w.order,
                    sparse_min=w.sparse_min, vbuffer=w.vbuffer, device=device, slack=slack, **kw)
    NB = int(np.prod(w.nblk))
    chunk_blocks = max(int(chunk_blocks), NB)
    staging = torch.empty(chunk_blocks * 64, dtype=torch.float64, device=device)
    stream = C.c_void_p(p.stream.cuda_stream)
    g = _Geom(w)
    c = 0
    while c < w.ncell:
        c1 = int(np.searchsorted(offsets, offsets[c] + chunk_blocks, side="right")) - 1
        c1 = min(max(c1, c + 1), w.ncell)
        nb = int(offsets[c1] - offsets[c])
        if nb > 0:
            _chk("vg_values", L.vg_values(*g.pack(w, ncomp, params), C.c_void_p(off_d.data_ptr()),
                                          C.c_void_p(ids_d.data_ptr()), c, c1, int(offsets[c]),
                                          C.c_void_p(staging.data_ptr()), stream))
            p.load_values(int(offsets[c]), nb, staging)
        c = c1
    torch.cuda.synchronize(device)
    del staging, params, off_d, ids_d
    return p

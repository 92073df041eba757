"""Ghost Translation active/source cell sets on a non-refined periodic cubic
domain (Section 3.1, the limiting of Section 3.2, the estimate of Section 3.3
and Fig. 4).

TEST INFRASTRUCTURE ONLY (part of the oracle).

Construction, in reverse sweep order d3, d2, d1 (the paper's Z -> X -> Y gives
d3 = Y):
  * d3-active  = local cells and their d3 face neighbours;
  * d3-sources = d3-active plus the 2-cell stencil along d3;
  * d2-active  = d3-sources and their d2 face neighbours; d2-sources likewise;
  * d1-active  = d2-sources and their d1 face neighbours; d1-sources likewise.
GTk keeps only the active cells within k layers of the local domain (GT3 keeps
all of them, GT1 a single layer); sources follow from the kept active cells.
Classical translation (Section 2.1) has the local cells as the active cells of
every direction and exchanges, per direction and side, 2 stencil layers plus 1
layer of remote contributions.

Everything here is brute force on a lattice mask, plus the closed forms those
masks obey.
"""
from __future__ import annotations

import numpy as np

STENCIL = 2


def _grow(mask, axis, r):
    out = mask.copy()
    for s in range(1, r + 1):
        out |= np.roll(mask, s, axis=axis)
        out |= np.roll(mask, -s, axis=axis)
    return out


def gt_sets(n, k, order=(2, 0, 1), margin=None):
    """Lattice masks of the GTk sets for a cubic local domain of edge n.

    Returns (local, active, sources) with active/sources dicts keyed by axis.
    `order` is the sweep order (axes 0=x, 1=y, 2=z); the paper uses Z, X, Y."""
    if margin is None:
        margin = 2 * (STENCIL + 1) + 2
    N = n + 2 * margin
    local = np.zeros((N, N, N), dtype=bool)
    sl = slice(margin, margin + n)
    local[sl, sl, sl] = True
    limit = np.zeros_like(local)
    lk = slice(margin - k, margin + n + k)
    limit[lk, lk, lk] = True
    active, sources = {}, {}
    prev = local
    for d in reversed(order):
        act = _grow(prev, d, 1) & limit
        src = _grow(act, d, STENCIL)
        active[d], sources[d] = act, src
        prev = src
    return local, active, sources


def ratios_lattice(n, k, order=(2, 0, 1)):
    """(active ratio, source ratio) of GTk against classical translation."""
    local, active, sources = gt_sets(n, k, order)
    act = sum(int(a.sum()) for a in active.values())
    union = np.zeros_like(local)
    for s in sources.values():
        union |= s
    classical_comm = 3 * 2 * (STENCIL + 1) * n * n
    return act / (3.0 * n ** 3), (int(union.sum()) - n ** 3) / classical_comm


def active_ratio_closed(n, k):
    """Closed form of the lattice active ratio (valid for 1 <= k <= 3)."""
    return (n * n * (n + 2) + n * (n + 2 * k) * (n + 2) + (n + 2 * k) ** 2 * (n + 2)) / (3.0 * n ** 3)


def source_union_closed(n, k):
    """Closed form of |union of sources| for k = 1, 2, 3."""
    if k == 3:
        return (n + 6.0) ** 3
    if k == 1:
        return (n + 2.0) ** 3 + 4 * (n + 2.0) ** 2 + 4 * n * (n + 2.0) + 4 * n * n
    raise ValueError("closed form given for k = 1 and k = 3 only")


def source_ratio_closed(n, k):
    return (source_union_closed(n, k) - n ** 3) / (3 * 2 * (STENCIL + 1) * n * n)


def pull_update_boxes(n, order=(0, 1, 2), k=3):
    """Update boxes of the flux (pull) form, derived from the GTk lattice sets:
    in flux form a cell is recomputed by the shear along d exactly when it is
    d-active and not merely a face neighbour written to by the push form, i.e.
    the d-active set shrunk by one layer along d.  Returned as (lo, hi) per
    sweep, in coordinates relative to the local box origin."""
    local, active, _ = gt_sets(n, k, order)
    margin = (local.shape[0] - n) // 2
    out = []
    for d in order:
        a = active[d]
        shrunk = a & np.roll(a, 1, axis=d) & np.roll(a, -1, axis=d)
        idx = np.argwhere(shrunk)
        lo = idx.min(axis=0) - margin
        hi = idx.max(axis=0) + 1 - margin
        # the set must be exactly that box
        box = np.zeros_like(shrunk)
        box[tuple(slice(margin + l, margin + h) for l, h in zip(lo, hi))] = True
        assert np.array_equal(box, shrunk)
        out.append((tuple(int(v) for v in lo), tuple(int(v) for v in hi)))
    return out

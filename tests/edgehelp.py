"""Padded states for partitions at a simulation edge along x: local cells of
the box plus boundary cells beyond its x faces, taken from two boundary
states of the same box (the cell at padded position g of a boundary layer is
the boundary state's cell at g - dir * n, wrapped in y and z)."""
import numpy as np

H = 3


def padded_with_boundaries(n, local, lo_state, hi_state, nblk):
    """CSR (offsets, ids, f) of the padded box (n + 6 per axis, x fastest):
    local cells from `local`, cells beyond the low / high x face from
    `lo_state` / `hi_state`, the other ghost cells periodic images of the local
    cells (the oracle's ghost update refreshes those)."""
    P = tuple(v + 2 * H for v in n)
    rows_id, rows_f, counts = [], [], []

    def cell(state, x, y, z):
        off, ids, f = state
        q = x + n[0] * (y + n[1] * z)
        a, b = off[q], off[q + 1]
        return ids[a:b], f[a * 64:b * 64]

    for gz in range(P[2]):
        for gy in range(P[1]):
            for gx in range(P[0]):
                y, z = (gy - H) % n[1], (gz - H) % n[2]
                if gx < H:
                    i, f = cell(lo_state, gx - H + n[0], y, z)
                elif gx >= H + n[0]:
                    i, f = cell(hi_state, gx - H - n[0], y, z)
                else:
                    i, f = cell(local, gx - H, y, z)
                rows_id.append(i)
                rows_f.append(f)
                counts.append(len(i))
    off = np.zeros(len(counts) + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return off, np.concatenate(rows_id).astype(np.int32), np.concatenate(rows_f)

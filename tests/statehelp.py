"""Test-side helpers for CSR phase-space states (no part of the method)."""
import numpy as np

from paper_2504_21450_amd import workloads as W


def random_state(n, nblk, seed, density=1.0, zero_frac=0.0, scale=1e-9):
    """Random nonnegative state: each cell holds each block with probability
    `density` (sorted ids); values uniform in [0, scale) with a fraction
    `zero_frac` of exact zeros."""
    rng = np.random.default_rng(seed)
    NB = int(np.prod(nblk))
    nc = int(np.prod(n))
    ids_l, cnt = [], []
    for _ in range(nc):
        if density >= 1.0:
            ids = np.arange(NB, dtype=np.int32)
        else:
            ids = np.nonzero(rng.uniform(size=NB) < density)[0].astype(np.int32)
        ids_l.append(ids)
        cnt.append(ids.size)
    offsets = np.zeros(nc + 1, np.int64)
    np.cumsum(cnt, out=offsets[1:])
    ids = np.concatenate(ids_l) if ids_l else np.zeros(0, np.int32)
    f = rng.uniform(0.0, scale, ids.size * 64)
    if zero_frac > 0:
        f[rng.uniform(size=f.size) < zero_frac] = 0.0
    return offsets, ids, f


def to_dense(offsets, ids, f, NB):
    """(ncell, NB, 64) dense array, absent blocks = 0."""
    nc = offsets.size - 1
    out = np.zeros((nc, NB, 64))
    f2 = f.reshape(-1, 64)
    for c in range(nc):
        b0, b1 = offsets[c], offsets[c + 1]
        out[c, ids[b0:b1]] = f2[b0:b1]
    return out


def dense_to_csr(dense):
    nc, NB, _ = dense.shape
    offsets = np.zeros(nc + 1, np.int64)
    offsets[1:] = np.cumsum(np.full(nc, NB))
    ids = np.tile(np.arange(NB, dtype=np.int32), nc)
    return offsets, ids, dense.reshape(-1).copy()


def lists_of(offsets, ids):
    return [tuple(ids[offsets[c]:offsets[c + 1]]) for c in range(offsets.size - 1)]


def rel_maxnorm(a, ref):
    m = np.max(np.abs(ref))
    return np.max(np.abs(a - ref)) / m if m > 0 else np.max(np.abs(a))


def roll_cells(dense, n, shift):
    """Periodic spatial shift of a (ncell, ...) x-fastest array by shift[d]."""
    g = dense.reshape(n[2], n[1], n[0], *dense.shape[1:])
    g = np.roll(g, shift[0], axis=2)
    g = np.roll(g, shift[1], axis=1)
    g = np.roll(g, shift[2], axis=0)
    return g.reshape(dense.shape)


def block_perm(nblk, perm):
    """Map of block ids and lanes under a permutation of the velocity axes:
    new axis a = old axis perm[a]."""
    NB = int(np.prod(nblk))
    b = np.arange(NB)
    bc = np.stack([b % nblk[0], (b // nblk[0]) % nblk[1], b // (nblk[0] * nblk[1])], axis=1)
    nb2 = [nblk[perm[a]] for a in range(3)]
    nbc = bc[:, list(perm)]
    newb = nbc[:, 0] + nb2[0] * (nbc[:, 1] + nb2[1] * nbc[:, 2])
    l = np.arange(64)
    lc = np.stack([l & 3, (l >> 2) & 3, l >> 4], axis=1)
    nlc = lc[:, list(perm)]
    newl = nlc[:, 0] + 4 * nlc[:, 1] + 16 * nlc[:, 2]
    return newb, newl, tuple(nb2)


__all__ = ["W", "random_state", "to_dense", "dense_to_csr", "lists_of", "rel_maxnorm",
           "roll_cells", "block_perm"]

"""Pins of the oracle's velocity moments and of the Ghost Translation set
construction against the figures printed in the paper."""
import math
import os

import numpy as np
import pytest

from oracle import OraclePartition, gt_sets
from statehelp import dense_to_csr

M_P = 1.67262192e-27
K_B = 1.380649e-23
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_ratios.txt")


def load_golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split()[:2]
        out[k] = float(v)
    return out


def _maxwellian_cell(nblk, vmin, dv, n, V, T):
    NB = int(np.prod(nblk))
    b = np.arange(NB)
    bc = np.stack([b % nblk[0], (b // nblk[0]) % nblk[1], b // (nblk[0] * nblk[1])], axis=1)
    l = np.arange(64)
    lc = np.stack([l & 3, (l >> 2) & 3, l >> 4], axis=1)
    j = 4 * bc[:, None, :] + lc[None, :, :]
    v = np.asarray(vmin) + (j + 0.5) * np.asarray(dv)
    s2 = K_B * T / M_P
    u2 = np.sum((v - np.asarray(V)) ** 2, axis=-1)
    return n * (2 * np.pi * s2) ** -1.5 * np.exp(-0.5 * u2 / s2)


def test_moments_of_a_resolved_maxwellian_match_the_closed_form():
    """Midpoint sums of a well-resolved Gaussian converge faster than any
    power of dv, so n, V and P = n k T I must be recovered to ~1e-10."""
    nblk = (16, 16, 16)
    dv = (12e3,) * 3
    vmin = (-384e3,) * 3
    cells = [(1.3e6, (37e3, -21e3, 8e3), 1.0e5), (2.9e6, (-15e3, 44e3, -30e3), 0.7e5)]
    dense = np.stack([_maxwellian_cell(nblk, vmin, dv, *c) for c in cells])
    p = OraclePartition((2, 1, 1), nblk, (1e5,) * 3, vmin, dv)
    p.load_local(*dense_to_csr(dense))
    dens, V, P, tot = p.moments()
    for q, (n, Vw, T) in enumerate(cells):
        assert abs(dens[q] / n - 1) < 1e-10
        assert np.max(np.abs(V[q] - Vw)) < 1e-10 * 1e5
        p0 = n * K_B * T
        assert np.max(np.abs(P[q, :3] / p0 - 1)) < 1e-9
        assert np.max(np.abs(P[q, 3:])) < 1e-9 * p0
    assert abs(tot - (dens[0] + dens[1]) * 1e15) <= 1e-15 * tot


def test_moments_of_a_single_velocity_cell():
    """All content in one velocity cell: n = f dv^3, V = that cell's centre
    velocity, P = 0."""
    nblk = (3, 2, 2)
    NB = 12
    dv = (10.0, 20.0, 30.0)
    vmin = (-60.0, -80.0, -120.0)
    dense = np.zeros((1, NB, 64))
    b, lane, f = 7, 37, 2.5
    dense[0, b, lane] = f
    p = OraclePartition((1, 1, 1), nblk, (1.0, 1.0, 1.0), vmin, dv)
    p.load_local(*dense_to_csr(dense))
    dens, V, P, _ = p.moments()
    bc = (b % 3, (b // 3) % 2, b // 6)
    lc = (lane & 3, (lane >> 2) & 3, lane >> 4)
    want = [vmin[d] + (4 * bc[d] + lc[d] + 0.5) * dv[d] for d in range(3)]
    assert dens[0] == pytest.approx(f * 6000.0, rel=1e-15)
    assert np.allclose(V[0], want, rtol=1e-15, atol=0)
    assert np.all(np.abs(P[0]) == 0.0)


def test_printed_ghost_translation_ratios():
    """Section 4.2 prints the ratios of ideal cubic periodic domains holding a
    mean of 1223 cells: the closed forms of the lattice construction give them
    to the printed two decimals."""
    g = load_golden()
    n = g["cells_per_task"] ** (1.0 / 3.0)
    assert round(gt_sets.active_ratio_closed(n, 1), 2) == g["active_ratio_gt1"]
    assert round(gt_sets.active_ratio_closed(n, 3), 2) == g["active_ratio_gt3"]
    assert round(gt_sets.source_ratio_closed(n, 1), 2) == g["source_ratio_gt1"]
    assert round(gt_sets.source_ratio_closed(n, 3), 2) == g["source_ratio_gt3"]


def test_printed_overhead_at_edge_32():
    """Fig. 4: for every variant the overhead at edge length 32 is at most
    27 % (rounded)."""
    g = load_golden()
    n = int(g["edge_length"])
    for k in (1, 2, 3):
        a = gt_sets.active_ratio_closed(n, k)
        assert round(100 * (a - 1)) <= g["max_overhead_percent"]
    assert round(100 * (gt_sets.active_ratio_closed(n, 3) - 1)) == g["max_overhead_percent"]
    for k in (1, 3):
        assert round(100 * (gt_sets.source_ratio_closed(n, k) - 1)) <= g["max_overhead_percent"]


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("n", [4, 6, 9])
def test_closed_forms_match_lattice_construction(n, k):
    a, s = gt_sets.ratios_lattice(n, k)
    assert a == pytest.approx(gt_sets.active_ratio_closed(n, k), rel=1e-14)
    if k != 2:
        assert s == pytest.approx(gt_sets.source_ratio_closed(n, k), rel=1e-14)


def test_gt3_sources_are_the_padded_box():
    """The union of GT3 sources is the local box padded by 3 layers, the
    ghost domain the partition allocates."""
    n = 5
    local, active, sources = gt_sets.gt_sets(n, 3)
    u = np.zeros_like(local)
    for s in sources.values():
        u |= s
    m = (local.shape[0] - n) // 2
    box = np.zeros_like(local)
    sl = slice(m - 3, m + n + 3)
    box[sl, sl, sl] = True
    assert np.array_equal(u, box)

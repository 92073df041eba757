"""Uneven batched cells (cold cells of ~80 blocks beside hot mixture cells of
~4,300) on the GPU: the device-side sampler against the host sampler, and
the translation step against the FP64 oracle on sampled sub-boxes (the
oracle's input always comes from the host sampler)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import OraclePartition
from paper_2504_21450_amd import binding as B
from paper_2504_21450_amd import devsample
from paper_2504_21450_amd import workloads as W
from gpuhelp import need_gpu, print_case
from statehelp import to_dense

pytestmark = pytest.mark.gpu
SUB = (4, 4, 4)
# one BF16 step: the initial rounding (2^-9 of a value) and, per shear, the
# rounding of the cell plus the residual carried in from its pencil
# neighbour (2^-9 each); next to hot cells the neighbour's value is the
# local maximum, so the bound is 3 * 2^-8 + 2^-9 of the maximum
TOL_BF16_STEP = 3 * 2.0 ** -8 + 2.0 ** -9


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def subbox_local(n, lo):
    z, y, x = np.meshgrid(*[(np.arange(lo[d], lo[d] + SUB[d]) % n[d]) for d in (2, 1, 0)], indexing="ij")
    return (x + n[0] * (y + n[1] * z)).reshape(-1)


def oracle_subbox(w, lo, steps=1):
    """The oracle's steps on the sub-box at lo with its true ghost domain,
    sampled on the host (first step only: later steps would need the ghost
    domain's own evolution)."""
    assert steps == 1
    cells = W.subbox_cells(w.n, lo, SUB, 3)
    off, ids, f = W.sample_cells(W.table_model(w.fields["params"]), w.nblk, w.vmin, w.dv,
                                 w.sparse_min, w.vbuffer, w.seed, cells, threads=16, batch=4)
    o = OraclePartition(SUB, w.nblk, w.dx, w.vmin, w.dv, w.order, w.sparse_min, w.vbuffer)
    o.load_padded(off, ids, f)
    oracle.lib().vlo_mark_ghosts_valid(o._h)
    o.step(w.dt)
    return o.export_local()


def compare(got, want, NB, tol, exact_lists):
    if exact_lists:
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), "lists differ"
    a, b = to_dense(*got, NB), to_dense(*want, NB)
    err = np.max(np.abs(a - b)) / np.max(np.abs(b))
    assert err <= tol, err
    return err


@pytest.fixture(scope="module")
def small():
    return W.blob_mixture(n=(16, 16, 8), hot_fraction=0.4, sample=False, storage=B.VL_F64)


def test_device_sampler_matches_host_sampler(small):
    w = small
    print_case("device sampler vs host sampler, 16x16x8 mixture")
    p = devsample.sample_partition(w, storage=B.VL_F64)
    hot = w.fields["hot"]
    cells = np.concatenate([np.nonzero(hot)[0][::97][:12], np.nonzero(~hot)[0][::61][:12]])
    got = p.export_cells(cells)
    want = W.sample_cells(W.table_model(w.fields["params"]), w.nblk, w.vmin, w.dv, w.sparse_min,
                          w.vbuffer, w.seed, cells, threads=16, batch=2)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    rel = np.max(np.abs(got[2] - want[2]) / want[2])
    print("device/host sampler max relative difference %.2e" % rel)
    assert rel <= 1e-14
    counts = np.diff(w.offsets)
    assert counts.min() == 81 and counts.max() > 4000
    p.close()


def test_mixture_step_matches_oracle_on_subboxes(small):
    w = small
    print_case("mixture FP64 step vs oracle sub-boxes")
    p = devsample.sample_partition(w, storage=B.VL_F64)
    p.fill_ghosts()
    s = p.step(w.dt, B.VL_COALESCED, stats=True)
    assert abs(s["mass_after"] + s["pruned_mass"] - s["mass_before"]) <= 1e-12 * s["mass_before"]
    NB = int(np.prod(w.nblk))
    for lo in [(0, 0, 0), (9, 5, 3)]:
        err = compare(p.export_cells(subbox_local(w.n, lo)), oracle_subbox(w, lo), NB, 1e-12, True)
        print("sub-box %s error %.2e" % (lo, err))
    p.close()
    del p
    torch.cuda.empty_cache()


@pytest.mark.parametrize("storage,tol", [(B.VL_F32, 1e-5), (B.VL_BF16, TOL_BF16_STEP)])
def test_mixture_reduced_storage_against_oracle(small, storage, tol):
    w = small
    print_case("mixture storage %d step vs oracle sub-box" % storage)
    p = devsample.sample_partition(w, storage=storage)
    for _ in range(3):
        p.fill_ghosts()
        s = p.step(w.dt, B.VL_COALESCED, stats=True)
        resid = s["mass_before"] - (s["mass_after"] + s["pruned_mass"] + s["ledger_mass"])
        assert abs(resid) <= 1e-12 * s["mass_before"]
    # no negative density is stored, next to hot cells either (the carried
    # rounding residual of a hot cell can exceed a cold neighbour's value)
    _, _, f = p.export()
    assert f.size and np.min(f) >= 0.0
    p.close()
    p = devsample.sample_partition(w, storage=storage)
    p.fill_ghosts()
    p.step(w.dt, B.VL_COALESCED)
    lo = (9, 5, 3)
    err = compare(p.export_cells(subbox_local(w.n, lo)), oracle_subbox(w, lo), int(np.prod(w.nblk)), tol,
                  False)
    print("storage %d sub-box error %.2e" % (storage, err))
    p.close()


def test_mixture_ghost_translation_equals_classical(small):
    w = small
    print_case("mixture coalesced vs per-sweep")
    a = devsample.sample_partition(w, storage=B.VL_F32)
    b = devsample.sample_partition(w, storage=B.VL_F32)
    for _ in range(2):
        a.fill_ghosts()
        a.step(w.dt, B.VL_COALESCED)
        b.step(w.dt, B.VL_PER_SWEEP)
    assert all(np.array_equal(x, y) for x, y in zip(a.export(), b.export()))
    a.close()
    b.close()


@pytest.mark.parametrize("n,hot,storage,tol", [
    ((128, 128, 64), 0.0993, B.VL_BF16, TOL_BF16_STEP),   # HBM-filling partition, mean ~500 blocks
    ((96, 96, 24), 0.4, B.VL_F32, 1e-5),          # uneven cells at half the z extent
])
def test_fullsize_mixture_step(n, hot, storage, tol):
    """The large mixture partitions, sampled on the device: one coalesced
    step, its mass balance, and a sampled sub-box against the oracle."""
    w = W.blob_mixture(n=n, hot_fraction=hot, sample=False, storage=storage)
    print_case("full-size mixture %s hot %g storage %d" % (n, hot, storage))
    p = devsample.sample_partition(w, slack=1.25)
    nb = int(w.offsets[-1])
    print("blocks %d (mean %.1f per cell), workspace %.1f GB" % (nb, nb / w.ncell, p.ws_bytes / 1e9))
    p.fill_ghosts()
    s = p.step(w.dt, B.VL_COALESCED, stats=True)
    resid = s["mass_before"] - (s["mass_after"] + s["pruned_mass"] + s["ledger_mass"])
    assert abs(resid) <= 1e-12 * s["mass_before"]
    hotc = np.nonzero(w.fields["hot"])[0]
    q = int(hotc[len(hotc) // 2])
    lo = (q % n[0] - 2, (q // n[0]) % n[1] - 2, q // (n[0] * n[1]) - 2)   # around a hot cell
    lo = tuple(v % n[d] for d, v in enumerate(lo))
    err = compare(p.export_cells(subbox_local(n, lo)), oracle_subbox(w, lo), int(np.prod(w.nblk)), tol,
                  False)
    print("sub-box %s error %.2e" % (lo, err))
    p.close()
    del p
    torch.cuda.empty_cache()

"""Reduced-precision storage (FP32, BF16 with FP32 reconstruction; FP64
Courant number, flux integral and update, rounding residual carried along the
pencil into an FP64 ledger) against the FP64 oracle."""
import numpy as np
import pytest

from paper_2504_21450_amd import binding as B
from paper_2504_21450_amd import workloads as W
from gpuhelp import gpu_partition, need_gpu, print_case, run_gpu, run_oracle
from statehelp import to_dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.fixture(scope="module")
def sparse_small():
    return W.maxwellian_sparse(n=(6, 5, 4), threads=8)


def dense_err(a, b, NB):
    da, db = to_dense(*a, NB), to_dense(*b, NB)
    return np.max(np.abs(da - db)) / np.max(np.abs(db)), np.sum(np.abs(da - db)) / np.sum(np.abs(db))


@pytest.mark.parametrize("storage,steps,tol", [(B.VL_F32, 1, 1e-6), (B.VL_F32, 5, 1e-5),
                                               (B.VL_BF16, 1, 8e-3), (B.VL_BF16, 5, 2e-2)])
def test_reduced_storage_against_fp64_oracle(sparse_small, storage, steps, tol):
    w = sparse_small
    print_case("storage %d, %d steps" % (storage, steps))
    p = gpu_partition(w, storage=storage)
    st = run_gpu(p, w.dt, steps, stats=True)
    o, _ = run_oracle(w, steps)
    NB = int(np.prod(w.nblk))
    mx, l1 = dense_err(p.export(), o.export_local(), NB)
    print("max-norm %.3e L1 %.3e" % (mx, l1))
    assert mx <= tol
    for s in st:
        resid = s["mass_before"] - (s["mass_after"] + s["pruned_mass"] + s["ledger_mass"])
        assert abs(resid) <= 1e-12 * s["mass_before"], resid / s["mass_before"]


@pytest.mark.parametrize("storage", [B.VL_F32, B.VL_BF16])
def test_reduced_storage_ghost_translation_equals_classical(sparse_small, storage):
    w = sparse_small
    a = gpu_partition(w, storage=storage)
    b = gpu_partition(w, storage=storage)
    sa = run_gpu(a, w.dt, 2, B.VL_COALESCED, stats=True)
    sb = run_gpu(b, w.dt, 2, B.VL_PER_SWEEP, stats=True)
    assert all(np.array_equal(x, y) for x, y in zip(a.export(), b.export()))
    assert [s["ledger_mass"] for s in sa] == [s["ledger_mass"] for s in sb] or all(
        abs(x["ledger_mass"] - y["ledger_mass"]) <= 1e-15 * x["mass_before"] for x, y in zip(sa, sb))


def test_fp32_initial_rounding_and_export(sparse_small):
    w = sparse_small
    p = gpu_partition(w, storage=B.VL_F32)
    o, i, f = p.export()
    assert np.array_equal(o, w.offsets) and np.array_equal(i, w.ids)
    assert np.array_equal(f, w.f.astype(np.float32).astype(np.float64))


def test_bf16_initial_rounding_is_nearest_even(sparse_small):
    w = sparse_small
    p = gpu_partition(w, storage=B.VL_BF16)
    _, _, f = p.export()
    # reference: the two bfloat16 neighbours of each (positive) value x are
    # consecutive multiples of ulp = 2^(e-7) with 2^e <= x < 2^(e+1); take the
    # nearer, ties to the even multiple
    x = w.f[:20000]
    assert np.all(x > 0)
    e = np.floor(np.log2(x))
    e = np.where(x < 2.0 ** e, e - 1, np.where(x >= 2.0 ** (e + 1), e + 1, e))
    ulp = 2.0 ** (e - 7)
    k = np.floor(x / ulp)
    lo, hi = k * ulp, (k + 1) * ulp
    dlo, dhi = x - lo, hi - x
    want = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi, np.where(k % 2 == 0, lo, hi)))
    assert np.array_equal(f[:20000], want)


@pytest.mark.parametrize("storage", [B.VL_F32, B.VL_BF16])
def test_reduced_storage_runs_are_identical_to_the_last_bit(sparse_small, storage):
    """Two runs give the same state and the same mass, pruned-mass and ledger
    sums bit for bit: the ledger is summed per pencil over its items in block
    id order, then over the pencils in order, with no atomic additions."""
    w = sparse_small
    print_case("determinism, storage %d" % storage)
    a = gpu_partition(w, storage=storage)
    b = gpu_partition(w, storage=storage)
    sa = run_gpu(a, w.dt, 3, stats=True)
    sb = run_gpu(b, w.dt, 3, stats=True)
    assert all(np.array_equal(x, y) for x, y in zip(a.export(), b.export()))
    for x, y in zip(sa, sb):
        for k in ("mass_before", "mass_after", "pruned_mass", "ledger_mass"):
            assert x[k] == y[k], k
    assert any(s["ledger_mass"] != 0.0 for s in sa)
    assert np.min(a.export()[2]) >= 0.0

"""The uneven batched-cell workload (blob mixture of cold solar-wind and hot
magnetosheath-like cells): host-side generator checks, no GPU."""
import numpy as np

from paper_2504_21450_amd import workloads as W


def test_hot_fraction_and_component_table():
    w = W.blob_mixture(n=(12, 10, 8), hot_fraction=0.4, sample=False)
    P, hot = w.fields["params"], w.fields["hot"]
    assert hot.sum() == round(0.4 * w.ncell)
    assert P.shape == (w.ncell, W.NCOMP, W.NPAR)
    # cold: one Maxwellian at -750 km/s; hot: core + beam, 0.9 + 0.1 of n_h
    assert np.all(P[~hot, 1, 0] == 0.0) and np.all(P[~hot, 0, 1] == -750e3)
    assert np.allclose(P[hot, 0, 0] + P[hot, 1, 0], 1e6)
    assert np.allclose(np.linalg.norm(P[hot, 1, 1:4], axis=1), 800e3)
    # the hot cells are where the blob field is largest
    B = W.blob_field(np.random.default_rng(w.seed), w.n)
    assert B[hot].min() >= B[~hot].max()


def test_blob_field_is_periodic():
    """Shifting the blob centres by one box length leaves the field unchanged
    (minimum-image distances)."""
    n = (9, 7, 5)
    a = W.blob_field(np.random.default_rng(3), n)
    assert a.shape == (315,)
    # the field at cell (0, y, z) and at (n-1, y, z) both see the wrap:
    # recompute with the box rolled by one cell and compare rolled values
    rng = np.random.default_rng(3)
    c = rng.uniform(0.0, 1.0, size=(16, 3)) * np.asarray(n, dtype=np.float64)
    r = rng.uniform(3.0, 8.0, size=16)
    x, y, z = 0.5, 3.5, 2.5
    want = 0.0
    for k in range(16):
        d2 = 0.0
        for d, p in enumerate((x, y, z)):
            t = abs(p - c[k, d])
            t = min(t, n[d] - t)
            d2 += t * t
        want += np.exp(-d2 / (2 * r[k] ** 2))
    assert abs(a[0 + n[0] * (3 + n[1] * 2)] - want) <= 1e-12 * want


def test_block_counts_cold_and_hot_cells():
    """Face-neighbour buffer: a cold T = 1e5 K cell keeps 81 blocks, a hot
    mixture cell about 4,300 (the uneven range the batching has to cover)."""
    w = W.blob_mixture(n=(12, 10, 8), hot_fraction=0.4, sample=False)
    hot = w.fields["hot"]
    cells = np.concatenate([np.nonzero(hot)[0][:2], np.nonzero(~hot)[0][:2]])
    o, i, f = W.sample_cells(W.table_model(w.fields["params"]), w.nblk, w.vmin, w.dv, 1e-15, 6,
                             w.seed, cells, threads=2, batch=1)
    cnt = np.diff(o)
    assert np.all(cnt[2:] == 81)
    assert np.all((cnt[:2] > 4000) & (cnt[:2] < 4700))
    assert np.all(f > 0)


def test_table_model_equals_dict_model():
    """The component-table path samples exactly what the per-cell dict model
    of the smooth Maxwellian workload samples."""
    n = (6, 5, 4)
    w = W.maxwellian_sparse(n=n, threads=2)
    fl = w.fields
    P = np.zeros((w.ncell, 2, W.NPAR))
    P[:, 0, 0] = fl["n"]
    P[:, 0, 1:4] = fl["V"]
    P[:, 0, 4] = fl["T"]
    P[:, 0, 5] = fl["T"]
    P[:, 0, 6] = 1.0
    cells = np.arange(0, w.ncell, 7)
    o, i, f = W.sample_cells(W.table_model(P), w.nblk, w.vmin, w.dv, w.sparse_min, w.vbuffer, w.seed,
                             cells, threads=2)
    o2, i2, f2 = W.take_cells(w.offsets, w.ids, w.f, cells)
    assert np.array_equal(o, o2) and np.array_equal(i, i2) and np.array_equal(f, f2)

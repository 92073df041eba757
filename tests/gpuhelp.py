"""Shared helpers of the GPU tests (parity of the HIP path against the oracle)."""
import numpy as np
import pytest

import oracle
from oracle import OraclePartition
from paper_2504_21450_amd import binding as B


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gpu_partition(w, storage=None, order=None, **kw):
    return B.Partition.from_workload(w, storage=storage, order=order, **kw)


def run_gpu(p, dt, steps, mode=B.VL_COALESCED, stats=False):
    out = []
    for _ in range(steps):
        if mode == B.VL_COALESCED:
            p.fill_ghosts()
        out.append(p.step(dt, mode, stats=stats))
    return out


def run_oracle(w, steps, mode=oracle.COALESCED, order=None):
    o = OraclePartition.from_workload(w, order=order)
    st = []
    for _ in range(steps):
        if mode == oracle.COALESCED:
            o.fill_ghosts()
        st.append(o.step(w.dt, mode))
    return o, st


def compare_states(a, b, tol):
    """a, b: CSR (offsets, ids, f).  Lists must be identical; values within
    tol relative max-norm (max |a-b| / max |b|).  Returns the error."""
    oa, ia, fa = a
    ob, ib, fb = b
    assert np.array_equal(oa, ob), "block counts differ"
    assert np.array_equal(ia, ib), "block lists differ"
    m = np.max(np.abs(fb)) if fb.size else 0.0
    err = np.max(np.abs(fa - fb)) / m if m > 0 else float(np.max(np.abs(fa))) if fa.size else 0.0
    assert err <= tol, err
    return err


def print_case(msg):
    print("[case] " + msg, flush=True)

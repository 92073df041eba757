"""Extreme and degenerate inputs of the HIP path against the oracle: an empty
partition, boxes one and two cells wide, the longest pencil the kernels take
(250 local + 6 ghost cells = 256), and the largest velocity mesh (131072
blocks per cell) with blocks at the corners of the block-id space."""
import numpy as np
import pytest

from paper_2504_21450_amd import binding as B
from paper_2504_21450_amd import workloads as W
from gpuhelp import compare_states, gpu_partition, need_gpu, print_case, run_gpu, run_oracle
from statehelp import random_state

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def workload(name, n, nblk, st, order=(0, 1, 2), sparse_min=2.5e-10, vbuffer=6):
    """Unit velocity cells centred on zero; dx = 2 nblk + 1 keeps every
    Courant number below 1 at dt = 1."""
    vmin = tuple(-2.0 * b for b in nblk)
    dx = tuple(2.0 * b + 1.0 for b in nblk)
    return W.Workload(name, n, dx, nblk, vmin, (1.0, 1.0, 1.0), 1.0, 2, sparse_min, vbuffer,
                      B.VL_F64, order, *st)


def both_modes_match_oracle(w, steps=2, **kw):
    want = None
    for mode in (B.VL_COALESCED, B.VL_PER_SWEEP):
        p = gpu_partition(w, **kw)
        run_gpu(p, w.dt, steps, mode)
        got = p.export()
        if want is None:
            o, _ = run_oracle(w, steps)
            want = o.export_local()
        compare_states(got, want, TOL64)
    return want


def test_empty_partition():
    n, nblk = (4, 3, 5), (2, 2, 2)
    st = (np.zeros(int(np.prod(n)) + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    w = workload("empty", n, nblk, st)
    print_case("empty partition")
    p = gpu_partition(w)
    s = run_gpu(p, w.dt, 3, stats=True)
    assert all(x["blocks"] == 0 and x["mass_after"] == 0.0 for x in s)
    o, a, f = p.export()
    assert not o.any() and a.size == 0 and f.size == 0
    dn, dV, dP, tot = p.moments()
    assert tot == 0.0 and float(dn.abs().max()) == 0.0
    both_modes_match_oracle(w)


@pytest.mark.parametrize("n,order", [((1, 1, 1), (0, 1, 2)), ((1, 2, 3), (2, 0, 1)), ((2, 1, 2), (1, 2, 0))])
def test_boxes_one_and_two_cells_wide(n, order):
    """The periodic images of the ghost layers wrap around the box several
    times."""
    nblk = (2, 3, 2)
    st = random_state(n, nblk, 91, density=0.5, zero_frac=0.1)
    w = workload("tiny", n, nblk, st, order)
    print_case("box %s order %s" % (n, order))
    both_modes_match_oracle(w, 3)


@pytest.mark.parametrize("n,order", [((250, 2, 2), (0, 1, 2)), ((2, 3, 250), (2, 0, 1))])
def test_longest_pencils(n, order):
    """256-cell pencils: every word of the presence masks in use."""
    nblk = (3, 3, 3)
    st = random_state(n, nblk, 92, density=0.3, zero_frac=0.05)
    w = workload("long", n, nblk, st, order, vbuffer=0)  # no dilation: the pencils keep gaps
    print_case("longest pencils %s" % (n,))
    both_modes_match_oracle(w)


def test_largest_velocity_mesh():
    """131072 block ids (1024 x 8 x 16 blocks): blocks at the corners and
    edges of the id space, plus random ones, in a 3x3x3 box."""
    n, nblk = (3, 3, 3), (1024, 8, 16)
    NB = int(np.prod(nblk))
    rng = np.random.default_rng(93)
    corners = [0, NB - 1, nblk[0] - 1, NB - nblk[0], nblk[0] * nblk[1] - 1, nblk[0] * (nblk[1] - 1)]
    ids_l, cnt = [], []
    for c in range(int(np.prod(n))):
        ids = np.unique(np.concatenate([np.array(corners[c % 3::3]),
                                        rng.integers(0, NB, 12)])).astype(np.int32)
        ids_l.append(ids)
        cnt.append(ids.size)
    off = np.zeros(len(cnt) + 1, np.int64)
    np.cumsum(cnt, out=off[1:])
    ids = np.concatenate(ids_l)
    f = rng.uniform(0.0, 1e-9, ids.size * 64)
    w = workload("widest", n, nblk, (off, ids, f))
    print_case("largest velocity mesh")
    # dilation around isolated blocks grows the lists about ninefold in the
    # first step, and the ghost domain of a 3x3x3 box is 26 times the box
    both_modes_match_oracle(w, slack=16.0)

"""vl_moments_static, the moments entry point that allocates nothing (its
scratch sits in the library's fixed device array), called through the C ABI:
its outputs equal vl_moments' bit for bit on two calls in a row, the second
on a smaller partition (the array keeps the first call's contents), with
cells split over several wavefronts in the first."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2504_21450_amd import binding as B
from paper_2504_21450_amd import workloads as W
from gpuhelp import gpu_partition, need_gpu, print_case, run_gpu

pytestmark = pytest.mark.gpu


def static_moments(p):
    dn = torch.full((p.ncell,), -1.0, dtype=torch.float64, device="cuda:0")
    dV = torch.full((p.ncell * 3,), -1.0, dtype=torch.float64, device="cuda:0")
    dP = torch.full((p.ncell * 6,), -1.0, dtype=torch.float64, device="cuda:0")
    tot = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
    rc = p.lib.vl_moments_static(p.h, C.c_void_p(dn.data_ptr()), C.c_void_p(dV.data_ptr()),
                                 C.c_void_p(dP.data_ptr()), C.c_void_p(tot.data_ptr()))
    assert rc == B.VL_OK, B.status_string(rc)
    torch.cuda.synchronize()
    return dn.cpu().numpy(), dV.cpu().numpy(), dP.cpu().numpy(), float(tot.cpu().numpy()[0])


def test_static_scratch_moments_equal_the_workspace_moments():
    need_gpu()
    big = W.blob_mixture(n=(6, 6, 4), hot_fraction=0.4, threads=16, storage=B.VL_F32)
    small = W.maxwellian_sparse(n=(4, 3, 2), threads=8)
    assert np.diff(big.offsets).max() > 2048
    for w in (big, small):
        print_case("vl_moments_static vs vl_moments on %s" % w.name)
        p = gpu_partition(w)
        run_gpu(p, w.dt, 1)
        sn, sV, sP, stot = static_moments(p)
        dn, dV, dP, tot = p.moments()
        assert np.array_equal(sn, dn.cpu().numpy())
        assert np.array_equal(sV, dV.cpu().numpy().reshape(-1))
        assert np.array_equal(sP, dP.cpu().numpy().reshape(-1))
        assert stot == tot
        assert np.all(sn > 0)
        p.close()


def test_static_scratch_rejects_nothing_it_can_hold():
    """A null handle is refused; a valid partition gets VL_OK."""
    need_gpu()
    lib = B.load()
    assert lib.vl_moments_static(None, None, None, None, None) == B.VL_ERR_ARG

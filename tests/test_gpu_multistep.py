"""Whole-box, multi-step parity of the FP64 path with the oracle on the
sparse-Maxwellian recipe (one Maxwellian per cell from seeded smooth fields,
100^3 velocity cells in 4^3 blocks, pruning at 1e-15 with the face buffer)
on a 32 x 32 x 16 box: every value of every local cell after steps 1, 5, 10
and 20 of 20 coalesced steps (lists exact), and after every step the same
updated phase-space cells per shear, blocks and pruned mass as the oracle."""
import numpy as np
import pytest

from oracle import OraclePartition
from paper_2504_21450_amd import binding as B
from paper_2504_21450_amd import workloads as W
from gpuhelp import compare_states, gpu_partition, need_gpu, print_case

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.timeout(900)
def test_twenty_steps_of_a_32x32x16_box_match_the_oracle():
    w = W.maxwellian_sparse(n=(32, 32, 16), threads=16)
    print_case("32x32x16 sparse maxwellian, 20 coalesced FP64 steps, %d blocks" % w.nblocks)
    p = gpu_partition(w, slack=4.0)
    o = OraclePartition.from_workload(w)
    worst = 0.0
    for k in range(20):
        p.fill_ghosts()
        g = p.step(w.dt, B.VL_COALESCED, stats=True)
        o.fill_ghosts()
        r = o.step(w.dt)
        assert g["updated_ps"] == r["updates"], k
        assert g["blocks"] == r["blocks"], k
        assert abs(g["pruned_mass"] - r["pruned_mass"]) <= 1e-12 * r["mass_before"], k
        assert abs(g["mass_after"] + g["pruned_mass"] - g["mass_before"]) <= 1e-12 * g["mass_before"], k
        if k in (0, 4, 9, 19):
            err = compare_states(p.export(), o.export_local(), TOL64)
            worst = max(worst, err)
            print("step %2d: max-norm %.3e, %d blocks" % (k + 1, err, r["blocks"]), flush=True)
    print("worst relative max-norm over the sampled steps %.3e" % worst)

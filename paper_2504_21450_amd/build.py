"""Build libvlasov.so and libvlgen.so (HIP, gfx950) in-tree.

    python -m paper_2504_21450_amd.build

Every source under csrc/ is compiled with hipcc for gfx950 only, with packed
FP32 instructions disabled, and linked into paper_2504_21450_amd/libvlasov.so
(the translation library).  gen/vlgen.hip, the device-side sampler of the
synthetic input states, is built the same way (plus no multiply-add
contraction) into paper_2504_21450_amd/libvlgen.so.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libvlasov.so")
GEN_SRC = os.path.join(HERE, "gen", "vlgen.hip")
GEN_LIB = os.path.join(HERE, "libvlgen.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["api.hip", "k_store.hip", "k_plan.hip", "k_sweep.hip", "k_prune.hip", "k_accel.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _compile(src, extra=()):
    path = src if os.path.isabs(src) else os.path.join(CSRC, src)
    obj = os.path.join(BUILD, os.path.splitext(os.path.basename(src))[0] + ".o")
    cmd = [HIPCC] + FLAGS + list(extra) + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    return obj, warn


def _link(objs, out):
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + list(objs)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, out)


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    jobs = [(s, ()) for s in SOURCES] + [(GEN_SRC, ("-ffp-contract=off",))]
    with ThreadPoolExecutor(len(jobs)) as ex:
        res = list(ex.map(lambda j: _compile(*j), jobs))
    if verbose:
        for o, w in res:
            if w:
                print(w, file=sys.stderr)
    _link([o for o, _ in res[:-1]], LIB)
    _link([res[-1][0]], GEN_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

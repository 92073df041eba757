"""Host-side checks of libvlasov.so: it loads, exports every entry point the
header declares, the ctypes structures match the C layout, and argument
validation works without touching a GPU."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2504_21450_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vlasov.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vl_[a-z_]+)\s*\(", src)))


def test_library_loads_and_exports_every_declared_function():
    lib = B.load()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(B.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (vl_[a-z_]+)", out))
    assert set(names) <= exported


def test_struct_layout_matches_the_header():
    """Compile a probe against the header with gcc and compare offsets."""
    probe = r"""
#include <stdio.h>
#include <stddef.h>
#include "vlasov.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(vl_desc), offsetof(vl_desc, storage),
         offsetof(vl_desc, dx), offsetof(vl_desc, sparse_min), offsetof(vl_desc, block_capacity),
         offsetof(vl_desc, ghost_block_capacity), sizeof(vl_step_stats),
         offsetof(vl_step_stats, local_blocks), offsetof(vl_step_stats, items));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "p.c")
        exe = os.path.join(td, "p")
        open(c, "w").write(probe)
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), c, "-o", exe])
        vals = [int(v) for v in subprocess.check_output([exe]).split()]
    D, S = B.VlDesc, B.VlStepStats
    want = [C.sizeof(D), D.storage.offset, D.dx.offset, D.sparse_min.offset, D.block_capacity.offset,
            D.ghost_block_capacity.offset, C.sizeof(S), S.local_blocks.offset, S.items.offset]
    assert vals == want


def good_desc(**kw):
    a = dict(n=(4, 3, 5), nblk=(2, 2, 2), dx=(4.0, 5.0, 7.0), vmin=(-4.0, -4.0, -4.0),
             dv=(1.0, 1.0, 1.0), block_capacity=1000, ghost_block_capacity=1000)
    a.update(kw)
    return B.make_desc(**a)


def test_workspace_bytes_and_descriptor_validation():
    assert B.workspace_bytes(good_desc()) > 0
    bad = [dict(n=(0, 3, 5)), dict(n=(251, 3, 5)), dict(nblk=(0, 2, 2)), dict(order=(0, 0, 1)),
           dict(storage=3), dict(stencil=3), dict(gt_level=0), dict(gt_level=4), dict(vbuffer=7),
           dict(dx=(0.0, 1.0, 1.0)), dict(dv=(1.0, -1.0, 1.0)), dict(block_capacity=0),
           dict(nblk=(64, 64, 64)), dict(nblk=(1025, 1, 1))]
    for kw in bad:
        assert B.workspace_bytes(good_desc(**kw)) == 0, kw
    for k in (1, 2, 3):  # Ghost Translation levels
        assert B.workspace_bytes(good_desc(gt_level=k)) > 0
    # larger pools need more workspace
    assert B.workspace_bytes(good_desc(block_capacity=5000)) > B.workspace_bytes(good_desc())


def test_init_rejects_bad_arguments_without_a_gpu():
    lib = B.load()
    d = good_desc()
    h = C.c_void_p()
    off = np.zeros(61, np.int64)
    # no workspace
    assert lib.vl_init_partition(C.byref(d), None, 0, None, B._ptr(off), None, None, C.byref(h)) == B.VL_ERR_ARG
    # misaligned workspace pointer
    assert lib.vl_init_partition(C.byref(d), C.c_void_p(8), 1 << 40, None, B._ptr(off), None, None,
                                 C.byref(h)) == B.VL_ERR_ARG
    assert not h.value


def test_status_strings():
    for s in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert len(B.status_string(s)) >= 2
    assert "Courant" in B.status_string(B.VL_ERR_CFL)


def test_null_handles_are_rejected():
    lib = B.load()
    assert lib.vl_fill_ghosts(None) == B.VL_ERR_ARG
    assert lib.vl_translate_step(None, 1.0, 0, None) == B.VL_ERR_ARG
    assert lib.vl_sync(None) == B.VL_ERR_ARG
    v3 = np.zeros(3, np.int32)
    assert lib.vl_set_shear_variants(None, B._ptr(v3)) == B.VL_ERR_ARG
    assert lib.vl_get_shear_variants(None, B._ptr(v3), None) == B.VL_ERR_ARG
    assert lib.vl_set_variant(None, 0) == B.VL_ERR_ARG
    lib.vl_destroy(None)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library the binding raises instead of falling back."""
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "libvlasov.so"))
    with pytest.raises(RuntimeError):
        B.load()


def test_edges_field_takes_the_reserved_slot():
    """The simulation-edge mask sits where the header's descriptor has it and
    only six face bits are accepted."""
    assert B.VlDesc.edges.offset == B.VlDesc.vbuffer.offset + 4
    assert B.workspace_bytes(good_desc(edges=63)) > 0
    assert B.workspace_bytes(good_desc(edges=64)) == 0
    assert B.workspace_bytes(good_desc(edges=-1)) == 0

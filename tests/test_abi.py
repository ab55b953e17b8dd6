"""The C-ABI library loads, exports every function that include/tr_stream.h
declares, its config struct matches the binding's layout, and argument
validation answers without a device."""

import ctypes
import os
import subprocess
import tempfile

import pytest

import paper_2307_00719_amd as P
from paper_2307_00719_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = P.load()
    names = P.declared_functions()
    assert "tr_stream_init" in names and "tr_stream_update" in names
    assert "tr_reconstruct_error" in names
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = {l.split()[-1] for l in out.splitlines() if l.strip()}
    missing = [n for n in names if n not in syms]
    assert not missing, missing


def test_config_struct_layout_matches_header():
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "tr_stream.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(tr_config), offsetof(tr_config, dims),
         offsetof(tr_config, sketch_size), offsetof(tr_config, seed),
         offsetof(tr_config, max_slices), offsetof(tr_config, device),
         offsetof(tr_config, hip_stream));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True,
                                               check=True).stdout.split()]
    T = _lib.tr_config
    assert vals == [ctypes.sizeof(T), T.dims.offset, T.sketch_size.offset, T.seed.offset,
                    T.max_slices.offset, T.device.offset, T.hip_stream.offset]


def test_validation_without_device():
    lib = P.load()
    h = ctypes.c_void_p()
    assert lib.tr_stream_init(None, None, 1, 0, None, 0, ctypes.byref(h)) == 1   # TR_ERR_ARG
    dims = (ctypes.c_int64 * 2)(4, 5)
    ranks = (ctypes.c_int32 * 3)(2, 40, 2)
    cfg = _lib.tr_config(order=3, dims=dims, ranks=ranks)
    x = (ctypes.c_double * 4)()
    cores = (ctypes.c_void_p * 3)(ctypes.addressof(x), ctypes.addressof(x), ctypes.addressof(x))
    assert lib.tr_stream_init(ctypes.byref(cfg), x, 2, 0, cores, 0, ctypes.byref(h)) == 8
    cfg2 = _lib.tr_config(order=2, dims=dims, ranks=ranks)
    assert lib.tr_stream_init(ctypes.byref(cfg2), x, 2, 0, cores, 0, ctypes.byref(h)) == 1
    assert not h
    assert P.tr_workspace_bytes([8, 8, 8, 4], [16, 16, 16, 16], "f32") > 0
    assert P.tr_workspace_bytes([8, 8, 8, 4], [16, 17, 16, 16], "f32") == 0
    assert lib.tr_stream_update(None, None, 0, 1, 0) == 1
    assert lib.tr_stream_num_slices(None) == -1


def test_product_path_does_not_import_oracle():
    """The package and its sources never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_2307_00719_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


def test_checkpoint_entry_points_validate_without_device(tmp_path):
    """tr_stream_load rejects a missing, foreign or truncated file before any
    device work; save / set_samples reject null arguments."""
    lib = P.load()
    h = ctypes.c_void_p()
    assert lib.tr_stream_load(None, None, ctypes.byref(h)) == 1
    assert lib.tr_stream_load(os.fsencode(str(tmp_path / "missing.bin")), None,
                              ctypes.byref(h)) == 1
    junk = tmp_path / "junk.bin"
    junk.write_bytes(b"not a saved tensor-ring stream" * 10)
    assert lib.tr_stream_load(os.fsencode(str(junk)), None, ctypes.byref(h)) == 1
    empty = tmp_path / "empty.bin"
    empty.write_bytes(b"")
    assert lib.tr_stream_load(os.fsencode(str(empty)), None, ctypes.byref(h)) == 1
    assert not h
    assert lib.tr_stream_save(None, b"x") == 1
    assert lib.tr_stream_set_samples(None, None, None, 0) == 1
    assert lib.tr_stream_get_stats(None, None) == 1
    assert lib.tr_batch_als(None, None, 0, 0, None, 0, 0, 0.0, None, None, None) == 1

"""The C ABI library loads, exports every entry point of include/rlu.h, and
the Python binding's struct layouts match the header (checked against a
program compiled from the header with gcc).  No GPU needed."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1601_04280_amd as rlu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rlu.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rlu_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ["rlu_create", "rlu_destroy", "rlu_workspace_size", "rlu_sketch_params", "rlu_sketch",
                 "rlu_factor", "rlu_tall_lu", "rlu_serve_start", "rlu_submit", "rlu_poll",
                 "rlu_serve_stop", "rlu_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(rlu.library_path):
        pytest.fail("librlu.so is not built (run __graft_entry__.build())")
    out = subprocess.run(["nm", "-D", "--defined-only", rlu.library_path], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\b[TW] (rlu_\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    lib = rlu.load_library()
    for f in declared_functions():
        assert hasattr(lib, f)


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r"""
#include <stdio.h>
#include <stddef.h>
#include "rlu.h"
#define F(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void) {
  printf("rlu_matrix %zu\nrlu_params %zu\nrlu_info %zu\nrlu_factors %zu\n",
         sizeof(rlu_matrix), sizeof(rlu_params), sizeof(rlu_info), sizeof(rlu_factors));
  F(rlu_matrix, values); F(rlu_matrix, ld); F(rlu_matrix, nnz);
  F(rlu_params, seed); F(rlu_params, flags); F(rlu_params, k2); F(rlu_params, l2);
  F(rlu_factors, perm_r); F(rlu_factors, Y); F(rlu_factors, ysel); F(rlu_factors, info);
  F(rlu_info, bad_index); F(rlu_info, zero_pivots_sel); F(rlu_info, min_gap_y); F(rlu_info, min_gap_b);
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    assert int(got["rlu_matrix"]) == ctypes.sizeof(rlu.Matrix)
    assert int(got["rlu_params"]) == ctypes.sizeof(rlu.Params)
    assert int(got["rlu_info"]) == ctypes.sizeof(rlu.Info)
    assert int(got["rlu_factors"]) == ctypes.sizeof(rlu.Factors)
    assert int(got["rlu_matrix.values"]) == rlu.Matrix.values.offset
    assert int(got["rlu_matrix.ld"]) == rlu.Matrix.ld.offset
    assert int(got["rlu_matrix.nnz"]) == rlu.Matrix.nnz.offset
    assert int(got["rlu_params.seed"]) == rlu.Params.seed.offset
    assert int(got["rlu_params.flags"]) == rlu.Params.flags.offset
    assert int(got["rlu_factors.perm_r"]) == rlu.Factors.perm_r.offset
    assert int(got["rlu_factors.Y"]) == rlu.Factors.Y.offset
    assert int(got["rlu_factors.ysel"]) == rlu.Factors.ysel.offset
    assert int(got["rlu_factors.info"]) == rlu.Factors.info.offset
    assert int(got["rlu_info.bad_index"]) == rlu.Info.bad_index.offset
    assert int(got["rlu_info.zero_pivots_sel"]) == rlu.Info.zero_pivots_sel.offset
    assert int(got["rlu_info.min_gap_y"]) == rlu.Info.min_gap_y.offset
    assert int(got["rlu_info.min_gap_b"]) == rlu.Info.min_gap_b.offset
    assert rlu.INFO_WORDS * 4 == int(got["rlu_info"])
    assert int(got["rlu_params.k2"]) == rlu.Params.k2.offset
    assert int(got["rlu_params.l2"]) == rlu.Params.l2.offset


def test_errors_are_reported_without_a_device():
    lib = rlu.load_library()
    p = rlu.Params(5, 4, 8, 0, 1, 0, 0)         # k > l
    st = lib.rlu_sketch_params(ctypes.byref(p), 16, None, None, None, None, None)
    assert st == rlu.RLU_ERR_INVALID_ARG
    assert b"k <= l" in lib.rlu_last_error()
    p = rlu.Params(2, 4, 12, 0, 1, 0, 0)        # s not a power of two
    assert lib.rlu_sketch_params(ctypes.byref(p), 16, None, None, None, None, None) == rlu.RLU_ERR_INVALID_ARG
    # second projection: l <= k2 <= l2, l2 a power of two, FP64 only
    for k2, l2, prec in [(2, 8, 0), (16, 8, 0), (6, 12, 0), (6, 16, 1), (4, 0, 0), (0, 16, 0)]:
        p = rlu.Params(2, 4, 8, prec, 1, 0, k2, l2, 0)
        assert lib.rlu_sketch_params(ctypes.byref(p), 16, None, None, None, None, None) == rlu.RLU_ERR_INVALID_ARG
    assert b"l2" in lib.rlu_last_error() or b"k2" in lib.rlu_last_error()
    p = rlu.Params(2, 4, 8, 0, 1, 0, 6, 16, 0)   # valid (without a device the call may still fail)
    assert lib.rlu_sketch_params(ctypes.byref(p), 16, None, None, None, None, None) != rlu.RLU_ERR_INVALID_ARG
    assert lib.rlu_create(0, None) == rlu.RLU_ERR_INVALID_ARG


def test_parameter_ranges_without_a_device():
    """s in [2, 65536] (powers of two), l <= 1024, l2 <= 8192, the flag bits:
    rejected or let through by the host-side validation alone."""
    lib = rlu.load_library()

    def status(k, l, s, flags=0, k2=0, l2=0):
        p = rlu.Params(k, l, s, 0, 1, flags, k2, l2, 0)
        return lib.rlu_sketch_params(ctypes.byref(p), 2048, None, None, None, None, None)

    bad = rlu.RLU_ERR_INVALID_ARG
    assert status(4, 8, 131072) == bad and b"65536" in lib.rlu_last_error()
    assert status(4, 8, 1) == bad
    assert status(4, 8, 65536) != bad
    assert status(4, 1024, 2048) != bad
    assert status(4, 1025, 2048) == bad and b"1024" in lib.rlu_last_error()
    assert status(4, 8, 16, k2=16, l2=16384) == bad and b"l2" in lib.rlu_last_error()
    assert status(4, 8, 16, k2=16, l2=8192) != bad
    assert status(4, 8, 16, flags=rlu.RLU_FLAG_DETERMINISTIC | rlu.RLU_FLAG_HADAMARD) != bad
    assert status(4, 8, 16, flags=rlu.RLU_FLAG_TRUNCATE) != bad
    assert status(4, 8, 16, flags=128) == bad and b"flag" in lib.rlu_last_error()

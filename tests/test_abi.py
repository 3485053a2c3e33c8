"""CPU checks of the C ABI: the built library loads and exports every function that
include/ibm.h declares, and the ctypes mirrors of the structs match the header's
layout (compiled with gcc). No device calls."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_2301_09349_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ibm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ibm_create_grid", "ibm_set_markers", "ibm_step", "ibm_wall_fluxes",
                     "ibm_workspace_bytes", "ibm_destroy", "ibm_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    # and the binding describes every one of them
    assert set(declared_functions()) <= set(_lib.SIGNATURES)


def test_struct_layouts_match_header():
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "ibm.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(ibm_grid_desc),
         offsetof(ibm_grid_desc, bc), offsetof(ibm_grid_desc, Re), offsetof(ibm_grid_desc, U_inf),
         offsetof(ibm_grid_desc, cg_maxit), offsetof(ibm_grid_desc, diffusion),
         sizeof(ibm_step_info), offsetof(ibm_step_info, mass),
         offsetof(ibm_step_info, diff_iters_total));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        vals = [int(v) for v in subprocess.check_output([exe]).split()]
    D, S = _lib.ibm_grid_desc, _lib.ibm_step_info
    assert vals == [ctypes.sizeof(D), D.bc.offset, D.Re.offset, D.U_inf.offset,
                    D.cg_maxit.offset, D.diffusion.offset, ctypes.sizeof(S), S.mass.offset,
                    S.diff_iters_total.offset]


def test_workspace_query_validates_descriptor():
    from paper_2301_09349_amd import inputs
    from paper_2301_09349_amd.solver import make_desc

    lib = _lib.load()
    d = make_desc(inputs.case("cfg1"))
    n1 = lib.ibm_workspace_bytes(ctypes.byref(d), 100, 0)
    assert n1 > 16384 * 8 * 20  # at least the state, predictor and CG vectors
    n2 = lib.ibm_workspace_bytes(ctypes.byref(d), 400, 0)
    assert n2 > n1
    bad = make_desc(inputs.case("cfg1"))
    bad.dim = 4
    assert lib.ibm_workspace_bytes(ctypes.byref(bad), 100, 0) == 0
    bad = make_desc(inputs.case("cfg1"))
    bad.bc[0][0] = 0  # periodic on one side only
    assert lib.ibm_workspace_bytes(ctypes.byref(bad), 100, 0) == 0
    bad = make_desc(inputs.case("cfg1"))
    bad.n[1] = 2
    assert lib.ibm_workspace_bytes(ctypes.byref(bad), 100, 0) == 0


def test_create_rejects_bad_arguments_without_touching_the_device():
    from paper_2301_09349_amd import inputs
    from paper_2301_09349_amd.solver import make_desc

    lib = _lib.load()
    d = make_desc(inputs.case("cfg1"))
    ctx = ctypes.c_void_p()
    # misaligned / NULL workspace: rejected before any HIP call
    assert lib.ibm_create_grid(ctypes.byref(d), None, 1 << 20, 0, None,
                               ctypes.byref(ctx)) == _lib.IBM_E_ARG
    assert lib.ibm_create_grid(ctypes.byref(d), ctypes.c_void_p(4096 + 8), 1 << 20, 0, None,
                               ctypes.byref(ctx)) == _lib.IBM_E_ARG
    assert not ctx.value


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/libibm_hip.so")
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()


def test_workspace_grows_by_one_tape_record_per_step():
    # a record: the state in the storage type ((dim + 2) N + sum NF words), then the
    # FP64 pressure (N), each part 256-byte aligned
    from paper_2301_09349_amd import inputs
    from paper_2301_09349_amd.solver import make_desc

    lib = _lib.load()
    c = inputs.case("cfg1")
    N = 128 * 128
    NF = 2 * 129 * 128
    up = lambda v: (v + 255) // 256 * 256
    for prec, w in (("fp64", 8), ("fp32", 4)):
        d = make_desc(c, prec)
        n = [lib.ibm_workspace_bytes(ctypes.byref(d), 100, t) for t in (0, 1, 2, 3)]
        rec = up(up((4 * N + NF) * w) + 8 * N)
        assert n[1] > n[0] + rec  # the first record also brings the adjoint's buffers
        assert n[2] - n[1] == rec and n[3] - n[2] == rec

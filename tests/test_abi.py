"""The C ABI: every entry point declared in include/dec.h is exported by the built library (CPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dec.h")
LIB = os.path.join(ROOT, "paper_2104_05999_amd", "libdec_hip.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(dec_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_path():
    names = declared()
    for want in ["dec_create", "dec_build_topology", "dec_hodge1", "dec_assemble", "dec_apply_bc", "dec_solve",
                 "dec_flux_effective_conductivity", "dec_spmv", "dec_get_fsai"]:
        assert want in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2104_05999_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    for name in declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(dec_\w+)", out))
    assert set(declared()) <= exported


def test_binding_covers_header(lib):
    from paper_2104_05999_amd import _lib
    assert set(_lib.SIGNATURES) == set(declared())


def test_host_only_calls_without_gpu(lib):
    from paper_2104_05999_amd import _lib
    L = _lib.load()
    assert L.dec_status_string(0) == b"ok"
    assert L.dec_status_string(-6) == b"invalid mesh topology"
    o = _lib.SolveOpts()
    assert L.dec_solve_opts_default(ctypes.byref(o)) == 0
    assert o.tol == 1e-10 and o.inner_tol == 1e-5 and o.chunk == 32 and o.max_iters == 100000
    assert L.dec_solve_opts_default(None) == -1
    assert L.dec_mesh_info(None, None, None, None, None, None, None) == -1

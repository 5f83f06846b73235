"""The C-ABI library loads and exports every entry point that include/bpmf.h
declares (no compute calls: these run without a GPU)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bpmf.h")
LIB = os.path.join(ROOT, "paper_1507_03703_amd", "libbpmf.so")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"BPMF_API\s+[\w\s\*]+?\b(bpmf_\w+)\s*\(",
                                 txt)))


def test_header_declares_the_five_core_calls():
    names = declared()
    for core in ("bpmf_grid_upload", "bpmf_ligand_setup", "bpmf_hmc_sweep",
                 "bpmf_exchange", "bpmf_energy_matrix"):
        assert core in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libbpmf.so not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    for name in declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (bpmf_\w+)", out))
    assert set(declared()) <= exported


def test_version_and_error_string(lib):
    lib.bpmf_version.restype = C.c_int
    assert lib.bpmf_version() == 100
    lib.bpmf_last_error.restype = C.c_char_p
    assert isinstance(lib.bpmf_last_error(), bytes)


def test_null_arguments_are_rejected_without_a_device(lib):
    # validation that precedes any device call
    lib.bpmf_create.restype = C.c_int
    assert lib.bpmf_create(None, 0, C.c_uint64(0), None, None, None,
                           None) == -1
    lib.bpmf_sync.restype = C.c_int
    assert lib.bpmf_sync(None) == -1
    lib.bpmf_destroy.restype = C.c_int
    assert lib.bpmf_destroy(None) == 0
    lib.bpmf_last_error.restype = C.c_char_p
    assert b"null context" in lib.bpmf_last_error()


def test_binding_lists_the_header(lib):
    import paper_1507_03703_amd as pkg
    assert pkg.EXPORTED == declared()
    L = pkg.library()
    for name in pkg.EXPORTED:
        assert getattr(L, name) is not None

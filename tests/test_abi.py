"""The C ABI: the built library loads and exports every declared function."""

import ctypes
import os
import re

from paper_1508_02512_amd import qmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "qmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qmc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("qmc_plan_sectors", "qmc_integrate", "qmc_submit", "qmc_create",
                 "qmc_bind", "qmc_run", "qmc_fetch"):
        assert want in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(qmc.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    # the binding knows every function too
    assert set(declared_functions()) <= set(qmc._SIGS)


def test_binding_structs_match_header_sizes():
    # sizes of the ABI structs on x86-64 (natural alignment)
    assert ctypes.sizeof(qmc.qmc_poly) == 24
    assert ctypes.sizeof(qmc.qmc_sector) == 8 + 16 + 48 + 32 + 16
    assert ctypes.sizeof(qmc.qmc_lattice) == 16
    assert ctypes.sizeof(qmc.qmc_coeff) == 32
    assert ctypes.sizeof(qmc.qmc_result) == 24 + 16 + 8 + 16 + 16

"""The C ABI: the built library loads and exports every declared function."""

import ctypes
import os
import re
import subprocess

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


STRUCTS = ("qmc_poly", "qmc_sector", "qmc_problem", "qmc_plan_opts", "qmc_lattice",
           "qmc_coeff", "qmc_plan_info", "qmc_result", "qmc_tune_choice", "qmc_class_stat",
           "qmc_request", "qmc_sector_info")


def test_binding_structs_match_header_layout(tmp_path):
    """Every ctypes struct has the size and field offsets that a C compiler
    gives the header's struct of the same name."""
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "qmc.h"',
             "int main(void) {"]
    for name in STRUCTS:
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in getattr(qmc, name)._fields_:
            # a trailing underscore marks a C field named like a Python keyword
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f.rstrip("_")}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.splitlines())
    for name in STRUCTS:
        T = getattr(qmc, name)
        assert int(got[name]) == ctypes.sizeof(T), name
        for f, _ in T._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(T, f).offset, f"{name}.{f}"


def test_limits_match_binding():
    text = open(os.path.join(ROOT, "include", "qmc.h")).read()
    for name in ("QMC_MAX_DIM", "QMC_MAX_ORDERS", "QMC_MAX_FACTORS", "QMC_MAX_POLES",
                 "QMC_POLES_SUBTRACT", "QMC_POLES_IBP"):
        m = re.search(rf"#define {name} (\d+)", text)
        assert m and int(m.group(1)) == getattr(qmc, name), name


def test_noalloc_scratch_size_matches_binding():
    text = open(os.path.join(ROOT, "include", "qmc.h")).read()
    m = re.search(r"#define QMC_NOALLOC_SCRATCH_BYTES \((\d+)u \* (\d+)u \* (\d+)u\)", text)
    assert m, "QMC_NOALLOC_SCRATCH_BYTES not found"
    size = int(m.group(1)) * int(m.group(2)) * int(m.group(3))
    assert size == qmc.QMC_NOALLOC_SCRATCH_BYTES

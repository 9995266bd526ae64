"""CPU-side checks of the C ABI: the library is built for gfx950, loads, and
exports every function that include/*.h declares (no compute calls)."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2405_05155_amd", "libsph.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?\w+\s*\**\s*(sph_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for required in ("sph_build_cells", "sph_neighbors", "sph_kernel_sum", "sph_correction_B",
                     "sph_euler_rhs", "sph_tlsph_rhs", "sph_relax_step"):
        assert required in names, required


@pytest.fixture(scope="module")
def built_lib():
    if not os.path.exists(LIB):
        from paper_2405_05155_amd import build
        build.build()
    return LIB


def test_library_exports_every_declared_symbol(built_lib):
    out = subprocess.run(["nm", "-D", "--defined-only", built_lib], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(built_lib)
    for n in declared_functions():
        assert hasattr(lib, n)


def test_library_contains_gfx950_code_object(built_lib):
    # the offload bundle embedded in the shared object names its target
    data = open(built_lib, "rb").read()
    assert b"gfx950" in data
    assert b"gfx942" not in data and b"sm_" not in data[:0]


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_2405_05155_amd.sph as S
    monkeypatch.setattr(S, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(S, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        S.lib()


def _c_struct_layouts(tmp_path, structs):
    """sizeof and offsetof of each field, as the C compiler lays out the
    header's structs (gcc, host ABI)."""
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sph.h"', "int main(void) {"]
    for name, fields in structs.items():
        lines.append(f'    printf("{name} size %zu\\n", sizeof({name}));')
        for f in fields:
            lines.append(f'    printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    return {tuple(line.split()[:2]): int(line.split()[2]) for line in out.splitlines()}


def test_binding_structs_match_header(tmp_path):
    """Every parameter struct of the binding has the header's size and field
    offsets (a field added on one side only would shift the others)."""
    from paper_2405_05155_amd import sph as S
    classes = {n: getattr(S, n) for n in dir(S) if n.startswith("sph_") and isinstance(getattr(S, n), type)
               and issubclass(getattr(S, n), ctypes.Structure)}
    assert {"sph_domain", "sph_euler_params", "sph_hllc_params", "sph_tlsph_params", "sph_relax_params",
            "sph_adamw_params"} <= set(classes)
    header = open(os.path.join(ROOT, "include", "sph.h")).read()
    for n in classes:
        assert re.search(r"\}\s*" + n + r"\s*;", header), n
    structs = {n: [f[0] for f in c._fields_] for n, c in classes.items()}
    lay = _c_struct_layouts(tmp_path, structs)
    for n, c in classes.items():
        assert lay[(n, "size")] == ctypes.sizeof(c), n
        for f in structs[n]:
            assert lay[(n, f)] == getattr(c, f).offset, (n, f)

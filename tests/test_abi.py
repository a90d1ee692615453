"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function include/sblm.h declares; the binding knows them all."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sblm.h")
LIB = os.path.join(ROOT, "paper_1208_4830_amd", "libsblm.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("sblm_magnify", "sblm_chi2", "ea_create", "ea_generation", "ea_fit",
              "ea_evaluate", "ea_save", "ea_load", "ea_destroy", "sblm_last_error"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsblm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_the_header():
    from paper_1208_4830_amd import sblm
    assert set(declared_functions()) == set(sblm.EXPORTS)


def test_oracle_is_not_imported_by_the_product():
    # the product path (package sources, HIP sources) never references the oracle
    pkg = os.path.join(ROOT, "paper_1208_4830_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "sblm_oracle" not in src, f


def test_struct_layouts_match_the_header(tmp_path):
    # sizes and field offsets of the header's structs, as gcc lays them out,
    # against the ctypes mirrors of the binding
    import shutil
    import subprocess
    from paper_1208_4830_amd import sblm
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    structs = {"ea_config": sblm.ea_config, "nm_config": sblm.nm_config,
               "ea_lc_summary": sblm.ea_lc_summary, "sblm_lcs": sblm.sblm_lcs}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "sblm.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines.append('  printf("sblm_stats size %zu\\n", sizeof(sblm_stats));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    for line in out.splitlines():
        name, field, value = line.split()
        if name == "sblm_stats":  # one uint64 per field of the binding's list
            assert int(value) == 8 * len(sblm.STATS_FIELDS)
            continue
        cls = structs[name]
        want = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert int(value) == want, (name, field, value, want)

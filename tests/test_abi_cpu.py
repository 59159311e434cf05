"""Host-side checks of the C ABI (no GPU needed): the built library exports
every function include/fiedler.h declares, the Python binding's ctypes
structures have the header's sizes and offsets, and the package fails loudly
when the library is missing."""
import ctypes as C
import os
import re
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fiedler.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fv_[a-z_]+)\s*\(", src)))


def test_header_lists_the_boundary():
    names = header_functions()
    for f in ["fv_build_hierarchy", "fv_fiedler_solve", "fv_fiedler_solve_batch", "fv_submit",
              "fv_poll", "fv_context_create", "fv_server_create"]:
        assert f in names


def test_library_exports_every_declared_symbol(fv):
    L = C.CDLL(fv.LIB_PATH)
    missing = [f for f in header_functions() if not hasattr(L, f)]
    assert not missing, missing
    assert sorted(fv.EXPORTS) == header_functions()


def test_ctypes_layouts_match_header(fv, tmp_path):
    structs = {"fv_csr": fv.fv_csr, "fv_hier_opts": fv.fv_hier_opts,
               "fv_solve_opts": fv.fv_solve_opts, "fv_solve_stats": fv.fv_solve_stats,
               "fv_server_opts": fv.fv_server_opts, "fv_request": fv.fv_request,
               "fv_result": fv.fv_result, "fv_batch_opts": fv.fv_batch_opts,
               "fv_partition_opts": fv.fv_partition_opts,
               "fv_partition_stats": fv.fv_partition_stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fiedler.h"',
             "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} sizeof %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            cname = "lambda" if fname == "lambda_" else fname
            lines.append(f'  printf("{name} {fname} %zu\\n", offsetof({name}, {cname}));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                           str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {}
    for line in out:
        if line:
            s, f, v = line.split()
            got[(s, f)] = int(v)
    for name, cls in structs.items():
        assert got[(name, "sizeof")] == C.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert got[(name, fname)] == getattr(cls, fname).offset, (name, fname)


def test_package_fails_loudly_without_library(tmp_path):
    code = textwrap.dedent(f"""
        import sys
        sys.path.insert(0, {ROOT!r})
        import paper_1602_04386_amd as fv
        fv.LIB_PATH = {str(tmp_path / 'missing.so')!r}
        try:
            fv.lib()
        except ImportError as e:
            print("raised", e)
            sys.exit(0)
        sys.exit(1)
    """)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert r.returncode == 0 and "raised" in r.stdout


def test_no_oracle_in_product_path():
    """The library sources and the binding never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_1602_04386_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "or_solve" not in text, f

"""The C ABI: header, shared library and Python binding agree (no GPU needed).

No compute call is made here; the library is only loaded and inspected.
"""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlb.h")
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                 if f.endswith(".h"))


def _header():
    text = ""
    for h in HEADERS:
        with open(h) as fh:
            text += fh.read() + "\n"
    return re.sub(r"/\*.*?\*/", "", text, flags=re.S)


def _declared_functions():
    """name -> number of parameters, from the prototypes in the header."""
    out = {}
    for m in re.finditer(r"^\s*(?:const\s+)?\w+\s*\*?\s*(mlb_\w+)\s*\(([^;]*?)\)\s*;", _header(), re.M | re.S):
        params = [p for p in m.group(2).split(",") if p.strip() and p.strip() != "void"]
        out[m.group(1)] = len(params)
    return out


def _declared_structs():
    out = {}
    for m in re.finditer(r"typedef\s+struct\s*\{(.*?)\}\s*(\w+)\s*;", _header(), re.S):
        fields = []
        for decl in m.group(1).split(";"):
            decl = decl.strip()
            if not decl:
                continue
            name = re.search(r"(\w+)\s*(?:\[\s*\d+\s*\])?\s*$", decl).group(1)
            fields.append(name)
        out[m.group(2)] = fields
    return out


def _declared_constants():
    return {m.group(1): int(m.group(2))
            for m in re.finditer(r"#define\s+(MLB_\w+)\s+(-?\d+)", _header())}


def _binding():
    from paper_1909_13585_amd import _binding as B
    return B


def _lib():
    B = _binding()
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libmlb.so is not built (run __graft_entry__.build())")
    return B.load()


def test_header_parses():
    fns = _declared_functions()
    assert len(fns) >= 20
    assert {"mlb_create", "mlb_buckling_dev", "mlb_sensitivities_dev", "mlb_vcycle_dev", "mlb_nn_conv3d"} <= set(fns)


def test_library_exports_every_declared_symbol():
    lib = _lib()
    missing = [name for name in _declared_functions() if not hasattr(lib, name)]
    assert not missing, missing


def test_exported_symbols_are_extern_c():
    B = _binding()
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libmlb.so is not built")
    nm = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True)
    if nm.returncode != 0:
        pytest.skip("nm not available")
    exported = {ln.split()[-1] for ln in nm.stdout.splitlines() if " T " in ln}
    for name in _declared_functions():
        assert name in exported, f"{name} is not an unmangled text symbol"


def test_binding_signatures_match_header():
    B = _binding()
    fns = _declared_functions()
    assert set(B._SIGS) == set(fns)
    for name, nparam in fns.items():
        assert len(B._SIGS[name][1]) == nparam, name


def test_constants_match_header():
    B = _binding()
    for name, value in _declared_constants().items():
        assert getattr(B, name) == value, name


def test_struct_fields_match_header():
    B = _binding()
    structs = _declared_structs()
    pairs = {"mlb_desc": B.MlbDesc, "mlb_opts": B.MlbOpts, "mlb_solve_info": B.MlbSolveInfo,
             "mlb_eig_info": B.MlbEigInfo, "mlb_tune_info": B.MlbTuneInfo, "mlb_batch_desc": B.MlbBatchDesc,
             "mlb_batch_opts": B.MlbBatchOpts, "mlb_batch_info": B.MlbBatchInfo, "mlb_mma_opts": B.MlbMmaOpts,
             "mlb_mma_info": B.MlbMmaInfo}
    assert set(pairs) <= set(structs)
    for cname, py in pairs.items():
        assert [f for f, _ in py._fields_] == structs[cname], cname


def test_struct_layout_matches_c_compiler(tmp_path):
    """sizeof/offsetof from gcc on the header equal the ctypes layout."""
    B = _binding()
    pairs = {"mlb_desc": B.MlbDesc, "mlb_opts": B.MlbOpts, "mlb_solve_info": B.MlbSolveInfo,
             "mlb_eig_info": B.MlbEigInfo, "mlb_tune_info": B.MlbTuneInfo, "mlb_batch_desc": B.MlbBatchDesc,
             "mlb_batch_opts": B.MlbBatchOpts, "mlb_batch_info": B.MlbBatchInfo, "mlb_mma_opts": B.MlbMmaOpts,
             "mlb_mma_info": B.MlbMmaInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>'] + [f'#include "{h}"' for h in HEADERS] + ["int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    cc = subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(src)], capture_output=True, text=True)
    if cc.returncode != 0:
        pytest.skip("gcc unavailable: " + cc.stderr[:200])
    got = dict(ln.split() for ln in subprocess.run([str(exe)], capture_output=True, text=True,
                                                   check=True).stdout.splitlines())
    for cname, py in pairs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)

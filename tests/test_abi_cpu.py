"""CPU-side checks of the C ABI: the library loads and exports every function
that include/*.h declares, and the binding's signature table matches."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2403_17518_amd", "libfwi.so")


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        for m in re.finditer(r"\b([A-Za-z_][A-Za-z0-9_]*)\s*\(", src):
            name = m.group(1)
            pre = src[:m.start()].rstrip()
            # a declaration: preceded by a return type, not a keyword/macro use
            if name in {"if", "for", "while", "return", "sizeof", "defined"}:
                continue
            if re.search(r"(int|void|char\s*\*|const char\s*\*|double|float)\s*\**\s*$", pre):
                names.add(name)
    return names


def test_header_declares_the_operators():
    names = _declared_functions()
    for op in ("fwi_forward", "fwi_gradient", "born_demig", "born_mig",
               "fwi_ctx_create", "fwi_ctx_destroy", "fwi_last_error"):
        assert op in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfwi.so not built")
def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (provides the HIP runtime the library links to)
    lib = ctypes.CDLL(LIB)
    missing = [n for n in sorted(_declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfwi.so not built")
def test_binding_signatures_cover_the_header():
    from paper_2403_17518_amd import _abi
    assert set(_abi.SIGNATURES) == _declared_functions()


def test_struct_layouts_match_header(tmp_path):
    """Sizes and field offsets of the ctypes mirrors equal what a C compiler
    makes of include/fwi.h and include/deblur.h."""
    import subprocess
    from paper_2403_17518_amd import _abi
    structs = {"fwi_grid": _abi.fwi_grid, "fwi_geom": _abi.fwi_geom, "fwi_stats": _abi.fwi_stats,
               "deblur_cfg": _abi.deblur_cfg, "deblur_layer_stat": _abi.deblur_layer_stat}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fwi.h"', '#include "deblur.h"',
             "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            cname = "pass" if f[0] == "pass_" else f[0]   # a Python keyword in the mirror
            lines.append(f'printf("{name}.{f[0]} %zu\\n", offsetof({name}, {cname}));')
    lines += ["return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.split("\n") if l)
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f in cls._fields_:
            assert int(got[f"{name}.{f[0]}"]) == getattr(cls, f[0]).offset, (name, f[0])


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2403_17518_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*"), recursive=True):
        if os.path.isfile(path) and path.endswith((".py", ".hip", ".h", ".cpp")):
            txt = open(path).read()
            assert "import oracle" not in txt and "from oracle" not in txt, path
            assert "fwi_oracle" not in txt and "liboracle" not in txt, path


def test_missing_library_fails_loudly(tmp_path):
    """Without the built library the binding raises; there is no fallback."""
    import subprocess
    import sys
    code = ("import paper_2403_17518_amd._abi as a\n"
            f"try:\n    a.load({str(tmp_path / 'libfwi.so')!r})\n"
            "except RuntimeError as e:\n    print('refused:', e)\nelse:\n    print('loaded')\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    assert "refused:" in r.stdout and "missing" in r.stdout

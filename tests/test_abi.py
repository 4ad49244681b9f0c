"""The C-ABI library builds, loads and exports every entry point that
include/ss.h declares (no GPU work is done here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ss.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(ss_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_core_entry_points():
    names = _declared()
    for must in ["ss_build_liouvillian", "ss_solve", "ss_submit", "ss_poll", "ss_prepare",
                 "ss_export_csr", "ss_apply", "ss_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1504_06768_amd import ss
    lib = ctypes.CDLL(ss.library_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    assert set(ss.EXPORTED) == set(_declared())


def test_options_defaults_and_version():
    from paper_1504_06768_amd import ss
    o = ss.options()
    assert (o.prec, o.ilu, o.ordering, o.gmres_m, o.maxiter) == (0, 0, 0, 20, 1000)
    assert o.sigma == 1e-15 and o.drop_tol == 1e-4 and o.fill == 10.0
    assert "gfx950" in ss.version()


def test_struct_layouts_match_header():
    """The ctypes mirrors have the sizes the header implies."""
    from paper_1504_06768_amd import ss
    assert ctypes.sizeof(ss._Csr) == 40
    assert ctypes.sizeof(ss._Options) == 8 * 4 + 5 * 8 + 8 + 2 * 4
    assert ctypes.sizeof(ss._Info) == 8 * 4 + 3 * 8 + 10 * 8 + 2 * 4
    assert ctypes.sizeof(ss._ServerStats) == 3 * 8 + 2 * 4 + 2 * 8 + 2 * 4


def test_product_package_does_not_touch_the_oracle():
    """The product path never imports, reads or runs the oracle."""
    pkg = os.path.join(ROOT, "paper_1504_06768_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert re.search(r"\boracle\b", text) is None, f


def test_binding_constants_match_the_header():
    """Every SS_* constant the binding defines has the header's value."""
    from paper_1504_06768_amd import ss
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+(SS_[A-Z0-9_]+)\s+(-?\d+)\b", src)}
    assert "SS_OP_APPLY_L" in defs and "SS_FLAG_MATRIX_FREE" in defs
    mismatched = {k: (v, getattr(ss, k)) for k, v in defs.items() if hasattr(ss, k) and getattr(ss, k) != v}
    assert not mismatched
    for k in ("SS_OP_APPLY_L", "SS_FLAG_MATRIX_FREE", "SS_AUTO", "SS_FLAG_COND_EST", "SS_OP_PRECOND_LEVELS"):
        assert getattr(ss, k) == defs[k]

"""Host-side checks of the C ABI library that need no GPU: it loads, it exports every function that
include/asdsm.h declares, and the binding's structures match the header."""
import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "asdsm.h"
HEADERS = sorted((ROOT / "include").glob("*.h"))


def _declared(path=None):
    names = set()
    for h in ([path] if path else HEADERS):
        text = h.read_text()
        names |= set(re.findall(r"^\s*(?:int|void|size_t|const char \*)\s*\*?\s*(asdsm_\w+)\s*\(", text, re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2303_01163_amd import asdsm
    if not asdsm.LIB_PATH.exists():
        from paper_2303_01163_amd.build import build_library
        build_library()
    return asdsm.load_library()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("asdsm_plan", "asdsm_solve", "asdsm_residual", "asdsm_workspace_size",
              "asdsm_set_workspace", "asdsm_mesh_solve", "asdsm_destroy", "asdsm_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2303_01163_amd.asdsm import EXPORTED, EXPORTED_LEARN
    assert sorted(EXPORTED) == _declared(HEADER)
    assert sorted(EXPORTED_LEARN) == _declared(ROOT / "include" / "asdsm_learn.h")
    names = _declared()
    assert sorted(EXPORTED + EXPORTED_LEARN) == names
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layouts_match_header():
    from paper_2303_01163_amd.asdsm import Opts, Stats, NPHASE
    text = HEADER.read_text()
    assert f"#define ASDSM_NPHASE           {NPHASE}" in text
    # field order of asdsm_opts / asdsm_stats as declared
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    opts_fields = re.search(r"typedef struct \{([^}]*)\} asdsm_opts;", text).group(1)
    decl = re.findall(r"(\w+)\s*(?:\[[^\]]*\])?;", opts_fields)
    assert decl == [f[0] for f in Opts._fields_]
    stats_fields = re.search(r"typedef struct \{([^}]*)\} asdsm_stats;", text).group(1)
    decl = re.findall(r"(\w+)\s*(?:\[[^\]]*\])?;", stats_fields)
    assert decl == [f[0] for f in Stats._fields_]


def test_errors_without_gpu_are_reported(lib):
    """Argument validation happens before any device call, so it works on a host without a GPU."""
    h = ctypes.c_void_p()
    a = (ctypes.c_double * 2)(1.0, 1.0)
    b = (ctypes.c_double * 2)(0.0, 0.0)
    assert lib.asdsm_plan(ctypes.byref(h), 5, a, b, 5, 0, 0, None) == -1
    assert b"d must be" in lib.asdsm_last_error()
    assert lib.asdsm_plan(ctypes.byref(h), 2, a, b, 5, 7, 0, None) == -2
    neg = (ctypes.c_double * 2)(1.0, -2.0)
    assert lib.asdsm_plan(ctypes.byref(h), 2, neg, b, 5, 0, 0, None) == -1
    assert lib.asdsm_solve(None, None, None, None, None, None) == -1


def test_product_path_does_not_import_the_oracle():
    """The library binding and the package never reference the oracle."""
    pkg = ROOT / "paper_2303_01163_amd"
    for f in list(pkg.glob("*.py")) + list((pkg / "csrc").glob("*")):
        assert "oracle" not in f.read_text(), f

"""CPU checks of the C ABI library: it loads without a GPU, exports every
entry point include/cbs.h declares, and the binding's structures match the
header's field order."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cbs.h")).read()
    return sorted(set(re.findall(r"^cbs_status\s+(cbs_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_2507_16087_amd import _lib
    lib = _lib.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_lib.EXPORTS) == names


def test_struct_fields_follow_header():
    from paper_2507_16087_amd import _lib
    src = open(os.path.join(ROOT, "include", "cbs.h")).read()
    for struct, cls in (("cbs_grid", _lib.Grid), ("cbs_solve_opts", _lib.SolveOpts),
                        ("cbs_solve_info", _lib.SolveInfo)):
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + struct + ";", src).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = re.findall(r"(\w+)(?:\[\d+\])?\s*[;,]", body)
        assert fields == [f for f, _ in cls._fields_], (struct, fields)


def test_binding_has_no_cpu_fallback(monkeypatch):
    """Without the built library the binding raises instead of computing."""
    from paper_2507_16087_amd import _lib
    monkeypatch.setattr(_lib, "_LIB", None)
    monkeypatch.setattr(_lib, "LIB_PATH", os.path.join(ROOT, "does-not-exist.so"))
    with pytest.raises(RuntimeError):
        _lib.lib()


def test_product_never_imports_oracle():
    pkg = os.path.join(ROOT, "paper_2507_16087_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", text).lower() or f == "workloads.py", f


def test_status_codes_match_header():
    from paper_2507_16087_amd import _lib
    src = open(os.path.join(ROOT, "include", "cbs.h")).read()
    for name in ("CBS_OK", "CBS_NOT_CONVERGED", "CBS_E_INVALID", "CBS_E_UNSUPPORTED",
                 "CBS_E_NOMEM", "CBS_E_DEVICE", "CBS_E_DIVERGED", "CBS_FP64", "CBS_FP32_REFINED"):
        m = re.search(name + r"\s*=\s*(-?\d+)", src)
        assert m and int(m.group(1)) == getattr(_lib, name), name

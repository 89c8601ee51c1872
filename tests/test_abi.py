"""The C-ABI library loads and exports every entry point include/skx.h declares
(no GPU needed: nothing here calls into the device)."""
import os
import re
import ctypes

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "skx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(skx_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("skx_set_cell", "skx_set_ions", "skx_set_functional",
                 "skx_evaluate_energy_potential", "skx_optimize_density", "skx_run_batch",
                 "skx_engine_submit", "skx_engine_step"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2601_23002_amd", "libskx.so"))
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_imports_without_gpu():
    from paper_2601_23002_amd import skx
    assert skx.OK == 0 and skx.E_NUMERIC == -5


def test_default_radix_orders_factor_the_length():
    """Host-side plan logic (no device call): the default radix order of every
    accepted length multiplies back to it and prefers radix 8."""
    from paper_2601_23002_amd import skx
    from paper_2601_23002_amd.workloads import ALLOWED_N
    for n in ALLOWED_N:
        r = skx.radix_order(n, skx.FP64)
        assert all(x in (2, 3, 4, 5, 8) for x in r)
        prod = 1
        for x in r:
            prod *= x
        assert prod == n, (n, r)
    assert skx.radix_order(64) == [8, 8]
    assert skx.radix_order(96) == [8, 4, 3]


def test_binding_refuses_to_load_without_the_library(tmp_path):
    """No CPU fallback: a copy of the binding with no libskx.so beside it
    fails at import, naming the missing library."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "skx_nolib"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_2601_23002_amd", "skx.py"), pkg / "skx.py")
    r = subprocess.run([sys.executable, "-c", "import skx_nolib.skx"], cwd=tmp_path,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "libskx.so not built" in r.stderr


def test_contexts_need_a_gpu():
    """Without a visible GPU the binding raises instead of computing on the
    host."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_2601_23002_amd import skx
    with pytest.raises(RuntimeError, match="needs a GPU"):
        skx.Context(0)

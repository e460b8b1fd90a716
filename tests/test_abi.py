"""The C-ABI library loads without a GPU and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hfsi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hfsi_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_hot_path():
    names = _declared()
    for must in ("hfsi_assemble_residual_tangent", "hfsi_amg_setup", "hfsi_krylov_amg_solve", "hfsi_newton_step"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1312_5561_amd import hfsi
    if not os.path.exists(hfsi.LIB_PATH):
        pytest.fail("libhfsi.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(hfsi.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.hfsi_abi_version() == 11


def test_binding_has_no_cpu_fallback():
    """The binding module must not import the oracle or any CPU solver."""
    src = open(os.path.join(ROOT, "paper_1312_5561_amd", "hfsi.py")).read()
    assert "oracle" not in src.replace("no fallback", "")
    assert "scipy" not in src


def test_c_example_links_and_checks_its_arguments():
    """The C example is built against the library and the HIP runtime; run
    without arguments it prints its usage and exits with status 2 before any
    GPU call."""
    import subprocess

    from paper_1312_5561_amd import build as b
    if not os.path.exists(b.DRIVER):
        pytest.fail(f"{b.DRIVER} is not built (run __graft_entry__.build())")
    r = subprocess.run([b.DRIVER], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "usage" in r.stderr


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0 and "one GPU only" in (r.stdout + r.stderr)

"""The C-ABI library loads on a machine without a GPU and exports every
entry point that include/vd.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vd_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_hot_path():
    names = _declared()
    for n in ("vd_poisson_solve", "vd_helmholtz_solve_batched", "vd_species_flux", "vd_reaction_source", "vd_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2507_08200_amd import vd
    if not os.path.exists(vd.LIB_PATH):
        from paper_2507_08200_amd import build
        build.build()
    lib = ctypes.CDLL(vd.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(vd.EXPORTS) == set(_declared())
    lib.vd_version.restype = ctypes.c_char_p
    assert lib.vd_version().startswith(b"libvd")


def test_binding_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    from paper_2507_08200_amd import vd
    with pytest.raises(ValueError):
        vd._dptr(torch.zeros(4, dtype=torch.float64), name="x")


def test_binding_fails_loudly_without_the_library(monkeypatch):
    """No CPU fallback: with the shared library absent the binding raises
    instead of computing anything."""
    from paper_2507_08200_amd import vd
    monkeypatch.setattr(vd, "_lib", None)
    monkeypatch.setattr(vd, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libvd.so"))
    with pytest.raises(ImportError):
        vd.load()


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits with a message and status 2
    before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stdout

"""The C-ABI library loads on the CPU and exports every entry point that
include/sim.h declares (no compute calls: those need a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(?:int|const char \*)\s*((?:sim|srv)_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("sim_create", "sim_destroy", "sim_step", "sim_rollout", "sim_backward", "sim_set_params",
              "srv_create", "srv_submit", "srv_result", "srv_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2603_25068_amd import sim
    lib = ctypes.CDLL(sim.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(_declared()) == sorted(sim.exported_symbols())


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2603_25068_amd import sim
    monkeypatch.setattr(sim, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(sim, "_LIB", None)
    import pytest
    with pytest.raises(RuntimeError):
        sim.lib()

"""The C-ABI library loads and exports every function include/stratego.h declares
(no GPU calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "stratego.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(stratego_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("stratego_init", "stratego_reset", "stratego_legal_mask", "stratego_step",
                     "stratego_encode_obs", "stratego_sample_actions", "stratego_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2511_07312_amd import build as B
    if B.is_stale():
        B.build()
    lib = ctypes.CDLL(B.LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    from paper_2511_07312_amd import engine
    assert sorted(engine.FUNCTIONS) == declared_functions()


def test_strerror_without_gpu():
    from paper_2511_07312_amd import engine
    assert engine.strerror(0) == "ok"
    assert "illegal" in engine.strerror(engine.E_ILLEGAL_ACTION)


def test_binding_rejects_host_tensors():
    import pytest
    import torch
    from paper_2511_07312_amd import engine
    with pytest.raises(TypeError):
        engine._ptr(torch.zeros(4, dtype=torch.int16), torch.int16, None, "actions")

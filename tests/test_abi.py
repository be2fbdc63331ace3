"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/mmfv.h declares, and rejects invalid configurations before touching
the device."""
import os
import re
import subprocess

import pytest

import paper_1704_00519_amd as pk
import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "mmfv.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("mm_create", "mm_init_state", "mm_step", "mm_get_conserved",
                 "mm_adjoint_step", "mm_destroy", "mm_last_error"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    if not os.path.exists(pk.LIB_PATH):
        pytest.skip("library not built")
    out = subprocess.run(["nm", "-D", "--defined-only", pk.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (mm_[a-z_]+)$", out, flags=re.M))
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    assert set(pk.EXPORTS) <= exported
    L = pk.load()
    for s in declared_symbols():
        assert hasattr(L, s)


@pytest.mark.parametrize("field,value", [("dim", 3), ("nx", 0), ("n_mat", 0),
                                         ("rk_order", 4), ("cfl", 0.0),
                                         ("k_ext", 9), ("inflow_mat", 5)])
def test_invalid_config_rejected(field, value):
    if not os.path.exists(pk.LIB_PATH):
        pytest.skip("library not built")
    cfg = wl.shock_tube_1d()["cfg"]
    cfg[field] = value
    with pytest.raises(pk.MMError) as e:
        pk.Solver(cfg)
    assert e.value.status == 1  # MM_EINVAL


def test_gamma_must_exceed_one():
    if not os.path.exists(pk.LIB_PATH):
        pytest.skip("library not built")
    cfg = wl.shock_tube_1d()["cfg"]
    cfg["gamma"] = [1.0, 1.4, 1.4]
    with pytest.raises(pk.MMError):
        pk.Solver(cfg)


def test_device_arguments_checked_before_the_call():
    """The binding refuses device-pointer arguments that are not contiguous
    CUDA tensors of the expected dtype and size (before any library call)."""
    import torch
    from paper_1704_00519_amd import _lib
    with pytest.raises(TypeError):
        _lib._device_arg(torch.zeros(4, dtype=torch.float64), "torch.float64", 4, "x")
    with pytest.raises(TypeError):
        _lib._device_arg(__import__("numpy").zeros(4), "torch.float64", 4, "x")

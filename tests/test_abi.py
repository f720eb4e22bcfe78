"""The C-ABI library loads and exports every entry point include/sbfwi.h declares
(no compute calls: this runs without a GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sbfwi.h")
LIB = os.path.join(ROOT, "paper_2501_06748_amd", "libsbfwi.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sbfwi_[a-z_]+)\s*\(", text)))


def test_header_declares_boundary_calls():
    names = declared()
    for n in ("sbfwi_build_mesh", "sbfwi_factor_elements", "sbfwi_forward", "sbfwi_adjoint", "sbfwi_gradient"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsbfwi.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsbfwi.so not built")
def test_binding_covers_every_symbol():
    from paper_2501_06748_amd import _abi
    assert set(declared()) == set(_abi.SIGNATURES)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsbfwi.so not built")
def test_host_validation_without_gpu():
    """Mesh validation is host code: a clockwise loop is rejected with SBFWI_EINVAL."""
    import numpy as np
    import paper_2501_06748_amd as sb
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], dtype=np.float64)
    with pytest.raises(sb.SbfwiError) as ei:
        sb.sbfwi_build_mesh(xy, [0, 4], [0, 3, 2, 1], [5])
    assert ei.value.code == -1
    assert "counter-clockwise" in sb.sbfwi_last_error() or "det J_b" in sb.sbfwi_last_error()

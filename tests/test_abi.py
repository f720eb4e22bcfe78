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


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsbfwi.so not built")
@pytest.mark.parametrize("case", ["shots", "receivers", "steps", "grad", "per_shot_grad", "misfit"])
def test_run_shape_mismatch_raises_before_any_device_call(case):
    """Arrays passed with a checkpoint handle are checked against the run's shot,
    receiver and step counts on the host (ValueError), before any pointer reaches
    the library: the C ABI takes no sizes for them."""
    import torch
    import paper_2501_06748_amd as sb
    S, R, N, P = 3, 5, 7, 40
    ck = sb.CkptHandle(None, None, n_shots=S, n_rec=R, n_steps=N, n_params=P)
    good = torch.zeros((S, R, N), dtype=torch.float64)
    bad = {"shots": torch.zeros((S - 1, R, N), dtype=torch.float64),
           "receivers": torch.zeros((S, R + 1, N), dtype=torch.float64),
           "steps": torch.zeros((S, R, N - 1), dtype=torch.float64)}
    grad = torch.zeros(P, dtype=torch.float64)
    mis = torch.zeros(1, dtype=torch.float64)
    if case in bad:
        with pytest.raises(ValueError):
            sb.sbfwi_adjoint(None, ck, bad[case], sb.GRAD_EXACT, grad)
        with pytest.raises(ValueError):
            sb.sbfwi_gradient(None, ck, good, bad[case], sb.GRAD_EXACT, mis, grad)
        with pytest.raises(ValueError):
            sb.sbfwi_gradient(None, ck, bad[case], good, sb.GRAD_EXACT, mis, grad)
    elif case == "grad":
        with pytest.raises(ValueError):
            sb.sbfwi_adjoint(None, ck, good, sb.GRAD_EXACT, torch.zeros(P - 1, dtype=torch.float64))
    elif case == "per_shot_grad":
        with pytest.raises(ValueError):
            sb.sbfwi_adjoint(None, ck, good, sb.GRAD_EXACT | sb.GRAD_PER_SHOT, grad)
    else:
        with pytest.raises(ValueError):
            sb.sbfwi_gradient(None, ck, good, good, sb.GRAD_EXACT | sb.GRAD_PER_SHOT,
                              mis, torch.zeros(S * P, dtype=torch.float64))
    # correctly sized arrays pass the shape check (and then stop at the device-pointer check)
    with pytest.raises(TypeError):
        sb.sbfwi_adjoint(None, ck, good, sb.GRAD_EXACT, grad)

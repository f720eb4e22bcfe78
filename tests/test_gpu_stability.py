"""The growth detector of forward runs on the GPU (SBFWI_EUNSTABLE).

- the paper's radial finite differences on the tiny plate with the void at the
  1e-5 density floor (a model the stability gate marks as growing): the run
  completes, and sbfwi_forward returns SBFWI_EUNSTABLE with the first step
  beyond the envelope, which lies where the oracle's loop crosses it (the
  first 40 steps);
- the radial Galerkin scheme on the same model runs clean;
- no false positive over 4000 steps on gate-passing models: the benchmark
  plate (homogeneous, n_b 16, N_r 32, four shots, direct coarse solver) and a
  reduced plate with a +-30 % random field and random-normal wavelets, which
  keep forcing the free plate's rigid-body mode.
"""

import re

import numpy as np
import pytest

import workloads as W

from ._gpu import GpuModel, log

pytestmark = pytest.mark.gpu


def test_finite_differences_on_floor_void_report_unstable():
    import paper_2501_06748_amd as sb
    wl = W.config_tiny(200)
    log("paper FD, void at the 1e-5 floor, 200 steps: expect SBFWI_EUNSTABLE")
    g = GpuModel(wl, wl.models["void_data"], coarse_solver=1)
    with pytest.raises(sb.SbfwiError) as ei:
        g.forward(n_steps=200)
    msg = sb.sbfwi_last_error()
    log(f"  {ei.value}")
    assert ei.value.code == sb._abi.EUNSTABLE
    step = int(re.search(r"step (\d+)", msg).group(1))
    assert 1 <= step <= 40


def test_galerkin_scheme_on_floor_void_runs_clean():
    wl = W.config_tiny(200)
    log("radial Galerkin, void at the 1e-5 floor, 200 steps: no detector trip")
    g = GpuModel(wl, wl.models["void_data"], coarse_solver=1, scheme=1)
    tr, _ = g.forward(n_steps=200)
    assert np.isfinite(tr.cpu().numpy()).all()


def test_no_false_positive_over_4000_steps_on_the_benchmark_plate():
    wl = W.config_paper(n_steps=4000, n_shots=4)
    log("benchmark plate, homogeneous, 4 shots, 4000 steps: no detector trip")
    g = GpuModel(wl, wl.models["homogeneous"], coarse_solver=1)
    tr, _ = g.forward(n_steps=4000)
    t = tr.cpu().numpy()
    assert np.isfinite(t).all() and np.abs(t).max() > 0


def test_no_false_positive_over_4000_steps_with_random_forcing():
    wl = W.config_small(nx=8, ny=4, segs=2, n_r=17, n_steps=4000, n_shots=2)
    wl.wavelets = np.random.default_rng(11).standard_normal((2, 4000))
    log("reduced plate, +-30 % random field, random-normal wavelets, 4000 steps: no detector trip")
    g = GpuModel(wl, wl.models["random30"], coarse_solver=1)
    tr, _ = g.forward(n_steps=4000)
    assert np.isfinite(tr.cpu().numpy()).all()

"""The growth envelope of the library's forward runs, checked on the oracle.

The detector flags step k of shot q when a nodal displacement exceeds
10 * 4 k r F_k (r = largest 1 / |K_g,ii|, F_k = sum of |force| up to step k).
On the oracle's time loop: gate-passing models (homogeneous, smooth void at
floor 0.5, +-30 % random field; a random-normal wavelet that keeps forcing the
free plate's rigid-body mode) stay below 0.15 of 4 k r F_k for every step, and
the radial Galerkin scheme stays below it on the void at the 1e-5 floor;
the paper's finite differences on that void (whose step map the stability
gate marks as growing) exceed 10 times it within the first 40 steps.
"""

import numpy as np
import pytest

import workloads as W
from oracle import stepper as stp


def _worst_ratio(wl, rho, nt, wav=None, scheme="paper_fd", stop=None):
    m = stp.Model(wl.mesh, rho, wl.c, wl.dt, scheme=scheme)
    r = 1.0 / np.abs(m.K.diagonal()).min()
    wav = wl.wavelets if wav is None else wav
    st = m.zero_state(np.float64)
    F, worst = 0.0, 0.0
    for k in range(1, nt + 1):
        f = np.zeros(wl.mesh.n_nodes)
        f[wl.src_nodes[0]] += wav[0][k - 1]
        F += abs(wav[0][k - 1])
        st = stp.step(m, st, f)
        mx = np.abs(st["U"]).max()
        if not np.isfinite(mx):
            return np.inf, k
        if F > 0:
            worst = max(worst, mx / (4.0 * k * r * F))
        if stop is not None and worst > stop:
            return worst, k
    return worst, nt


@pytest.mark.parametrize("name", ["homogeneous", "void_floor_half", "random30"])
def test_stable_models_stay_inside_the_envelope(name):
    wl = W.config_tiny(200)
    worst, _ = _worst_ratio(wl, wl.models[name], 200)
    assert worst < 0.15


def test_rigid_body_forcing_stays_inside_the_envelope():
    wl = W.config_tiny(200)
    wav = np.random.default_rng(7).standard_normal((1, 200))
    worst, _ = _worst_ratio(wl, wl.models["homogeneous"], 200, wav=wav)
    assert worst < 0.15


def test_galerkin_scheme_on_the_floor_void_stays_inside():
    wl = W.config_tiny(200)
    worst, _ = _worst_ratio(wl, wl.models["void_data"], 200, scheme="radial_galerkin")
    assert worst < 0.15


def test_finite_differences_on_the_floor_void_leave_the_envelope():
    wl = W.config_tiny(200)
    worst, k = _worst_ratio(wl, wl.models["void_data"], 200, stop=10.0)
    assert worst > 10.0 and k <= 40

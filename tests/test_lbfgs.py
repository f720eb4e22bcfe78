"""Host logic of the outer L-BFGS loop (CPU tensors; no GPU, no library calls)."""

import math

import torch

from paper_2501_06748_amd import lbfgs
from paper_2501_06748_amd._abi import EUNSTABLE, SbfwiError


def _quadratic(n=40, seed=0):
    g = torch.Generator().manual_seed(seed)
    Q = torch.randn(n, n, generator=g, dtype=torch.float64)
    A = Q @ Q.T / n + 0.5 * torch.eye(n, dtype=torch.float64)
    b = torch.randn(n, generator=g, dtype=torch.float64)

    def fg(x):
        return float(0.5 * x @ A @ x - b @ x), A @ x - b
    return A, b, fg


def test_unconstrained_quadratic_converges():
    A, b, fg = _quadratic()
    x0 = torch.zeros(40, dtype=torch.float64)
    res = lbfgs.minimize_box(fg, x0, -1e9, 1e9, iters=80, memory=10, first_step=0.5)
    xs = torch.linalg.solve(A, b)
    assert torch.linalg.norm(res.x - xs) <= 1e-6 * torch.linalg.norm(xs)
    assert all(h1 <= h0 for h0, h1 in zip(res.history, res.history[1:]))


def test_box_constraints_hold_and_reach_projected_optimum():
    # separable objective: minimiser of each coordinate is known in closed form
    c = torch.linspace(-2.0, 3.0, 25, dtype=torch.float64)
    w = torch.linspace(1.0, 4.0, 25, dtype=torch.float64)

    def fg(x):
        return float((w * (x - c) ** 2).sum()), 2 * w * (x - c)
    lo, hi = 0.0, 1.0
    res = lbfgs.minimize_box(fg, torch.full((25,), 0.5, dtype=torch.float64), lo, hi, iters=60, first_step=0.25)
    assert float(res.x.min()) >= lo and float(res.x.max()) <= hi
    assert torch.allclose(res.x, c.clamp(lo, hi), atol=1e-8)


def test_line_search_backs_off_from_blow_up():
    # objective that "blows up" (raises like the library does) beyond x0 > 0.8
    def fg(x):
        if float(x[0]) > 0.8:
            raise SbfwiError(EUNSTABLE, "unstable")
        return float(((x - 2.0) ** 2).sum()), 2 * (x - 2.0)
    res = lbfgs.minimize_box(fg, torch.zeros(3, dtype=torch.float64), -5.0, 5.0, iters=8, first_step=1.5)
    assert res.rejected > 0
    assert float(res.x[0]) <= 0.8
    assert res.f < 12.0 and math.isfinite(res.f)


def test_other_library_errors_propagate():
    from paper_2501_06748_amd._abi import EINVAL

    def fg(x):
        raise SbfwiError(EINVAL, "bad input")
    try:
        lbfgs.minimize_box(fg, torch.zeros(2, dtype=torch.float64), -1.0, 1.0)
    except SbfwiError as e:
        assert e.code == EINVAL
    else:
        raise AssertionError("EINVAL must propagate")

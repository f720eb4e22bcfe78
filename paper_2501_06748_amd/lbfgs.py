"""The outer loop of the inversion: limited-memory BFGS with box constraints.

The paper minimises the waveform misfit over the densities with L-BFGS and
bound constraints (implementation notes of Section "Numerical examples").
This is a projected L-BFGS on device tensors: the two-loop recursion over the
last ``memory`` curvature pairs gives the search direction on the free
variables (those not held at a bound by the gradient), the trial point is
projected onto the box, and a backtracking line search accepts the first
step with sufficient decrease (Armijo) along the projected path.  A trial
point at which the simulation reports a blow-up (``SbfwiError`` with
SBFWI_EUNSTABLE or SBFWI_ENONFINITE) counts as an infinite objective, so the
line search backs off from it.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

from ._abi import EUNSTABLE, ENONFINITE, SbfwiError


@dataclass
class LbfgsResult:
    x: torch.Tensor
    f: float
    history: list = field(default_factory=list)       # objective after every accepted iteration
    evaluations: int = 0
    rejected: int = 0                                   # trial points that blew up or did not decrease


def _two_loop(g, S, Y):
    q = g.clone()
    alphas = []
    for s, y in zip(reversed(S), reversed(Y)):
        rho = 1.0 / torch.dot(y, s)
        a = rho * torch.dot(s, q)
        q -= a * y
        alphas.append((a, rho))
    if S:
        s, y = S[-1], Y[-1]
        q *= torch.dot(s, y) / torch.dot(y, y)
    for (s, y), (a, rho) in zip(zip(S, Y), reversed(alphas)):
        b = rho * torch.dot(y, q)
        q += (a - b) * s
    return q


def minimize_box(fun_grad, x0, lower, upper, iters=10, memory=10, first_step=0.05, c1=1e-4,
                 max_backtracks=12, callback=None) -> LbfgsResult:
    """Minimise f over lower <= x <= upper.

    fun_grad(x) -> (f: float, g: tensor like x); may raise SbfwiError.
    first_step: the first iteration (and any restart) moves along the
    projected steepest descent with max |dx| = first_step."""
    x = torch.clamp(x0.detach().clone(), lower, upper)
    f, g = fun_grad(x)
    res = LbfgsResult(x=x, f=float(f), history=[float(f)], evaluations=1)
    S, Y = [], []
    for it in range(iters):
        free = ~(((x <= lower) & (g > 0)) | ((x >= upper) & (g < 0)))
        gf = torch.where(free, g, torch.zeros_like(g))
        if float(gf.abs().max()) == 0.0:
            break
        d = -_two_loop(gf, S, Y) if S else None
        if d is not None:
            d = torch.where(free, d, torch.zeros_like(d))
        if d is None or float(torch.dot(d, gf)) >= 0.0:
            S, Y = [], []
            d = -gf * (first_step / float(gf.abs().max()))
        t = 1.0
        accepted = False
        for _ in range(max_backtracks):
            xt = torch.clamp(x + t * d, lower, upper)
            try:
                ft, gt = fun_grad(xt)
                ft = float(ft)
            except SbfwiError as err:
                if err.code not in (EUNSTABLE, ENONFINITE):
                    raise
                ft, gt = math.inf, None
            res.evaluations += 1
            if math.isfinite(ft) and ft <= f + c1 * float(torch.dot(g, xt - x)):
                accepted = True
                break
            res.rejected += 1
            t *= 0.5
        if not accepted:
            break
        s, y = xt - x, gt - g
        sy = float(torch.dot(s, y))
        if sy > 1e-12 * float(s.norm() * y.norm()):
            S.append(s)
            Y.append(y)
            if len(S) > memory:
                S.pop(0)
                Y.pop(0)
        x, f, g = xt, ft, gt
        res.history.append(f)
        if callback is not None:
            callback(it, x, f, g)
    res.x, res.f = x, f
    return res

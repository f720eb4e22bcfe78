"""Differentiable forward simulation: densities -> receiver traces.

The forward run (factorisation of every element, then the condensed time loop
with sqrt(T) checkpoints) is the forward of a ``torch.autograd.Function``;
its backward is the library's adjoint run (``sbfwi_adjoint``): the
checkpointed forward segments are recomputed in reverse, the adjoint state is
stepped back in time, and the zero-lag correlation of adjoint and forward
fields gives the vector-Jacobian product with respect to every fine-grid
density (Section "Adjoint method": the gradient of an objective of the
traces needs one additional, backward simulation).

Any differentiable objective of the traces can sit on top; for the waveform
misfit of eq. misfit use ``misfit``.  The backward of mode
``GRAD_PAPER_KERNEL`` is the paper's truncated kernel, an approximation of
the vector-Jacobian product (kept for comparison with the paper); the default
``GRAD_EXACT`` is exact for the discrete model.
"""

from __future__ import annotations

from dataclasses import dataclass

import torch
from torch.autograd.function import once_differentiable

from . import (GRAD_EXACT, sbfwi_adjoint, sbfwi_misfit, sbfwi_factor_elements, sbfwi_forward, sbfwi_mesh_info,
               sbfwi_set_solver)


@dataclass
class WaveProblem:
    """Everything of a forward run except the densities (device tensors on one GPU).

    mesh: handle from sbfwi_build_mesh; src [S] int64, wavelet [S, N_t] f64,
    rec [R] int64; n_ckpt as in sbfwi_forward (-1 = sqrt(T) checkpoints,
    >= N_t = full storage); mode: GRAD_EXACT or GRAD_PAPER_KERNEL; rtol: relative
    residual of the iterative coarse solves (the library default 1e-13 when None);
    coarse_solver: 1 = direct (factored once per model), 0 = BiCGStab;
    scheme: SCHEME_PAPER_FD (0) or SCHEME_RADIAL_GALERKIN (1)."""
    mesh: object
    c: float
    dt: float
    src: torch.Tensor
    wavelet: torch.Tensor
    rec: torch.Tensor
    beta: float = 0.25
    gamma: float = 0.5
    n_ckpt: int = -1
    mode: int = GRAD_EXACT
    rtol: float = None
    coarse_solver: int = 1
    scheme: int = 0

    @property
    def n_params(self) -> int:
        return sbfwi_mesh_info(self.mesh)["n_params"]

    def trace_shape(self):
        return (int(self.wavelet.shape[0]), int(self.rec.shape[0]), int(self.wavelet.shape[1]))


class _Traces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho, prob):
        rho_d = rho.detach().contiguous()
        f = sbfwi_factor_elements(prob.mesh, rho_d, prob.c, prob.dt, prob.beta, prob.gamma,
                                  scheme=prob.scheme, coarse_solver=prob.coarse_solver)
        if prob.rtol is not None:
            sbfwi_set_solver(f, prob.rtol, 500)
        traces = torch.zeros(prob.trace_shape(), dtype=torch.float64, device=rho.device)
        need = ctx.needs_input_grad[0]
        ck = sbfwi_forward(f, prob.src, prob.wavelet, prob.rec, traces, n_ckpt=prob.n_ckpt if need else 0)
        ctx.prob, ctx.f, ctx.ck = prob, f, ck
        ctx.n_params = rho.numel()
        return traces

    @staticmethod
    @once_differentiable
    def backward(ctx, g_traces):
        if ctx.ck is None:
            return None, None
        grad = torch.empty(ctx.n_params, dtype=torch.float64, device=g_traces.device)
        sbfwi_adjoint(ctx.f, ctx.ck, g_traces.contiguous().to(torch.float64), ctx.prob.mode, grad)
        return grad, None


def simulate(rho: torch.Tensor, prob: WaveProblem) -> torch.Tensor:
    """Receiver traces [S, R, N_t] of the forward run at densities rho [n_params];
    differentiable with respect to rho (backward = adjoint run)."""
    if rho.dtype != torch.float64 or not rho.is_cuda or rho.dim() != 1:
        raise TypeError("rho must be a 1-D float64 CUDA (ROCm) tensor")
    return _Traces.apply(rho, prob)


class _Misfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, traces, observed, dt):
        tr, ob = traces.detach().contiguous(), observed.detach().contiguous()
        val = torch.zeros(1, dtype=torch.float64, device=tr.device)
        res = torch.empty_like(tr)
        sbfwi_misfit(ob, tr, dt, val, residual=res)
        ctx.save_for_backward(res)
        return val[0]

    @staticmethod
    @once_differentiable
    def backward(ctx, g):
        (res,) = ctx.saved_tensors
        return res * g, -res * g, None


def misfit(traces: torch.Tensor, observed: torch.Tensor, dt: float) -> torch.Tensor:
    """Waveform misfit of eq. misfit with the rectangle rule, 1/2 sum dt (u - d)^2,
    computed by the library (sbfwi_misfit, which also returns the residual
    dt (u - d) that the backward passes on)."""
    return _Misfit.apply(traces.to(torch.float64), observed.to(torch.float64), float(dt))

"""Gradient checks and the L-BFGS inversion on the 128 x 64 plate (one GPU).

    python -m paper_2501_06748_amd.invert [--nt 400] [--shots 8] [--fd-params 64]
                                          [--full-steps 48] [--iters 10] [--data fem|sbfem]

On the 0.1 x 0.05 m plate of 128 x 64 elements (n_b 16, N_r 32) with
``--shots`` Ricker sources on the top edge, it

1. simulates observed data on a model with two elliptical voids: by default
   (``--data fem``) with the bilinear finite element generator on the
   512 x 256 grid (four times finer per direction), the voids sharp at the
   1e-5 density floor, so that the inversion does not see its own
   discretisation; with ``--data sbfem`` by the scaled boundary model itself
   on smoothed voids at density floor 0.5;
2. evaluates the misfit and its gradient at the homogeneous starting model
   through the autograd Function (sqrt(T) checkpoints, adjoint backward);
3. checks the gradient against central finite differences on
   ``--fd-params`` seeded parameters (h = 1e-6 relative) and along a smooth
   direction (the +-30 % random field minus rho0), against the dot-product
   test along the same direction, and against the full-storage backward (on
   the first ``--full-steps`` steps, since full storage of the plate costs
   about 0.1 GB per shot and step).  With the direct coarse solver (the
   default) every coarse solve is exact up to rounding.  With the iterative
   one (``--coarse-solver 0``) the checks run with solves to 1e-15 relative
   residual (``--check-rtol``): a finite difference of one density among
   four million changes the misfit by about 1e-9 of itself, below what the
   default 1e-13 solves resolve;
4. runs ``--iters`` L-BFGS iterations (memory 10) on the density scaling
   field rho / rho0 within [1e-6, 2], and reports the normalised misfit and
   the correlation of the recovered scaling field with the true one at the
   fine-grid points.

Prints progress lines and, at the end, one JSON object.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import lbfgs, sbfwi_build_mesh, sbfwi_fem_forward
from .autograd import WaveProblem, misfit, simulate


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--nt", type=int, default=400)
    ap.add_argument("--shots", type=int, default=8)
    ap.add_argument("--fd-params", type=int, default=64)
    ap.add_argument("--full-steps", type=int, default=48)
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--check-rtol", type=float, default=1e-15)
    ap.add_argument("--coarse-solver", type=int, default=1)
    ap.add_argument("--data", choices=["fem", "sbfem"], default="fem")
    ap.add_argument("--scheme", type=int, default=0, help="0: the paper's radial finite differences; 1: radial Galerkin")
    ap.add_argument("--phases", default="checks,lbfgs",
                    help="checks (finite differences, dot product, full storage) and/or lbfgs")
    args = ap.parse_args(argv)
    phases = {p.strip() for p in args.phases.split(",") if p.strip()}

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as W

    dev = "cuda"
    wl = W.config_paper(n_steps=args.nt, n_shots=args.shots)
    m = wl.mesh
    mesh = sbfwi_build_mesh(m.node_xy, m.elem_ptr, m.elem_nodes, m.n_r, xi0=wl.xi0)

    def problem(nt, n_ckpt=-1, rtol=None):
        return WaveProblem(mesh=mesh, c=wl.c, dt=wl.dt, rtol=rtol,
                           src=torch.tensor(wl.src_nodes, dtype=torch.int64, device=dev),
                           wavelet=torch.tensor(np.ascontiguousarray(wl.wavelets[:, :nt]), dtype=torch.float64,
                                                device=dev),
                           rec=torch.tensor(wl.rec_nodes, dtype=torch.int64, device=dev),
                           beta=wl.beta, gamma=wl.gamma, n_ckpt=n_ckpt, coarse_solver=args.coarse_solver,
                           scheme=args.scheme)

    prob = problem(args.nt)
    rho0 = float(wl.rho0)
    rho_h = torch.full((m.n_params,), rho0, dtype=torch.float64, device=dev)
    out = {"workload": wl.name, "time_steps": args.nt, "shots": args.shots, "n_params": int(m.n_params),
           "coarse_solver": "direct" if args.coarse_solver == 1 else "bicgstab",
           "scheme": "radial Galerkin" if args.scheme == 1 else "paper finite differences"}

    t0 = time.perf_counter()
    if args.data == "fem":
        g = W.fem_grid(wl)

        def fem_data(name):
            d = torch.empty((wl.n_shots, len(wl.rec_nodes), args.nt), dtype=torch.float64, device=dev)
            sbfwi_fem_forward(g.nx, g.ny, g.lx, g.ly,
                              torch.tensor(W.fem_density(wl, g, name), dtype=torch.float64, device=dev),
                              wl.c, wl.dt, torch.tensor(W.fem_nodes(wl, g, wl.src_nodes), device=dev),
                              prob.wavelet, torch.tensor(W.fem_nodes(wl, g, wl.rec_nodes), device=dev), d)
            return d

        obs = fem_data("voids_data")
        truth = wl.fields["voids_data"](W.fine_point_positions(m)) / wl.rho0
        out["data"] = {"generator": "bilinear FEM", "grid": [g.nx, g.ny], "model": "voids_data"}
    else:
        with torch.no_grad():
            obs = simulate(torch.tensor(wl.models["voids_floor_half"], dtype=torch.float64, device=dev), prob)
        truth = wl.models["voids_floor_half"] / wl.rho0
        out["data"] = {"generator": "scaled boundary model", "model": "voids_floor_half"}
    torch.cuda.synchronize()
    out["data"]["seconds"] = time.perf_counter() - t0
    _log(f"[invert] observed data ({args.data}): {out['data']['seconds']:.2f} s")

    def value_grad(rho, p=prob, d=obs):
        r = rho.detach().clone().requires_grad_(True)
        val = misfit(simulate(r, p), d, wl.dt)
        val.backward()
        return float(val.item()), r.grad.detach()

    def value(rho, p=prob, d=obs):
        with torch.no_grad():
            return float(misfit(simulate(rho, p), d, wl.dt).item())

    t0 = time.perf_counter()
    J0, g0 = value_grad(rho_h)
    torch.cuda.synchronize()
    out["misfit0"] = J0
    out["gradient_eval_s"] = time.perf_counter() - t0
    _log(f"[invert] misfit {J0:.6e}, gradient in {out['gradient_eval_s']:.2f} s")
    if args.data == "fem":
        # discretisation difference alone: both models on the homogeneous plate
        with torch.no_grad():
            Jh = float(misfit(simulate(rho_h, prob), fem_data("homogeneous"), wl.dt).item())
        out["modelling_error_misfit_fraction"] = Jh / J0
        _log(f"[invert] scaled boundary vs finite element misfit on the homogeneous plate: {Jh / J0:.4f} of J0")
    # the checks: with the iterative solver, the same problem with tighter coarse solves
    if args.coarse_solver == 0:
        chk = problem(args.nt, rtol=args.check_rtol)
        Jc, gc = value_grad(rho_h, chk)
        out["check_rtol"] = args.check_rtol
        out["gradient_rel_change_with_rtol"] = float(torch.linalg.norm(gc - g0) / torch.linalg.norm(gc))
    else:
        chk, gc = prob, g0

    if "checks" in phases:
        _checks(args, wl, out, rho_h, rho0, gc, chk, value, value_grad, problem, obs)

    if "lbfgs" in phases:
        _lbfgs(args, out, rho_h, rho0, J0, value_grad, truth)
    print(json.dumps(out))


def _checks(args, wl, out, rho_h, rho0, gc, chk, value, value_grad, problem, obs):
    """Finite differences on seeded parameters and along a smooth direction, the
    dot-product test and the sqrt(T) checkpoints against full storage."""
    dev = rho_h.device
    rng = np.random.default_rng(3 * 1000 + 1)
    gn = gc.cpu().numpy()
    cand = np.flatnonzero(np.abs(gn) >= 1e-2 * np.abs(gn).max())
    picks = rng.choice(cand, size=min(args.fd_params, cand.size), replace=False)
    errs = []
    for i, p in enumerate(picks):
        e = torch.zeros_like(rho_h)
        h = 1e-6 * rho0
        e[p] = h
        fd = (value(rho_h + e, chk) - value(rho_h - e, chk)) / (2 * h)
        errs.append(abs(fd - gn[p]) / abs(gn[p]))
        if (i + 1) % 8 == 0:
            _log(f"[invert] finite differences {i + 1}/{len(picks)}: worst relative error {max(errs):.2e}")
    d = torch.tensor(wl.models["random30"], dtype=torch.float64, device=dev) - rho0
    hd = 1e-6
    fd_dir = (value(rho_h + hd * d, chk) - value(rho_h - hd * d, chk)) / (2 * hd)
    ad_dir = float(torch.dot(gc, d))
    out["fd_single"] = {"params": int(len(picks)), "worst_rel": float(max(errs)), "median_rel": float(np.median(errs))}
    out["fd_direction_rel"] = abs(fd_dir - ad_dir) / abs(ad_dir)
    _log(f"[invert] directional FD relative error {out['fd_direction_rel']:.2e}")

    r = rho_h.clone().requires_grad_(True)
    tr = simulate(r, chk)
    dd = torch.tensor(rng.standard_normal(tuple(tr.shape)), dtype=torch.float64, device=dev)
    tr.backward(dd)
    rhs = float(torch.dot(d, r.grad))
    hdt = 1e-5
    with torch.no_grad():
        jd = (simulate(rho_h + hdt * d, chk) - simulate(rho_h - hdt * d, chk)) / (2 * hdt)
    lhs = float((jd * dd).sum())
    out["dot_product_rel"] = abs(lhs - rhs) / abs(rhs)
    _log(f"[invert] dot-product test relative error {out['dot_product_rel']:.2e}")

    nf = min(args.full_steps, args.nt)
    obs_f = obs[:, :, :nf].contiguous()
    _, g_ck = value_grad(rho_h, problem(nf, -1), obs_f)
    _, g_full = value_grad(rho_h, problem(nf, nf), obs_f)
    out["full_storage"] = {"steps": nf, "rel_l2": float(torch.linalg.norm(g_ck - g_full) / torch.linalg.norm(g_full))}
    _log(f"[invert] sqrt(T) vs full storage over {nf} steps: {out['full_storage']['rel_l2']:.2e}")


def _lbfgs(args, out, rho_h, rho0, J0, value_grad, truth):
    """L-BFGS iterations on the density scaling field within [1e-6, 2]."""

    def fg(mv):
        v, g = value_grad(rho0 * mv)
        return v / J0, g * (rho0 / J0)

    def cb(it, x, f, g):
        _log(f"[invert] L-BFGS iteration {it + 1}: normalised misfit {f:.5f}")

    t0 = time.perf_counter()
    res = lbfgs.minimize_box(fg, torch.ones_like(rho_h), 1e-6, 2.0, iters=args.iters, memory=10,
                             first_step=0.05, callback=cb)
    torch.cuda.synchronize()
    out["lbfgs"] = {"iterations": len(res.history) - 1, "normalised_misfit": res.history,
                    "evaluations": res.evaluations, "rejected": res.rejected,
                    "seconds": time.perf_counter() - t0,
                    "scaling_min": float(res.x.min()), "scaling_max": float(res.x.max()),
                    "image_correlation": float(np.corrcoef(res.x.cpu().numpy(), truth)[0, 1])}


if __name__ == "__main__":
    main()

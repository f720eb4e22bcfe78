"""Epoch times on the workload shape of the paper's timing tables (one GPU).

    python -m paper_2501_06748_amd.tables [--cells 1000 2000 4000 8000] [--intervals 5 7]
                                          [--schemes 0 1] [--reps 5]

For every centroidal Voronoi mesh (cells), radial interval count and radial
scheme it times one inversion epoch as the paper counts it: the element
factorisation of the model, the forward runs of both sources (200 steps,
sqrt(T) checkpoints) and the adjoint runs with the exact gradient, at the
homogeneous model against data from the model with a central hole.  The
low-frequency expansion path (scheme 2, the paper's benchmark column) is
timed once per mesh, with its element matrices condensed from 33 radial
levels, the forward runs keeping every nodal velocity and the paper's
truncated kernel as the gradient.  Each
line reports the median over ``--reps`` epochs after one warm-up, the rate in
element x radial-level x step x shot units per second, and the paper's CPU
seconds per epoch for the same mesh size and interval count (12 threads of a
laptop CPU; context only: the paper's plate, meshes and data are not
available, the plate here is 0.1 x 0.05 m).

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

from . import (GRAD_EXACT, GRAD_PAPER_KERNEL, LAUNCH_GRAPHS, sbfwi_build_mesh, sbfwi_factor_elements, sbfwi_forward,
               sbfwi_gradient, sbfwi_set_launch)

# seconds per epoch in the paper's timing table of the hole specimen (12 CPU threads)
PAPER_CPU_S = {(1000, 5): 0.95, (1000, 7): 1.32, (2000, 5): 2.39, (2000, 7): 3.21,
               (4000, 5): 5.49, (4000, 7): 6.82, (8000, 5): 11.19, (8000, 7): 13.92,
               (1000, "LFE"): 0.23, (2000, "LFE"): 0.46, (4000, "LFE"): 1.27, (8000, "LFE"): 2.70}
LFE_LEVELS = 33


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--cells", type=int, nargs="+", default=[1000, 2000, 4000, 8000])
    ap.add_argument("--intervals", type=int, nargs="+", default=[5, 7])
    ap.add_argument("--schemes", type=int, nargs="+", default=[0, 1, 2])
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--graphs", type=int, default=0, help="1: forward steps replayed from HIP graphs")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as W

    dev = "cuda"
    rows = []
    for n_cells in args.cells:
        t0 = time.perf_counter()
        base = W.config_cvt(n_cells, args.intervals[0])
        _log(f"[tables] mesh of {n_cells} cells generated in {time.perf_counter() - t0:.1f} s")
        runs = [(iv, sc) for iv in args.intervals for sc in args.schemes if sc != 2]
        if 2 in args.schemes:
            runs.append((LFE_LEVELS - 1, 2))
        for iv in sorted({r[0] for r in runs}, key=lambda v: (v == LFE_LEVELS - 1, v)):
            wl = base if iv == args.intervals[0] else W.config_cvt(n_cells, iv, mesh=base.mesh)
            m = wl.mesh
            mesh = sbfwi_build_mesh(m.node_xy, m.elem_ptr, m.elem_nodes, m.n_r, xi0=wl.xi0)
            src = torch.tensor(wl.src_nodes, device=dev)
            wav = torch.tensor(wl.wavelets, dtype=torch.float64, device=dev)
            rec = torch.tensor(wl.rec_nodes, device=dev)
            S, R, N = wl.n_shots, len(wl.rec_nodes), wl.n_steps
            rho_h = torch.tensor(wl.models["homogeneous"], dtype=torch.float64, device=dev)
            rho_d = torch.tensor(wl.models["hole_floor_half"], dtype=torch.float64, device=dev)
            units = int(m.n_r.astype(np.int64).sum()) * N * S
            for scheme in [sc for (v, sc) in runs if v == iv]:
                obs = torch.zeros((S, R, N), dtype=torch.float64, device=dev)
                fd = sbfwi_factor_elements(mesh, rho_d, wl.c, wl.dt, wl.beta, wl.gamma, scheme=scheme,
                                           coarse_solver=1)
                sbfwi_forward(fd, src, wav, rec, obs)
                fd.close()
                tr = torch.zeros_like(obs)
                mis = torch.zeros(1, dtype=torch.float64, device=dev)
                grad = torch.zeros(int(m.n_params), dtype=torch.float64, device=dev)

                mode = GRAD_PAPER_KERNEL if scheme == 2 else GRAD_EXACT

                def epoch():
                    f = sbfwi_factor_elements(mesh, rho_h, wl.c, wl.dt, wl.beta, wl.gamma, scheme=scheme,
                                              coarse_solver=1)
                    if args.graphs:
                        sbfwi_set_launch(f, LAUNCH_GRAPHS, 1)
                    ck = sbfwi_forward(f, src, wav, rec, tr, n_ckpt=-1)
                    sbfwi_gradient(f, ck, obs, tr, mode, mis, grad)
                    ck.close()
                    f.close()

                epoch()
                torch.cuda.synchronize()
                times = []
                for _ in range(args.reps):
                    t = time.perf_counter()
                    epoch()
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t)
                sec = float(np.median(times))
                name = ["paper FD", "radial Galerkin", "LFE"][scheme]
                key = (n_cells, "LFE" if scheme == 2 else iv)
                row = {"cells": n_cells, "intervals": None if scheme == 2 else iv, "scheme": name,
                       "n_b_max": int(m.n_b().max()), "nodes": int(m.n_nodes), "receivers": R,
                       "seconds_per_epoch": sec, "units_per_s": None if scheme == 2 else units / sec,
                       "finite": bool(torch.isfinite(grad).all().item()),
                       "gradient": "paper kernel" if scheme == 2 else "exact", "graphs": bool(args.graphs),
                       "paper_cpu_seconds_per_epoch": PAPER_CPU_S.get(key)}
                rows.append(row)
                _log(f"[tables] {n_cells} cells, {row['intervals']} intervals, {name}: {sec * 1e3:.1f} ms per epoch, "
                     f"{row['units_per_s']} units/s (paper CPU: {row['paper_cpu_seconds_per_epoch']} s)")
            mesh.close()
    print(json.dumps({"workload": "cvt timing-table shape: 0.1 x 0.05 m, c 6000, dt 0.2 us, 200 steps, 2 shots",
                      "rows": rows}))


if __name__ == "__main__":
    main()

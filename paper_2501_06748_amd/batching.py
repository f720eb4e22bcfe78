"""Batched multi-shot gradient evaluation on the ragged quadtree plate, against
the plain per-shot path (one GPU).

    python -m paper_2501_06748_amd.batching [--nt 4000] [--shots 16]

Workload: the 0.1 x 0.05 m plate as a quadtree refined from level 4 to level
8 around three seeded voids (about 6200 elements, n_b 8 .. 14, N_r 16 .. 64),
16 Ricker shots on the top edge, 32 receivers, 4000 steps.  Both paths
evaluate the misfit and its exact gradient at the homogeneous model against
data of the three-void model (simulated first, untimed):

* plain: one run per shot (1 shot per launch, default launch shapes,
  ordinary launches), gradients summed on the device;
* batched: all shots in one run, with the launch plan chosen by the
  autotuner and the forward steps replayed from HIP graphs.

Reports element x level x step x shot units per second of both, the speedup,
the autotuned plan and the agreement of the two gradients.  Prints progress
lines and one JSON object.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import (GRAD_EXACT, LAUNCH_GRAPHS, sbfwi_autotune, sbfwi_build_mesh, sbfwi_factor_elements,
               sbfwi_forward, sbfwi_gradient, sbfwi_mesh_info, sbfwi_set_launch, sbfwi_solver_stats)


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--nt", type=int, default=4000)
    ap.add_argument("--shots", type=int, default=16)
    ap.add_argument("--coarse-solver", type=int, default=1)
    ap.add_argument("--skip-plain", action="store_true", help="run the batched path only (profiling)")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as W

    dev = "cuda"
    wl = W.config_quadtree(n_steps=args.nt, n_shots=args.shots)
    m = wl.mesh
    mesh = sbfwi_build_mesh(m.node_xy, m.elem_ptr, m.elem_nodes, m.n_r, xi0=wl.xi0)
    info = sbfwi_mesh_info(mesh)
    S, N, R = wl.n_shots, wl.n_steps, len(wl.rec_nodes)
    src = torch.tensor(wl.src_nodes, dtype=torch.int64, device=dev)
    wav = torch.tensor(wl.wavelets, dtype=torch.float64, device=dev)
    rec = torch.tensor(wl.rec_nodes, dtype=torch.int64, device=dev)
    rho0 = torch.tensor(wl.models["homogeneous"], dtype=torch.float64, device=dev)
    rho_t = torch.tensor(wl.models["voids_floor_half"], dtype=torch.float64, device=dev)
    units = int(m.n_r.astype(np.int64).sum()) * N * S
    out = {"workload": wl.name, "elements": int(m.n_elem), "nodes": int(m.n_nodes),
           "n_b": sorted(set(int(v) for v in m.n_b())), "n_r": [int(m.n_r.min()), int(m.n_r.max())],
           "time_steps": N, "shots": S, "units": units}

    def factor(rho):
        return sbfwi_factor_elements(mesh, rho, wl.c, wl.dt, wl.beta, wl.gamma, coarse_solver=args.coarse_solver)

    ft = factor(rho_t)
    observed = torch.zeros((S, R, N), dtype=torch.float64, device=dev)
    sbfwi_set_launch(ft, LAUNCH_GRAPHS, 1)
    sbfwi_forward(ft, src, wav, rec, observed)
    ft.close()
    torch.cuda.synchronize()
    _log(f"[batching] observed data: {wl.name}, {m.n_elem} elements, {S} shots, {N} steps")

    # plain path: one run per shot
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f = factor(rho0)
    g_plain = torch.zeros(info["n_params"], dtype=torch.float64, device=dev)
    mis_plain = 0.0
    gs = torch.zeros_like(g_plain)
    mis = torch.zeros(1, dtype=torch.float64, device=dev)
    for s in range(0 if args.skip_plain else S):
        tr = torch.zeros((1, R, N), dtype=torch.float64, device=dev)
        ck = sbfwi_forward(f, src[s:s + 1], wav[s:s + 1].contiguous(), rec, tr, n_ckpt=-1)
        sbfwi_gradient(f, ck, observed[s:s + 1].contiguous(), tr, GRAD_EXACT, mis, gs)
        g_plain += gs
        mis_plain += float(mis.item())
        ck.close()
        _log(f"[batching] plain path: shot {s + 1}/{S} done")
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    f.close()

    # batched path: all shots, autotuned plan, graph replay
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f = factor(rho0)
    t_tune = time.perf_counter()
    plan = sbfwi_autotune(f, S)
    t_tune = time.perf_counter() - t_tune
    sbfwi_set_launch(f, LAUNCH_GRAPHS, 1)
    tr = torch.zeros((S, R, N), dtype=torch.float64, device=dev)
    g_b = torch.zeros_like(g_plain)
    ck = sbfwi_forward(f, src, wav, rec, tr, n_ckpt=-1)
    sbfwi_gradient(f, ck, observed, tr, GRAD_EXACT, mis, g_b)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    stats = sbfwi_solver_stats(f)
    ck.close()
    f.close()
    _log(f"[batching] batched path done in {t_batch:.2f} s (plain {t_plain:.2f} s)")

    # HBM roofline of the whole batched evaluation on the method's byte model: per element,
    # level, time step and shot 48 n_b^2 / S + 192 n_b bytes (forward, checkpoint recompute,
    # adjoint and gradient; S shots share each streamed factor block), with S the run's shot
    # count (ideal sharing) and with S the autotuned recover shots per block of each n_b class
    nb = m.n_b().astype(np.float64)
    nr = m.n_r.astype(np.float64)
    cls = np.where(nb <= 8, 0, np.where(nb <= 16, 1, 2))
    s_blk = np.asarray([max(plan["recover"]["shots_per_block"][c], 1) for c in cls], dtype=np.float64)
    eval_ideal = float((nr * N * S * (48 * nb * nb / S + 192 * nb)).sum())
    eval_plan = float((nr * N * S * (48 * nb * nb / s_blk + 192 * nb)).sum())
    out["batched"] = {"seconds": t_batch, "units_per_s": units / t_batch, "misfit": float(mis.item()),
                      "autotune_seconds": t_tune, "plan": plan, "coarse_solver": stats,
                      "roofline": {"bound": "hbm", "peak_GBs": 8000.0,
                                   "algorithmic_bytes_shared_by_all_shots": eval_ideal,
                                   "frac": eval_ideal / t_batch / 8e12,
                                   "algorithmic_bytes_at_plan_shots_per_block": eval_plan,
                                   "frac_at_plan": eval_plan / t_batch / 8e12}}
    if not args.skip_plain:
        out["plain"] = {"seconds": t_plain, "units_per_s": units / t_plain, "misfit": mis_plain}
        out["speedup"] = t_plain / t_batch
        out["gradient_rel_l2"] = float(torch.linalg.norm(g_b - g_plain) / torch.linalg.norm(g_plain))
    print(json.dumps(out))


if __name__ == "__main__":
    main()

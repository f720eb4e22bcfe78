#!/usr/bin/env python3
"""Throughput of the SBFEM radial-condensation FWI hot path on one MI355X.

One *step* is one full gradient evaluation of the inversion on the paper-size
synthetic plate: factorisation of every element (coefficient matrices,
radial rows, block elimination, coarse assembly), the forward run of all
shots with sqrt(T) checkpoints (condense, coarse solve, recover, Newmark per
time step), the misfit, and the exact adjoint run with segment recompute and
the zero-lag gradient correlation.  The metric counts element x radial level
x time step x shot units of forward + adjoint per second.

Workload (synthetic, seeded): 0.1 x 0.05 m plate, 128 x 64 square elements,
16 boundary nodes and 32 radial levels per element, c = 3000 m/s,
rho0 = 2700 kg/m^3, dt = 2e-8 s, 4000 steps, 4 Ricker shots (500 kHz) and 32
receivers on the top edge.  The gradient is evaluated at the homogeneous
starting model against observed data generated before the timed region by
the bilinear finite element model on a 512 x 256 grid (four times finer per
direction) with two sharp elliptical voids at the 1e-5 density floor; that
generator's time-step kernel is timed and reported on its own.

    python bench.py [--steps K] [--warmup W] [--nt N_t] [--shots S]

Prints one JSON line.  --gpus above 1 is not supported (one GPU only).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def kernel_bytes(mesh, NS, nnz):
    """Algorithmic HBM bytes per launch of each kernel: every input and output of
    the kernel read or written once (FP64 values, int32 column indices).  Sweep
    kernels: per element with n interior levels, nb boundary nodes, NS shots.
    Coarse-solve kernels: per active launch (one BiCGStab iteration), K_g with
    nnz entries on n nodes."""
    nb = mesh.n_b().astype("int64")
    n = mesh.n_r.astype("int64") - 1
    blk = n * nb * nb + nb * nb                   # stored pivot inverses + one per-element dense block
    band = lambda levels: 3 * nb * levels         # cyclic tridiagonal blocks
    out = {
        # reads phi~^-1 (n blocks), G, bands P (n+1), theta (n+1); the interior w (n levels) and
        # the nodal w on the loop; writes q (n levels), y_n and f_hat on the loop
        "condense": blk + band(n + 1) + band(n + 2) + NS * (n * nb + nb + n * nb + 2 * nb),
        # reads phi~^-1, psi~_0, bands psi (n-1); q, r, w, u_n; writes r, w
        "recover": blk + band(n - 1) + NS * (3 * n * nb + nb + 2 * n * nb),
        # the checkpoint recompute's variant also stores the unknowns with ghosts (n+3 levels)
        # and the accelerations (n+1 levels) for the adjoint
        "recover_store": blk + band(n - 1) + NS * (3 * n * nb + nb + 2 * n * nb)
                         + NS * ((n + 3) + (n + 1)) * nb,
        # reads phi~^-1, psi~_0, the density rows (n+1) and the rows' coefficients (27 per node)
        # instead of the bands psi, psi_{n-1}; seeds u~ (n); writes z (n) and the coupling (1)
        "adj_condense": blk + (n + 1) * nb + 27 * nb + band(1) + NS * (n * nb + n * nb + nb),
        # reads G, phi~^-1, the density rows and coefficients instead of theta, P, theta_-1^-1,
        # P_n, theta_0; lambda_B, z, seeds v-bar, a-bar (2 n); writes seeds u~, v-bar, a-bar (3 n),
        # P_n^T lambda_n, adjoint rows (n+3)
        "adj_recover": blk + 2 * nb * nb + (n + 1) * nb + 27 * nb + band(2) +
                       NS * (nb + n * nb + 2 * n * nb + 3 * n * nb + nb + (n + 3) * nb),
        # reads unknowns and adjoint rows (n+3 levels each), accelerations (n+1), alpha; grad RMW
        "grad_exact": 32 * nb + 2 * (n + 1) * nb + NS * (2 * (n + 3) * nb + (n + 1) * nb),
    }
    # joint sweeps: the condense of the next step takes its w (u~) from the recover sweep in
    # LDS; the joint transposed sweep does not write u~ either
    out["joint"] = out["recover"] + out["condense"] - NS * n * nb
    out["joint_store"] = out["recover_store"] + out["condense"] - NS * n * nb
    out["adj_joint"] = out["adj_recover"] + out["adj_condense"] - 2 * NS * n * nb
    res = {k: int(8 * v.sum()) for k, v in out.items()}
    nn = int(mesh.n_nodes)
    res["solve_v"] = 12 * nnz + 8 * nn + 8 * NS * nn * 7      # K, D^-1; phat, r, rhat, w in; v, s, shat out
    res["solve_t"] = 12 * nnz + 8 * NS * nn * 3               # K; shat, s in; t out
    res["solve_x"] = 8 * nn + 8 * NS * nn * 11                # D^-1; x, phat, p r/w, shat, s, t, v, w in; r out
    return res


def method_bytes(mesh, NS):
    """Algorithmic HBM bytes per launch of the HBM-bound sweeps from the method's
    per-unit byte model (a unit = one element, radial level and shot of one time
    step; 8-byte words): every pass over an element streams two dense n_b x n_b
    blocks per level, shared by the S = NS shots of the launch, plus the level
    state of each shot -- forward 16 n_b^2/S + 48 n_b (u, v, a read and
    written), checkpoint recompute 16 n_b^2/S + 64 n_b (plus the stores the
    adjoint needs), adjoint and gradient 16 n_b^2/S + 80 n_b (adjoint state read
    and written, forward unknowns read, gradient).  A sweep over half a step (a
    condense or a recover on its own, each adjoint sweep) takes one block and
    half the state; the joint sweep (recover of a step with the condense of the
    next) the whole step, and so does the joint transposed sweep (two blocks and
    the adjoint state's 48 n_b); the gradient contraction the rest of the
    adjoint's 80 n_b: 32 n_b.  Returns bytes per launch and per unit of the whole
    evaluation (fwd + recompute + adjoint + gradient = 48 n_b^2/S + 192 n_b).
    The model counts the state as u, v, a; the sweeps keep two combinations of
    them (r, w), so they move fewer state bytes than it counts, and more for
    the banded rows and the swept sources it leaves out (kernel_bytes)."""
    nb = mesh.n_b().astype("float64")
    units = mesh.n_r.astype("float64") * NS            # units of one launch, per element
    blk = nb * nb / NS
    per_unit = {"joint": 16 * blk + 48 * nb, "joint_store": 16 * blk + 64 * nb, "adj_joint": 16 * blk + 48 * nb,
                "condense": 8 * blk + 24 * nb, "recover": 8 * blk + 24 * nb,
                "recover_store": 8 * blk + 32 * nb,
                "adj_condense": 8 * blk + 24 * nb, "adj_recover": 8 * blk + 24 * nb,
                "grad_exact": 32 * nb}
    per_launch = {k: float((units * v).sum()) for k, v in per_unit.items()}
    evaluation_per_step = float((units * (48 * blk + 192 * nb)).sum())
    return per_launch, evaluation_per_step


# kernel instances as rocprofv3 names them (uniform 16-node elements, 4 shots per block)
ROCPROF_NAME = {"joint": "joint_kernel<16, 4, false>", "joint_store": "joint_kernel<16, 4, true>",
                "condense": "condense_kernel<16, 4>", "recover": "recover_kernel<16, 4, false>",
                "recover_store": "recover_kernel<16, 4, true>", "adj_joint": "adj_joint_kernel<16, 4, true>",
                "adj_condense": "adj_condense_kernel<16, 4, true>",
                "adj_recover": "adj_recover_kernel<16, 4, true>", "grad_exact": "grad_exact_kernel<16, 4, false>"}


def fem_bytes(nx, ny, S, R):
    """Algorithmic HBM bytes per launch of the finite element time step: u_k read,
    u_{k-1} read and u_{k+1} written per node and shot, the lumped inverse mass per
    node and the padded element coefficients once, one trace sample per receiver."""
    nn = (nx + 1) * (ny + 1)
    return 8 * (3 * S * nn + nn + (nx + 2) * (ny + 2) + S * R)


def src_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {"solve_v": ["paper_2501_06748_amd/csrc/coarse.hip"],
                  "solve_t": ["paper_2501_06748_amd/csrc/coarse.hip"],
                  "solve_x": ["paper_2501_06748_amd/csrc/coarse.hip"],
                  "condense": ["paper_2501_06748_amd/csrc/step.hip"],
                  "recover": ["paper_2501_06748_amd/csrc/step.hip"],
                  "recover_store": ["paper_2501_06748_amd/csrc/step.hip"],
                  "joint": ["paper_2501_06748_amd/csrc/step.hip"],
                  "joint_store": ["paper_2501_06748_amd/csrc/step.hip"],
                  "adj_condense": ["paper_2501_06748_amd/csrc/adjoint.hip"],
                  "adj_recover": ["paper_2501_06748_amd/csrc/adjoint.hip"],
                  "adj_joint": ["paper_2501_06748_amd/csrc/adjoint.hip"],
                  "grad_exact": ["paper_2501_06748_amd/csrc/adjoint.hip"],
                  "coarse_solve": ["paper_2501_06748_amd/csrc/coarse.hip"],
                  "fem_step": ["paper_2501_06748_amd/csrc/fem.hip"]}


def measured_traffic(kernel, wl_name):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        tab = json.load(fh)
    ent = tab.get(f"{kernel}@{wl_name}")
    if not ent or ent.get("source_sha") != src_hash(KERNEL_SOURCES.get(kernel, [])):
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(n_steps_target, short=10, long=1000):
    """The oracle, as it stands, on a bounded sample with the benchmark's element
    type: an 8 x 4 patch of the same elements (n_b 16, N_r 32, dt 2e-8), one
    shot, factor + forward + exact adjoint gradient, timed at two step counts;
    the time is fitted as a + b N_t and the rate reported for the workload's N_t
    (the gradient contraction is a per-parameter cost independent of N_t)."""
    import numpy as np
    import workloads as W
    from oracle import adjoint as oadj
    from oracle import stepper as ostp
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    le = 0.1 / 128
    mesh = W.uniform_rect_mesh(8 * le, 4 * le, 8, 4, segs=4, n_r=32)
    dt = 2e-8
    src = np.asarray([W.nearest_top_node(mesh, 4 * le)], dtype=np.int64)
    rec = W.top_edge_nodes(mesh)[::2]
    times = {}
    cpu_s = wall_s = 0.0
    for nt in (short, long):
        wav = W.ricker(nt, dt, 5e5, t0=20 * dt)[None]
        t0, c0 = time.perf_counter(), time.process_time()
        model = ostp.Model(mesh, W.homogeneous(mesh), 3000.0, dt)
        oadj.exact_gradient(model, src, wav, rec, np.zeros((1, len(rec), nt)), nt)
        times[nt] = time.perf_counter() - t0
        cpu_s += time.process_time() - c0
        wall_s += times[nt]
    # threads actually used: CPU time of all the process's threads over wall time
    # (the per-element loops are Python; only the library calls inside them fan out)
    used = cpu_s / max(wall_s, 1e-9)
    b = max((times[long] - times[short]) / (long - short), 1e-12)
    a = max(times[short] - b * short, 0.0)
    per_step_units = int(mesh.n_r.sum())
    rate = per_step_units * n_steps_target / (a + b * n_steps_target)
    return {"value": rate, "unit": "element*radial*steps/s", "cores": max(1, int(round(used))), "kind": "oracle",
            "sample": f"oracle factor+forward+exact gradient on an 8x4 patch of the benchmark's elements "
                      f"(n_b 16, N_r 32, dt 2e-8, 1 shot): {times[short]:.2f} s at {short} steps, "
                      f"{times[long]:.2f} s at {long} steps; fitted a + b*N_t with a = {a:.2f} s, "
                      f"b = {b * 1e3:.2f} ms/step, rate extrapolated to N_t = {n_steps_target}; "
                      f"CPU time / wall time {used:.2f} (BLAS pool of {threads} threads)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nt", type=int, default=4000, help="time steps of the workload")
    ap.add_argument("--shots", type=int, default=4)
    ap.add_argument("--solver-iters", type=int, default=0, help="BiCGStab iterations enqueued per solve (0 = default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--coarse-solver", type=int, default=1,
                    help="0: BiCGStab every step; 1: nested-dissection LU factored once per model (default)")
    ap.add_argument("--scheme", type=int, default=0,
                    help="radial scheme: 0 the paper's finite differences (default), 1 radial Galerkin")
    ap.add_argument("--graphs", type=int, default=0,
                    help="1: forward steps replayed from HIP graphs (their launches are then not seen by the "
                         "live kernel timing)")
    ap.add_argument("--overlap", type=int, default=1,
                    help="1: backward pass overlaps the segment recompute with the adjoint steps (default)")
    ap.add_argument("--autotune", type=int, default=0,
                    help="1: sweep launch plan autotuned once per mesh and shot count, before the timed region")
    ap.add_argument("--tail-gib", type=float, default=-1.0,
                    help="tail store of the forward run in GiB (the fields of its last checkpoint segments, "
                         "so that the backward pass recomputes only the segments before them); -1 = the device "
                         "memory left free by everything else the evaluation needs, less 8 GiB")
    ap.add_argument("--subtree-cut", type=int, default=0,
                    help="direct solver: subtree launches rooted at the shallowest dissection level with at "
                         "least this many supernodes (0 = the library's default, 512)")
    ap.add_argument("--counter-probe", type=int, default=0, metavar="K",
                    help="run K gradient steps of the workload (--nt steps each) plus a 1 GiB device copy, "
                         "print nothing else and exit: the program profiled by hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(shots would shard across GPUs, with one all-reduce of the gradient; not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    import paper_2501_06748_amd as sb

    dev = torch.device("cuda:0")
    wl = W.config_paper(n_steps=args.nt, n_shots=args.shots)
    mesh = wl.mesh
    mh = sb.sbfwi_build_mesh(mesh.node_xy, mesh.elem_ptr, mesh.elem_nodes, mesh.n_r, xi0=wl.xi0)
    info = sb.sbfwi_mesh_info(mh)
    rho0 = torch.tensor(wl.models["homogeneous"], dtype=torch.float64, device=dev)
    rho_true = torch.tensor(wl.models["voids_floor_half"], dtype=torch.float64, device=dev)
    src = torch.tensor(wl.src_nodes, dtype=torch.int64, device=dev)
    wav = torch.tensor(wl.wavelets, dtype=torch.float64, device=dev)
    rec = torch.tensor(wl.rec_nodes, dtype=torch.int64, device=dev)
    S, R, N = wl.n_shots, len(wl.rec_nodes), wl.n_steps
    traces = torch.zeros((S, R, N), dtype=torch.float64, device=dev)
    observed = torch.zeros((S, R, N), dtype=torch.float64, device=dev)
    misfit = torch.zeros(1, dtype=torch.float64, device=dev)
    grad = torch.zeros(info["n_params"], dtype=torch.float64, device=dev)

    plan = None

    overlap = args.overlap
    # tail store budget: what the device has free beyond the evaluation's own footprint
    if args.tail_gib >= 0:
        tail_kib = int(args.tail_gib * (1 << 20))
    else:
        pb = sb.sbfwi_plan_bytes(mh, S, N, -1)
        need = pb["factors"] + pb["checkpoints"] + max(pb["forward_work"], pb["backward_work"])
        free, _ = torch.cuda.mem_get_info()
        tail_kib = max(0, (free - need - (8 << 30)) >> 10)
    tail_kib = min(tail_kib, (1 << 31) - 1)
    tail_steps = {"steps": 0}

    # observed data: bilinear finite elements on the data grid (sharp voids at the density floor)
    fg = W.fem_grid(wl)
    f_rho = torch.tensor(W.fem_density(wl, fg, "voids_data"), dtype=torch.float64, device=dev)
    f_src = torch.tensor(W.fem_nodes(wl, fg, wl.src_nodes), device=dev)
    f_rec = torch.tensor(W.fem_nodes(wl, fg, wl.rec_nodes), device=dev)

    def fem_data():
        sb.sbfwi_fem_forward(fg.nx, fg.ny, fg.lx, fg.ly, f_rho, wl.c, wl.dt, f_src, wav, f_rec, observed)

    def factor(rho):
        f = sb.sbfwi_factor_elements(mh, rho, wl.c, wl.dt, wl.beta, wl.gamma, scheme=args.scheme,
                                     coarse_solver=args.coarse_solver)
        if args.solver_iters:
            sb.sbfwi_set_launch(f, 0, args.solver_iters)
        if args.graphs:
            sb.sbfwi_set_launch(f, sb.LAUNCH_GRAPHS, 1)
        sb.sbfwi_set_launch(f, 3, overlap)
        sb.sbfwi_set_launch(f, sb.LAUNCH_TAIL_STORE_KIB, tail_kib)
        if args.subtree_cut:
            sb.sbfwi_set_launch(f, sb.LAUNCH_SUBTREE_CUT, args.subtree_cut)
        if plan is not None:
            sb.apply_plan(f, plan)
        return f

    if args.counter_probe:
        fem_data()
        for _ in range(args.counter_probe):
            f = factor(rho0)
            ck = sb.sbfwi_forward(f, src, wav, rec, traces, n_ckpt=-1)
            sb.sbfwi_gradient(f, ck, traces, traces, sb.GRAD_EXACT, misfit, grad)
            ck.close()
            f.close()
        # reference copy of known size for scaling the counters: 1 GiB read + 1 GiB written
        xa = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        ya = torch.empty_like(xa)
        ya.copy_(xa)
        torch.cuda.synchronize()
        mh.close()
        sb.sbfwi_finalize()
        print("[bench] counter probe done", file=sys.stderr, flush=True)
        return

    # observed data and the launch plan (outside the timed region); the data generator is run
    # twice (the first call pays for module loading) and its time step timed by events
    fem_data()
    torch.cuda.synchronize()
    sb.sbfwi_profile(["fem_step"])
    t_d = time.perf_counter()
    fem_data()
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t_d
    fem_prof = sb.sbfwi_profile_read(reset=True).get("fem_step", {"launches": 0, "ms": 0.0})
    sb.sbfwi_profile(0)
    fem_avg = fem_prof["ms"] / 1e3 / max(fem_prof["launches"], 1)
    fem_b = fem_bytes(fg.nx, fg.ny, S, R)
    fem_gbs = fem_b / max(fem_avg, 1e-12) / 1e9
    fem_out = {"generator": "bilinear FEM, lumped mass, central differences", "grid": [fg.nx, fg.ny],
               "model": "voids_data (floor 1e-5)", "seconds": round(t_data, 4),
               "node_steps_per_s": fg.n_nodes * S * (N - 1) / t_data,
               "fem_step": {"launches": fem_prof["launches"], "avg_us": round(fem_avg * 1e6, 2),
                            "algorithmic_bytes_per_launch": fem_b, "GB/s": round(fem_gbs, 1),
                            "frac_hbm_peak": round(fem_gbs / HBM_PEAK_GBS, 3),
                            "traffic": measured_traffic("fem_step", f"paper-{fg.nx}x{fg.ny}-{S}shots")}}
    if args.autotune:
        ft = factor(rho_true)
        plan = sb.sbfwi_autotune(ft, S)
        ft.close()
    torch.cuda.synchronize()
    print(f"[bench] observed data generated ({wl.name}, {S} shots, {N} steps, FEM {fg.nx}x{fg.ny}: "
          f"{t_data:.3f} s)", file=sys.stderr, flush=True)

    def step(prof_fwd=None, prof_bwd=None):
        f = factor(rho0)
        if prof_fwd is not None:
            sb.sbfwi_profile(prof_fwd)
        ck = sb.sbfwi_forward(f, src, wav, rec, traces, n_ckpt=-1)
        if prof_bwd is not None:
            sb.sbfwi_profile(prof_bwd)
        sb.sbfwi_gradient(f, ck, observed, traces, sb.GRAD_EXACT, misfit, grad)
        stats = sb.sbfwi_solver_stats(f)
        tail_steps["steps"] = sb.sbfwi_ckpt_info(ck)["tail_steps"]
        ck.close()
        f.close()
        return stats

    # kernel census (untimed, before the warmup): one gradient evaluation with the backward pass
    # on one stream, so that every kernel runs alone, each kernel kind timed by events
    overlap = 0
    torch.cuda.synchronize()
    t_f = time.perf_counter()
    factor(rho0).close()   # the whole factorisation of a model (element factors, coarse assembly, coarse LU)
    t_factor = time.perf_counter() - t_f
    sb.sbfwi_profile([k for k in sb.PROFILE_KERNELS if not k.startswith("solve_")])
    step()
    torch.cuda.synchronize()
    census = sb.sbfwi_profile_read(reset=True)
    sb.sbfwi_profile(0)
    overlap = args.overlap
    # warmup: every kernel id except the coarse solve as a whole (its kernels are timed one by one)
    warm_ids = [k for k in sb.PROFILE_KERNELS if k != "coarse_solve"]
    sb.sbfwi_profile(warm_ids)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    warm = sb.sbfwi_profile_read(reset=True)
    print(f"[bench] warmup done: {json.dumps({k: round(v['ms'], 1) for k, v in warm.items()})}", file=sys.stderr,
          flush=True)
    # The dominant kernel: the HBM-bound sweep kind (one kernel instance on this mesh) with the
    # largest total time in the census.  Its launches are timed live by events over the timed
    # region; in the overlapped backward pass launches share the device, and their durations
    # (live and under rocprofv3 alike) include that sharing.
    sweep_kinds = list(ROCPROF_NAME)
    tot = lambda k: census.get(k, {}).get("ms", 0.0)
    dominant = max(sweep_kinds, key=tot)
    # timed region: events around the dominant kernel's launches only
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for _ in range(args.steps):
        stats = step([dominant], [dominant])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    live = sb.sbfwi_profile_read(reset=True)
    print(f"[bench] timed {args.steps} step(s) in {el:.3f} s", file=sys.stderr, flush=True)
    sb.sbfwi_profile(0)

    units = int(mesh.n_r.astype(np.int64).sum()) * N * S
    value = units * args.steps / el
    kb = kernel_bytes(mesh, S, info["nnz"])
    mb, eval_bytes_per_step = method_bytes(mesh, S)
    d_launches = live.get(dominant, {}).get("launches", 0)
    d_ms = live.get(dominant, {}).get("ms", 0.0)
    avg_s = d_ms / 1e3 / max(d_launches, 1)
    achieved = mb[dominant] / max(avg_s, 1e-12) / 1e9
    alone = census.get(dominant, {"launches": 0, "ms": 0.0})
    alone_s = alone["ms"] / 1e3 / max(alone["launches"], 1)
    # every sweep kind alone (census), against the method's bytes and against the builder's
    # own every-input-and-output model (which also counts the q round trip and the band rows)
    sweeps = {}
    for k in sweep_kinds:
        c = census.get(k)
        if not c or c["launches"] == 0:
            continue
        a_s = c["ms"] / 1e3 / c["launches"]
        sweeps[k] = {"launches": c["launches"], "avg_us_alone": round(a_s * 1e6, 2),
                     "method_bytes_per_launch": int(mb[k]),
                     "frac": round(mb[k] / a_s / 1e9 / HBM_PEAK_GBS, 4),
                     "model_bytes_per_launch": kb.get(k),
                     "frac_model": round(kb[k] / a_s / 1e9 / HBM_PEAK_GBS, 4) if k in kb else None}
    eval_bytes = eval_bytes_per_step * N
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dominant, wl.name),
            "kernel": dominant, "rocprof_kernel": ROCPROF_NAME[dominant],
            "timed_launches": "every launch of the kernel in the timed region",
            "avg_launch_us": avg_s * 1e6, "launches": d_launches,
            "algorithmic_bytes_per_launch": int(mb[dominant]),
            "bytes_model": "16 n_b^2/S + 48 n_b (forward), + 64 n_b (recompute), + 80 n_b (adjoint + "
                           "gradient) bytes per element*level*shot; half-step sweeps take one block and half "
                           "the state",
            "alone": {"avg_launch_us": round(alone_s * 1e6, 2),
                      "frac": round(mb[dominant] / max(alone_s, 1e-12) / 1e9 / HBM_PEAK_GBS, 4)},
            "sweeps_alone": sweeps,
            "evaluation": {"algorithmic_bytes": eval_bytes, "GB/s": eval_bytes * args.steps / el / 1e9,
                           "frac": eval_bytes * args.steps / el / 1e9 / HBM_PEAK_GBS,
                           "bytes_per_unit": eval_bytes_per_step / (units / N)}}
    breakdown = {k: round(v["ms"] / max(args.warmup, 1), 3) for k, v in warm.items()}
    # per-kernel rates of the census (kernels alone): HBM-bound sweeps and contraction against
    # 8 TB/s, the element factorisation against FP64 (8 n_b^3 flop per element and level)
    kernels = {}
    for k, v in census.items():
        if v["launches"] == 0:
            continue
        avg = v["ms"] / v["launches"]
        ent = {"launches": v["launches"], "avg_us": round(avg * 1e3, 2)}
        if k in kb and not k.startswith("solve_"):
            gbs = kb[k] / (avg * 1e-3) / 1e9
            ent.update({"GB/s": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 3)})
        if k == "factor":
            flop = float(8 * (mesh.n_b().astype("int64") ** 3 * mesh.n_r.astype("int64")).sum())
            ent.update({"GFLOP/s": round(flop / (avg * 1e-3) / 1e9, 1), "frac_fp64_peak": round(flop / (avg * 1e-3) / 78.6e12, 4)})
        kernels[k] = ent
    kernels["factorisation_s"] = round(t_factor, 4)
    out = {
        "metric": "element*radial*steps/s fwd+adj FP64",
        "value": value,
        "unit": "element*radial*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "elements": mesh.n_elem, "n_b": 16, "n_r": 32, "time_steps": N,
                   "shots": S, "receivers": R, "dt": wl.dt, "checkpoints": "sqrt(T)", "gradient": "exact",
                   "coarse_solver": "nested-dissection LU, factored per model" if args.coarse_solver == 1
                   else "BiCGStab, rtol 1e-13",
                   "graphs": bool(args.graphs), "launch_plan": "autotuned" if plan is not None else "default",
                   "overlapped_backward": bool(args.overlap),
                   "tail_store_steps": tail_steps["steps"],
                   "scheme": "radial Galerkin" if args.scheme == 1 else "paper finite differences",
                   "units_per_step": units},
        "roofline": roof,
        "kernel_ms_per_step_warmup": breakdown,
        "kernels_alone": kernels,
        "observed_data": fem_out,
        "coarse_solver": stats,
        "misfit": float(misfit.item()),
    }
    mh.close()
    sb.sbfwi_finalize()   # no library stream or event outlives the run
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(N)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

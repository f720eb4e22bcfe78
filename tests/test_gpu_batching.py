"""Batching pattern: ragged meshes, many shots, launch plans, graph replay.

Every sweep launch shape (shots per block 1..16 per n_b class, or one
persistent launch over all classes, joint or separate sweeps, rows of the
central-difference scheme formed on the fly or read) computes each (element,
shot) with the same arithmetic, so results must be bit-identical to the
default plan; the
same holds for the autotuned plan and for graph replay of the forward steps.
The batched multi-shot run must agree with one run per shot, and the ragged
multi-shot run with the oracle.
"""

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import stepper as ostp

from ._gpu import GpuModel, log, rel_l2

pytestmark = pytest.mark.gpu


def _multishot(wl, n_shots, n_steps):
    """Replace the workload's shots by n_shots Ricker sources spread over the top edge."""
    top = W.top_edge_nodes(wl.mesh)
    idx = np.linspace(1, len(top) - 2, n_shots).round().astype(int)
    wl.src_nodes = top[idx].astype(np.int64)
    wl.wavelets = np.stack([W.ricker(n_steps, wl.dt, wl.f0, t0=(0.5 + 0.1 * s) / wl.f0) for s in range(n_shots)])
    wl.n_steps = n_steps
    return wl


def _meshes():
    qt = _multishot(W.config_quadtree_tiny(), 5, 30)
    wide = _multishot(W.config_small(nx=6, ny=3, segs=6, n_r=8, n_steps=30, n_shots=5), 5, 30)
    return [("quadtree", qt), ("nb24", wide)]


def _run(g, steps, obs=None, n_ckpt=-1):
    if obs is None:
        tr, ck = g.forward(n_steps=steps, n_ckpt=n_ckpt)
        return tr.cpu().numpy(), ck
    return g.gradient(obs, n_steps=steps, n_ckpt=n_ckpt)


@pytest.mark.parametrize("name", ["quadtree", "nb24"])
def test_sweep_plans_bit_identical(name):
    wl = dict(_meshes())[name]
    sb_ = None
    rho = wl.models["random30"]
    g = GpuModel(wl, rho)
    sb_ = g.sb
    steps = wl.n_steps
    obs = _run(g, steps, n_ckpt=0)[0] * 0.9
    tr0, mis0, g0, _ = g.gradient(obs, n_steps=steps)
    log(f"launch plans on {name}: {wl.mesh.n_elem} elements, n_b {sorted(set(wl.mesh.n_b().tolist()))}, 5 shots")
    variants = [("S=%d" % S, [(sb_.launch_param_shots(k, c), S) for k in range(4) for c in range(3)])
                for S in (1, 2, 4, 8, 16)]
    variants += [("fused S=%d" % S, [(sb_.launch_param_fused(k), S) for k in range(4)]) for S in (1, 4, 16)]
    # the recover and condense sweeps of consecutive steps run one after the other
    # instead of as one joint sweep (the default), also with other plans
    variants += [("separate sweeps", [(sb_.LAUNCH_JOINT_SWEEPS, 0)]),
                 ("separate sweeps S=2", [(sb_.LAUNCH_JOINT_SWEEPS, 0)] +
                  [(sb_.launch_param_shots(k, c), 2) for k in range(4) for c in range(3)])]
    # the transposed sweeps read the rows theta, psi, P from the factors instead of
    # forming them from the densities (the default for n_b <= 16)
    variants += [("rows read", [(sb_.LAUNCH_ROWS_ON_THE_FLY, 0)]),
                 ("rows read, separate sweeps", [(sb_.LAUNCH_ROWS_ON_THE_FLY, 0), (sb_.LAUNCH_JOINT_SWEEPS, 0)]),
                 ("rows read S=1", [(sb_.LAUNCH_ROWS_ON_THE_FLY, 0)] +
                  [(sb_.launch_param_shots(k, c), 1) for k in range(4) for c in range(3)])]
    for label, params in variants:
        sb_.sbfwi_set_launch(g.f, sb_.LAUNCH_RESET_PLAN, 0)
        sb_.sbfwi_set_launch(g.f, sb_.LAUNCH_JOINT_SWEEPS, 1)
        sb_.sbfwi_set_launch(g.f, sb_.LAUNCH_ROWS_ON_THE_FLY, 1)
        for p, v in params:
            sb_.sbfwi_set_launch(g.f, p, v)
        tr, mis, gr, _ = g.gradient(obs, n_steps=steps)
        same = np.array_equal(tr, tr0) and np.array_equal(gr, g0) and mis == mis0
        log(f"  {label}: bit-identical {same}")
        assert same
    sb_.sbfwi_set_launch(g.f, sb_.LAUNCH_RESET_PLAN, 0)
    sb_.sbfwi_set_launch(g.f, sb_.LAUNCH_JOINT_SWEEPS, 1)
    sb_.sbfwi_set_launch(g.f, sb_.LAUNCH_ROWS_ON_THE_FLY, 1)


def test_autotuned_plan_and_graph_replay_bit_identical():
    wl = dict(_meshes())["quadtree"]
    g = GpuModel(wl, wl.models["random30"])
    sb = g.sb
    steps = wl.n_steps
    obs = _run(g, steps, n_ckpt=0)[0] * 0.9
    tr0, mis0, g0, _ = g.gradient(obs, n_steps=steps)
    plan = sb.sbfwi_autotune(g.f, wl.n_shots)
    log(f"autotuned plan: {plan}")
    for k, v in plan.items():
        assert all(s in (0, 1, 2, 4, 8) for s in v["shots_per_block"])   # 5 shots: at most 8 per block
        assert v["fused"] in (0, 1, 2, 4, 8)
    tr1, mis1, g1, _ = g.gradient(obs, n_steps=steps)
    assert np.array_equal(tr1, tr0) and np.array_equal(g1, g0) and mis1 == mis0
    sb.sbfwi_set_launch(g.f, sb.LAUNCH_GRAPHS, 1)
    for joint in (1, 0):   # graphs of joint sweeps (default) and of separate ones
        sb.sbfwi_set_launch(g.f, sb.LAUNCH_JOINT_SWEEPS, joint)
        for rep in range(2):   # every step replays the captured graphs; the run itself is repeated
            trg, ck = g.forward(n_steps=steps, n_ckpt=0)
            assert np.array_equal(trg.cpu().numpy(), tr0), f"graph replay run {rep} differs (joint {joint})"
            trg2, misg, gg, _ = g.gradient(obs, n_steps=steps)
            assert np.array_equal(trg2, tr0) and np.array_equal(gg, g0) and misg == mis0
    log("graph replay: forward traces and gradients bit-identical over two runs, joint and separate sweeps")
    sb.sbfwi_set_launch(g.f, sb.LAUNCH_GRAPHS, 0)
    sb.sbfwi_set_launch(g.f, sb.LAUNCH_JOINT_SWEEPS, 1)


def test_batched_shots_equal_per_shot_and_oracle():
    wl = _multishot(W.config_quadtree_tiny(), 6, 40)
    rho = wl.models["random30"]
    g = GpuModel(wl, rho)
    g.sb.sbfwi_autotune(g.f, 6)
    g.sb.sbfwi_set_launch(g.f, g.sb.LAUNCH_GRAPHS, 1)
    tr_all = _run(g, 40, n_ckpt=0)[0]
    for s in range(6):
        tr1, _ = g.forward(n_steps=40, shots=[s])
        assert rel_l2(tr1.cpu().numpy()[0], tr_all[s]) <= 1e-13
    om = ostp.Model(wl.mesh, rho, wl.c, wl.dt, wl.beta, wl.gamma, wl.xi0)
    ref = ostp.forward(om, wl.src_nodes, wl.wavelets, wl.rec_nodes, 40)
    err = rel_l2(tr_all, ref)
    obs = ostp.forward(ostp.Model(wl.mesh, rho * 0.97, wl.c, wl.dt, wl.beta, wl.gamma, wl.xi0),
                       wl.src_nodes, wl.wavelets, wl.rec_nodes, 40)
    _, mis, grad, _ = g.gradient(obs, n_steps=40)
    gref, Jref = oadj.exact_gradient(om, wl.src_nodes, wl.wavelets, wl.rec_nodes, obs, 40)
    gerr = rel_l2(grad, gref)
    log(f"6-shot ragged quadtree (autotuned, graphs): traces vs oracle {err:.2e}, gradient vs oracle {gerr:.2e}")
    assert err <= 1e-10
    assert mis == pytest.approx(Jref, rel=1e-10, abs=0)
    assert gerr <= 1e-8

"""Direct coarse solver (nested-dissection LU of K_g, coarse_solver = 1) against the oracle.

The oracle solves K_g exactly with a sparse LU; the direct path must match it
to the same bars as the iterative path (wavefields 1e-10, gradients 1e-8),
and agree with the BiCGStab path (residual 1e-13) to about 1e-11.
"""

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import stepper as ostp

from ._gpu import GpuModel, log, rel_l2

pytestmark = pytest.mark.gpu


def _om(wl, rho):
    return ostp.Model(wl.mesh, rho, wl.c, wl.dt, wl.beta, wl.gamma, wl.xi0)


@pytest.mark.parametrize("cfg,steps", [("tiny", 200), ("small", 60), ("quadtree", 40)])
def test_direct_forward_parity(cfg, steps):
    wl = {"tiny": W.config_tiny, "small": W.config_small, "quadtree": W.config_quadtree_tiny}[cfg]()
    rho = wl.models["random30"]
    g = GpuModel(wl, rho, coarse_solver=1)
    tr, _ = g.forward(n_steps=steps)
    ref = ostp.forward(_om(wl, rho), wl.src_nodes, wl.wavelets[:, :steps], wl.rec_nodes, steps)
    err = rel_l2(tr.cpu().numpy(), ref)
    log(f"direct forward parity {cfg}: traces relative L2 = {err:.3e}")
    assert err <= 1e-10
    stats = g.sb.sbfwi_solver_stats(g.f)
    assert stats["solves"] == steps and stats["iterations"] == 0


@pytest.mark.parametrize("shots", [2, 3])
def test_direct_gradient_parity_and_multishot(shots):
    wl = W.config_small(nx=4, ny=2, segs=2, n_r=7, n_steps=24, n_shots=shots)
    rho = wl.models["random30"]
    om = _om(wl, rho)
    obs = ostp.forward(_om(wl, rho * 0.95), wl.src_nodes, wl.wavelets, wl.rec_nodes, 24)
    g = GpuModel(wl, rho, coarse_solver=1)
    _, mis, grad, _ = g.gradient(obs, n_steps=24, n_ckpt=5)
    gref, Jref = oadj.exact_gradient(om, wl.src_nodes, wl.wavelets, wl.rec_nodes, obs, 24)
    err = rel_l2(grad, gref)
    log(f"direct exact gradient parity ({shots} shots): {err:.3e}")
    assert mis == pytest.approx(Jref, rel=1e-10, abs=0)
    assert err <= 1e-8


@pytest.mark.parametrize("shots", [4, 16])
def test_direct_full_size_matches_iterative(shots):
    # 16 shots: the largest supernode fronts do not fit 16 shots in LDS, so the solve runs in two passes
    steps = 3
    wl = W.config_paper(n_steps=steps, n_shots=shots)
    rng = np.random.default_rng(1000 * 1 + 8)
    wl.wavelets = rng.standard_normal((wl.n_shots, steps))
    wl.rec_nodes = np.arange(wl.mesh.n_nodes, dtype=np.int64)
    rho = wl.models["random30"]
    gi = GpuModel(wl, rho, coarse_solver=0)
    gd = GpuModel(wl, rho, coarse_solver=1)
    ti = gi.forward(n_steps=steps)[0].cpu().numpy()
    td = gd.forward(n_steps=steps)[0].cpu().numpy()
    err = rel_l2(td, ti)
    log(f"full size, {shots} shots: direct vs BiCGStab nodal wavefield relative L2 = {err:.3e}")
    assert err <= 1e-11


@pytest.mark.parametrize("n_ckpt", [-1, 3])
def test_overlapped_recompute_is_bit_identical(n_ckpt):
    """The backward pass with the segment recompute overlapped on a second stream and
    fed with the forward run's kept coarse solutions (the defaults) gives the same bits
    as one segment after the other with coarse solves, and the oracle's gradient;
    several segments, odd and even counts."""
    wl = W.config_small(nx=4, ny=2, segs=2, n_r=7, n_steps=40, n_shots=3)
    rho = wl.models["random30"]
    obs = ostp.forward(_om(wl, rho * 0.95), wl.src_nodes, wl.wavelets, wl.rec_nodes, 40)
    g = GpuModel(wl, rho, coarse_solver=1)
    _, mis1, grad1, _ = g.gradient(obs, n_steps=40, n_ckpt=n_ckpt)
    for overlap, keep in ((0, 1), (1, 0), (0, 0)):
        g.sb.sbfwi_set_launch(g.f, 3, overlap)
        g.sb.sbfwi_set_launch(g.f, 4, keep)
        _, mis0, grad0, _ = g.gradient(obs, n_steps=40, n_ckpt=n_ckpt)
        log(f"n_ckpt {n_ckpt}, overlap {overlap}, kept solutions {keep}: bit-identical "
            f"{np.array_equal(grad1, grad0)}")
        assert np.array_equal(grad1, grad0) and mis1 == mis0
    gref, Jref = oadj.exact_gradient(_om(wl, rho), wl.src_nodes, wl.wavelets, wl.rec_nodes, obs, 40)
    err = rel_l2(grad1, gref)
    log(f"overlapped recompute with kept solutions (n_ckpt {n_ckpt}): vs oracle {err:.3e}")
    assert err <= 1e-8


def test_tail_store_is_bit_identical():
    """With the tail store the forward run keeps the fields of its last checkpoint
    segments and the exact backward pass recomputes only the segments before them:
    the same bits as recomputing every segment, for no, some and all segments in
    the tail, with the recompute overlapped and one segment after the other; the
    paper kernel (which does not use the tail) is unchanged too."""
    wl = W.config_small(nx=4, ny=2, segs=2, n_r=7, n_steps=40, n_shots=3)
    rho = wl.models["random30"]
    obs = ostp.forward(_om(wl, rho * 0.95), wl.src_nodes, wl.wavelets, wl.rec_nodes, 40)
    g = GpuModel(wl, rho, coarse_solver=1)
    sb = g.sb
    n_ckpt = 5                                            # segments of 8 steps
    _, mis0, grad0, _ = g.gradient(obs, n_steps=40, n_ckpt=n_ckpt)
    _, misp0, gradp0, _ = g.gradient(obs, n_steps=40, n_ckpt=n_ckpt, mode=1)
    nb, nr = wl.mesh.n_b().astype(np.int64), wl.mesh.n_r.astype(np.int64)
    per_step = 8 * wl.n_shots * int((nb * (2 * nr + 2)).sum())   # unknowns with ghosts + accelerations
    seen = set()
    for segs in (1, 3, 5, 9):
        kib = (segs * 8 * per_step + 1023) // 1024
        sb.sbfwi_set_launch(g.f, sb.LAUNCH_TAIL_STORE_KIB, kib)
        tr, ck = g.forward(n_steps=40, n_ckpt=n_ckpt)
        tail = sb.sbfwi_ckpt_info(ck)["tail_steps"]
        ck.close()
        assert tail == min(segs, 5) * 8, (segs, tail)
        seen.add(tail)
        for overlap in (1, 0):
            sb.sbfwi_set_launch(g.f, sb.LAUNCH_OVERLAP_BACKWARD, overlap)
            _, mis1, grad1, _ = g.gradient(obs, n_steps=40, n_ckpt=n_ckpt)
            log(f"tail of {tail} steps, overlap {overlap}: bit-identical {np.array_equal(grad1, grad0)}")
            assert np.array_equal(grad1, grad0) and mis1 == mis0
        _, misp1, gradp1, _ = g.gradient(obs, n_steps=40, n_ckpt=n_ckpt, mode=1)
        assert np.array_equal(gradp1, gradp0) and misp1 == misp0
        sb.sbfwi_set_launch(g.f, sb.LAUNCH_OVERLAP_BACKWARD, 1)
    assert seen == {8, 24, 40}
    sb.sbfwi_set_launch(g.f, sb.LAUNCH_TAIL_STORE_KIB, 0)


def test_solve_program_structure():
    """The solve programs evaluate every row once: the forward program |J| + |B_J|
    rows per supernode (y and the update vector), the backward one |J|; one launch
    per dissection level above the cut plus one for the subtrees."""
    import paper_2501_06748_amd as sb
    wl = W.config_paper(n_steps=2)
    m = wl.mesh
    mh = sb.sbfwi_build_mesh(m.node_xy, m.elem_ptr, m.elem_nodes, m.n_r, xi0=wl.xi0)
    info = sb.sbfwi_direct_info(mh)
    fwd, bwd = sb.sbfwi_direct_launches(mh, 0), sb.sbfwi_direct_launches(mh, 1)
    n = int(m.n_nodes)
    log(f"dissection: {info}; {len(fwd)} forward and {len(bwd)} backward launches")
    assert sum(L["rows"] for L in fwd) == n + info["sum_B"]
    assert sum(L["rows"] for L in bwd) == n
    # every block assembles its supernode's whole vector (blocks sharing a supernode reread it)
    assert sum(L["slot_records"] for L in fwd) >= n
    assert sum(L["slot_records"] for L in bwd) >= n + info["sum_B"]
    assert len(fwd) == len(bwd) and fwd[0]["subtrees"] == 1 and bwd[-1]["subtrees"] == 1
    assert all(L["subtrees"] == 0 for L in fwd[1:]) and fwd[-1]["blocks"] >= 1
    assert all(1 <= L["lanes"] <= 64 and L["slots"] >= 1 for L in fwd + bwd)


@pytest.mark.parametrize("cut", [1, 2, 4, 8, 10 ** 9])
def test_subtree_cut_levels_against_the_oracle(cut):
    """The solve programs rebuilt with the subtree launches at other depths
    (sbfwi_set_launch param 6) on a 12 x 6 plate whose dissection tree has five
    levels (1, 2, 4, 8, 8 supernodes): cut 1 makes the whole tree one subtree
    walked by one block in each direction, 2, 4 and 8 root the subtrees at
    levels 1, 2 and 3, and a cut no level reaches gives one launch per level.
    Forward traces and the exact gradient (which runs the transposed programs)
    match the oracle."""
    import paper_2501_06748_amd as sb
    wl = W.config_small(nx=12, ny=6, segs=2, n_r=7, n_steps=24, n_shots=2)
    rho = wl.models["random30"]
    om = _om(wl, rho)
    obs = ostp.forward(_om(wl, rho * 0.95), wl.src_nodes, wl.wavelets, wl.rec_nodes, 24)
    g = GpuModel(wl, rho, coarse_solver=1)
    sb.sbfwi_set_launch(g.f, sb.LAUNCH_SUBTREE_CUT, cut)
    fwd, bwd = sb.sbfwi_direct_launches(g.mesh, 0), sb.sbfwi_direct_launches(g.mesh, 1)
    subtrees = sum(L["subtrees"] for L in fwd) + sum(L["subtrees"] for L in bwd)
    log(f"subtree cut {cut}: {len(fwd)} forward / {len(bwd)} backward launches, "
        f"first forward {fwd[0]}, subtree launches {subtrees}")
    info = sb.sbfwi_direct_info(g.mesh)
    if cut == 1:
        assert len(fwd) == 1 and len(bwd) == 1 and fwd[0]["subtrees"] == 1 and fwd[0]["blocks"] == 1
    elif cut > info["max_per_level"]:
        assert subtrees == 0 and len(fwd) == info["depth"] + 1
    else:
        assert fwd[0]["subtrees"] == 1 and bwd[-1]["subtrees"] == 1 and fwd[0]["blocks"] >= cut
    tr, mis, grad, _ = g.gradient(obs, n_steps=24, n_ckpt=5)
    sb.sbfwi_set_launch(g.f, sb.LAUNCH_SUBTREE_CUT, 512)
    gref, Jref = oadj.exact_gradient(om, wl.src_nodes, wl.wavelets, wl.rec_nodes, obs, 24)
    tref = ostp.forward(om, wl.src_nodes, wl.wavelets, wl.rec_nodes, 24)
    et, eg = rel_l2(tr, tref), rel_l2(grad, gref)
    log(f"  traces {et:.2e}, gradient {eg:.2e}")
    assert et <= 1e-10 and eg <= 1e-8
    assert mis == pytest.approx(Jref, rel=1e-10, abs=0)

"""The benchmarked configuration against the oracle at full size.

The 128 x 64 plate (n_b 16, N_r 32, 8192 elements, 58113 nodes) with the
benchmark's 4 sources and 32 receivers, run exactly as bench.py runs it: the
direct coarse solver (whose transposed solve also runs its subtree launches at
this size), sqrt(T) checkpoints (8 steps: 3 segments, the last one short),
every step's coarse solution kept, the segment recompute overlapped with the
adjoint steps on a second stream, joint sweeps, the gradient contraction on a
third stream.  8 steps of seeded N(0, 1) wavelets, the +-30 % random density
field, zero observed data.  Expected values: tests/golden/paper_gradient_8steps.txt,
written by tests/golden/make_paper_gradient.py (oracle only).  Bars: traces to
relative L2 <= 1e-10, misfit to 1e-10, the gradient of the 32 sampled
elements (the 6 nearest to each source and 8 seeded others) to relative L2
<= 1e-8 together, and each element whose gradient is at least 1e-3 of the
largest element's to relative L2 <= 1e-8 (after 8 steps the fields far from
the sources are exponentially small tails whose relative rounding is larger).
"""

import os
import sys

import numpy as np
import pytest

from ._gpu import GpuModel, log, rel_l2

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_paper_gradient as golden  # noqa: E402


@pytest.mark.skipif(not os.path.exists(golden.OUT), reason="golden file not written")
@pytest.mark.parametrize("tail_gib", [0, 2])
def test_full_size_gradient_matches_the_oracle(tail_gib):
    """tail_gib 2: the forward run also keeps the unknowns and accelerations of
    its last two segments (steps 4-8, 277 MB a step), as bench.py's tail store
    does, and the backward pass recomputes only the first segment."""
    wl, wav, obs, elems = golden.case()
    g_elems, J_ref, tr_ref, g_ref = golden.load()
    assert np.array_equal(g_elems, elems)
    wl.wavelets = wav
    log(f"full size: {wl.mesh.n_elem} elements, {wl.mesh.n_nodes} nodes, 4 shots, {golden.STEPS} steps, "
        f"direct solver, kept solutions, overlapped recompute, tail store {tail_gib} GiB")
    g = GpuModel(wl, wl.models["random30"], coarse_solver=1)
    g.sb.sbfwi_set_launch(g.f, g.sb.LAUNCH_TAIL_STORE_KIB, tail_gib << 20)
    tr, mis, grad, ck = g.gradient(obs, n_steps=golden.STEPS, n_ckpt=-1)
    info = g.sb.sbfwi_ckpt_info(ck)
    assert info["interval"] == 3                     # segments 1-3, 4-6, 7-8
    assert info["tail_steps"] == (5 if tail_gib else 0)
    launches = g.sb.sbfwi_direct_launches(g.mesh, 1)
    assert launches[-1]["subtrees"] == 1             # the transposed solve's subtree launch ran
    et = rel_l2(tr, tr_ref)
    offs = wl.mesh.param_offsets()
    got = np.concatenate([grad[offs[e]:offs[e + 1]] for e in elems])
    eg = rel_l2(got, g_ref)
    worst = 0.0
    k = 0
    norms, errs = [], []
    for e in elems:
        size = int(offs[e + 1] - offs[e])
        norms.append(np.linalg.norm(g_ref[k:k + size]))
        errs.append(rel_l2(got[k:k + size], g_ref[k:k + size]))
        k += size
    norms, errs = np.asarray(norms), np.asarray(errs)
    significant = norms >= 1e-3 * norms.max()
    worst = float(errs[significant].max())
    assert significant.sum() >= 16
    log(f"  traces {et:.2e}, misfit {mis:.6e} vs {J_ref:.6e}, gradient of 32 elements {eg:.2e} "
        f"(worst of {int(significant.sum())} significant elements {worst:.2e})")
    assert np.abs(g_ref).max() > 0
    assert et <= 1e-10
    assert mis == pytest.approx(J_ref, rel=1e-10, abs=0)
    assert eg <= 1e-8 and worst <= 1e-8

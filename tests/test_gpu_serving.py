"""Serving: each request's result is the same alone and in the mix.

Alone: one request at a time on a server with one slot, no batching, no
factor cache and no graph replay.  Mix: all requests submitted at once to a
server with three slots, continuous batching, factor cache, graph replay and
a memory budget small enough that admission has to wait.  Traces, misfit and
per-shot gradient of every request must agree to 1e-12 relative (batching
changes only the block partition of the coarse solver's reductions).
"""

import numpy as np
import pytest

from workloads.serving import serving_requests

from ._gpu import log, rel_l2

pytestmark = pytest.mark.gpu


def _requests(n, steps):
    reqs = serving_requests(n, seed=4 * 1000 + 5, rate=1000.0)
    for r in reqs:
        r.model.n_steps = steps
        r.n_steps = steps
    return reqs


def test_results_same_alone_and_in_the_mix():
    from paper_2501_06748_amd.serving import ShotServer, summarize
    reqs = _requests(10, 60)
    alone = ShotServer(slots=1, batching=False, cache=False, graphs=False)
    alone.start()
    res_alone = {}
    for i, r in enumerate(reqs):
        alone.submit(r)
        res_alone = alone.wait(i + 1, timeout=240)
    alone.stop()
    # a budget that holds about two runs at a time forces admission to wait
    biggest = max(alone._footprint(r.model.key, 1, r.n_steps)[1] for r in reqs)
    mix = ShotServer(slots=3, batching=True, cache=True, graphs=True, budget_bytes=int(2.5 * biggest))
    mix.start()
    for r in reqs:
        mix.submit(r)
    res_mix = mix.wait(len(reqs), timeout=240)
    mix.stop()
    s = summarize(res_mix, reqs)
    log(f"mix: {s}")
    assert s["errors"] == 0 and all(not res_alone[r.rid].error for r in reqs)
    assert max(res_mix[r.rid].batch_shots for r in reqs) > 1         # some requests were batched
    worst = 0.0
    for r in reqs:
        a, m = res_alone[r.rid], res_mix[r.rid]
        worst = max(worst, rel_l2(m.traces, a.traces), abs(m.misfit - a.misfit) / abs(a.misfit),
                    rel_l2(m.grad, a.grad))
        assert np.isfinite(m.grad).all()
    log(f"worst relative difference alone vs mix over {len(reqs)} requests: {worst:.2e}")
    assert worst <= 1e-12


def test_served_results_match_the_oracle():
    """Two small requests served side by side (two slots, batching, factor cache,
    graph replay) against the oracle: traces to relative L2 <= 1e-10, misfit to
    1e-10, per-shot exact gradient to relative L2 <= 1e-8."""
    from oracle import adjoint as oadj
    from oracle import stepper as ostp
    from paper_2501_06748_amd.serving import ShotServer
    steps = 40
    reqs = [r for r in serving_requests(40, seed=4 * 1000 + 5, rate=1000.0) if r.model.key in ("u29", "u21")][:2]
    assert len({r.model.key for r in reqs}) == 2
    for r in reqs:
        r.model.n_steps = steps
        r.n_steps = steps
    srv = ShotServer(slots=2, batching=True, cache=True, graphs=True)
    srv.start()
    for r in reqs:
        srv.submit(r)
    res = srv.wait(len(reqs), timeout=240)
    srv.stop()
    for r in reqs:
        got = res[r.rid]
        assert not got.error, got.error
        mesh, rho = r.model.build()
        src, wav, rec, obs = r.inputs(mesh)
        om = ostp.Model(mesh, rho, r.model.c, r.model.dt)
        gref, Jref = oadj.exact_gradient(om, np.asarray([src]), wav[None], rec, obs[None], steps)
        tref = ostp.forward(om, np.asarray([src]), wav[None], rec, steps)[0]
        et, eg = rel_l2(got.traces, tref), rel_l2(got.grad, gref)
        log(f"served request {r.rid} ({r.model.key}, {mesh.n_elem} elements): traces {et:.2e}, "
            f"misfit {got.misfit:.6e} vs {Jref:.6e}, gradient {eg:.2e}")
        assert et <= 1e-10 and eg <= 1e-8
        assert got.misfit == pytest.approx(Jref, rel=1e-10, abs=0)

"""Writes the oracle's exact gradient on the benchmark's full-size plate for the
GPU parity test of that configuration.  Calls only ``oracle`` and
``workloads``; run from the repository root (about 5 to 15 minutes and 40 GB
of host memory): python tests/golden/make_paper_gradient.py

Case: the 128 x 64 plate (n_b 16, N_r 32, 8192 elements, 58113 nodes), the
+-30 % random density field, the benchmark's 4 sources and 32 receivers,
8 time steps of seeded N(0, 1) wavelets (so that every step carries signal),
zero observed data; the gradient is contracted on 32 elements: the 6 nearest
to each source (in 8 steps the forward field is significant only there; the
adjoint field covers the top edge) and 8 seeded others.
Output: paper_gradient_8steps.txt with the element ids, the traces
[shot][receiver][step] and the gradient entries of those elements (level-major
per element, the library's fine-grid layout), and the misfit.
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import adjoint as adj  # noqa: E402
from oracle import stepper as stp  # noqa: E402

STEPS = 8
OUT = os.path.join(HERE, "paper_gradient_8steps.txt")


def case():
    """The workload, wavelets, observed data and sampled elements of the case."""
    wl = W.config_paper(n_steps=STEPS, n_shots=4)
    rng = np.random.default_rng(1000 * 1 + 31)
    wav = rng.standard_normal((wl.n_shots, STEPS))
    obs = np.zeros((wl.n_shots, len(wl.rec_nodes), STEPS))
    mesh = wl.mesh
    cen = np.stack([mesh.node_xy[mesh.loop(e)].mean(axis=0) for e in range(mesh.n_elem)])
    near = []
    for sn in wl.src_nodes:
        d = np.linalg.norm(cen - mesh.node_xy[sn], axis=1)
        near += [int(e) for e in np.argsort(d, kind="stable")[:6]]
    others = [int(e) for e in rng.permutation(mesh.n_elem) if int(e) not in near][:8]
    elems = np.sort(np.asarray(near + others, dtype=np.int64))
    assert len(set(elems.tolist())) == 32
    return wl, wav, obs, elems


def main():
    wl, wav, obs, elems = case()
    m = stp.Model(wl.mesh, wl.models["random30"], wl.c, wl.dt)
    tr = stp.forward(m, wl.src_nodes, wav, wl.rec_nodes, STEPS)
    g, J = adj.exact_gradient(m, wl.src_nodes, wav, wl.rec_nodes, obs, STEPS, elements=elems)
    offs = wl.mesh.param_offsets()
    gsel = np.concatenate([g[offs[e]:offs[e + 1]] for e in elems])
    assert np.isfinite(gsel).all()
    with open(OUT, "w") as fh:
        fh.write("# oracle exact gradient, 128x64 plate (n_b 16, N_r 32), random30 model, 4 shots, "
                 f"{STEPS} steps of seeded N(0,1) wavelets, zero data; written by make_paper_gradient.py\n")
        fh.write("elements " + " ".join(str(int(e)) for e in elems) + "\n")
        fh.write(f"misfit {J:.17e}\n")
        fh.write("traces " + " ".join(f"{v:.17e}" for v in tr.ravel()) + "\n")
        fh.write("gradient " + " ".join(f"{v:.17e}" for v in gsel) + "\n")


def load():
    """(elements, misfit, traces [4, 32, STEPS], gradient entries of the elements)."""
    vals = {}
    with open(OUT) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            key, *rest = line.split()
            vals[key] = rest
    elems = np.asarray([int(v) for v in vals["elements"]], dtype=np.int64)
    tr = np.asarray([float(v) for v in vals["traces"]]).reshape(4, 32, STEPS)
    return elems, float(vals["misfit"][0]), tr, np.asarray([float(v) for v in vals["gradient"]])


if __name__ == "__main__":
    main()

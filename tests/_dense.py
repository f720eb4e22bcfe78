"""Brute-force time loop of the uncondensed system (test infrastructure).

The global matrix holds every element's rows of eq. system (levels -1 .. n+1
with the ghost rows) and the element flux rows summed at the shared boundary
nodes; each Newmark step is one dense solve of it.  No condensation, no
coarse assembly: an independent route to the fields of the oracle's
condensed stepper.  Uniform meshes (one element group) only.
"""

from __future__ import annotations

import numpy as np

from oracle import element as el


class DenseSystem:
    def __init__(self, model):
        assert len(model.groups) == 1, "one (n_b, N_r) group only"
        g = model.groups[0]
        self.model, self.g = model, g
        n, nb, E = g.n, g.n_b, len(g.elem_ids)
        Ae = el.element_system(g.theta, g.phi, g.psi)
        # unknowns per element: levels -1 .. n-1 and n+1 (internal); then the global nodes
        blocks = list(range(0, n + 1)) + [n + 2]
        ic = np.concatenate([np.arange(b * nb, (b + 1) * nb) for b in blocks])
        bc = np.arange((n + 1) * nb, (n + 2) * nb)
        ir = np.arange(0, (n + 2) * nb)
        br = np.arange((n + 2) * nb, (n + 3) * nb)
        NI = ic.size
        mesh = model.mesh
        N = E * NI + mesh.n_nodes
        A = np.zeros((N, N))
        for e in range(E):
            sl = slice(e * NI, (e + 1) * NI)
            nodes = E * NI + g.loops[e]
            A[sl, sl] = Ae[e][np.ix_(ir, ic)]
            A[sl, nodes] += Ae[e][np.ix_(ir, bc)]
            A[np.ix_(nodes, np.arange(e * NI, (e + 1) * NI))] += Ae[e][np.ix_(br, ic)]
            A[np.ix_(nodes, nodes)] += Ae[e][np.ix_(br, bc)]
        self.A, self.NI, self.N = A, NI, N

    def run(self, nodes, amps, n_steps):
        """Newmark loop driven by point forces amps[c][k - 1] at nodes[c] in step k.
        Returns per step a dict with the unknowns X (levels -1 .. n+1 per element),
        the nodal displacement U and the velocities in the fine-grid layout
        (levels 0 .. n of every element; level n = the nodal velocity)."""
        g, nm, A, NI, N = self.g, self.model.nm, self.A, self.NI, self.N
        n, nb, E = g.n, g.n_b, len(g.elem_ids)
        nn = self.model.mesh.n_nodes
        U = V = Acc = np.zeros(nn)
        u = v = a = np.zeros((E, n, nb))
        out = []
        for k in range(1, n_steps + 1):
            Wn = nm.a0 * U + nm.a1 * V + nm.a2 * Acc
            wi = nm.a0 * u + nm.a1 * v + nm.a2 * a
            p = np.einsum("ejab,ejb->eja", g.P, np.concatenate([wi, Wn[g.loops][:, None]], 1))
            b = np.zeros(N)
            for e in range(E):
                b[e * NI + nb:e * NI + (n + 2) * nb] = p[e].ravel()
            np.add.at(b, E * NI + np.asarray(nodes), np.asarray(amps)[:, k - 1])
            X = np.linalg.solve(A, b)
            Un = X[E * NI:]
            loc = X[:E * NI].reshape(E, n + 2, nb)
            un = loc[:, 1:n + 1]
            U, V, Acc = Un, nm.c1 * (Un - U) + nm.c2 * V + nm.c3 * Acc, nm.a0 * Un - Wn
            u, v, a = un, nm.c1 * (un - u) + nm.c2 * v + nm.c3 * a, nm.a0 * un - wi
            Xd = np.concatenate([loc[:, :n + 1], U[g.loops][:, None], loc[:, n + 1:]], axis=1)
            vel = np.concatenate([v, V[g.loops][:, None]], axis=1)        # [E, n+1, nb]
            fine = np.zeros(self.model.mesh.n_params)
            offs = self.model.mesh.param_offsets()
            for i, e in enumerate(g.elem_ids):
                fine[offs[e]:offs[e + 1]] = vel[i].ravel()
            out.append({"X": Xd, "U": U.copy(), "v_fine": fine})
        return out

"""CPU oracle for the SBFEM full-waveform-inversion hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 (and
complex128, for complex-step checks) NumPy/SciPy implementation of what the
GPU path computes, written from the paper (Daneshyar & Kollmannsberger,
"Full-waveform inversion via the scaled boundary finite element method").
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product path (``paper_2501_06748_amd``)
never imports, links or executes anything here, and this package shares no
code with it: the only common dependency is the seeded input generator
``workloads``, which holds none of the method's arithmetic.

Modules
-------
``element``   geometry, coefficient matrices E0, E1, E2, M0 (eq. Es), their
              radial finite differences, the three-point block rows and the
              ghost/boundary rows (eq. system), and the paper's condensation
              sweep that yields the dynamic stiffness S and effective source;
              also the rows of the radial Galerkin scheme (linear elements in
              xi, lumped radial mass) in the same block layout.
``stepper``   coarse assembly, exact sparse LU coarse solve, the per-step
              condense / solve / recover / Newmark loop, receivers, misfit.
``adjoint``   exact discrete adjoint gradient of the misfit (transposed
              solves of the uncondensed block system by block elimination)
              and the paper's truncated zero-lag kernel.
``lfe``       conventional SBFEM by low-frequency expansion (Riccati +
              Lyapunov) for radially constant density, and the time-domain
              path over element K, M from the radial condensation.
``stability`` step-map spectrum of the coupled discrete system (gate for
              models on which the radial finite-difference scheme is stable).
``radial_galerkin`` linear radial elements for one element, assembled
              densely: its stiffness, mass and condensed dynamic stiffness (an
              independent limit of the finite differences and the reference
              of the Galerkin rows).
``fem``       bilinear finite elements with lumped mass and central
              differences: the generator of observed data from a finer,
              conventional model (no inverse crime).

Every function cites the passage of the paper it follows.  Parity-unpinned
functions say so in their docstrings.
"""

"""The oracle reproduces its committed regression fixture (written by
tests/golden/make_golden.py, which calls only the oracle)."""

import os

import numpy as np

import workloads as W
from oracle import stepper as stp

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_tiny_traces_fixture():
    ref = np.loadtxt(os.path.join(HERE, "tiny_random30_traces_60.txt"))
    cfg = W.config_tiny(n_steps=60)
    m = stp.Model(cfg.mesh, cfg.models["random30"], cfg.c, cfg.dt)
    tr = stp.forward(m, cfg.src_nodes, cfg.wavelets, cfg.rec_nodes, cfg.n_steps)
    np.testing.assert_allclose(tr[0].T, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())

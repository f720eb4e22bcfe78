"""Writes the oracle regression fixtures in this folder.  Calls only ``oracle`` and
``workloads``; run from the repository root: python tests/golden/make_golden.py"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import stepper as stp  # noqa: E402


def main():
    cfg = W.config_tiny(n_steps=60)
    m = stp.Model(cfg.mesh, cfg.models["random30"], cfg.c, cfg.dt)
    tr = stp.forward(m, cfg.src_nodes, cfg.wavelets, cfg.rec_nodes, cfg.n_steps)
    np.savetxt(os.path.join(HERE, "tiny_random30_traces_60.txt"), tr[0].T, fmt="%.17e",
               header="oracle traces [step][receiver], tiny 8x8 plate (n_b 8, N_r 16), "
                      "random30 model, 60 steps, written by make_golden.py")


if __name__ == "__main__":
    main()

"""The allocation-free observed-data generator (sbfwi_fem_forward_noalloc)
against the allocating entry point (sbfwi_fem_forward), through the C ABI.

Both run the same kernels on the same inputs, so their traces must agree bit
for bit.  Two calls in a row, the second on a smaller grid with fewer shots
and receivers (the shared scratch array then holds the first call's larger
fields, which must not leak into the second), each checked against a fresh
allocating run; a grid beyond the scratch array is refused before any launch.
"""

import numpy as np
import pytest

import workloads as W
from oracle import fem as ofem

from ._gpu import log

pytestmark = pytest.mark.gpu


def _host_inputs(nx, ny, lx, ly, n_shots, nt, seed):
    g = W.FemGrid(nx, ny, lx, ly)
    rng = np.random.default_rng(seed)
    rho = 2700.0 * rng.uniform(0.05, 2.0, g.n_elem)
    dt = 0.8 * ofem.stable_dt(g.nx, g.ny, g.lx, g.ly, 3000.0)
    # sources on the top row of grid nodes (node (i, j) has id j (nx + 1) + i)
    src = np.array([ny * (nx + 1) + int((s + 0.5) * nx / n_shots) for s in range(n_shots)], dtype=np.int64)
    rec = np.unique(np.linspace(0, g.n_nodes - 1, 13).astype(np.int64))
    wav = np.stack([W.ricker(nt, dt, 5e5, t0=(1.0 + 0.2 * s) * 2e-6) for s in range(n_shots)])
    return g, rho, dt, src, wav, rec


def _inputs(*args):
    import torch
    g, rho, dt, src, wav, rec = _host_inputs(*args)
    d = "cuda"
    return (g, torch.tensor(rho, device=d), dt, torch.tensor(src, device=d), torch.tensor(wav, device=d),
            torch.tensor(rec, device=d))


def _both(g, rho, dt, src, wav, rec):
    import torch
    import paper_2501_06748_amd as sb
    S, N = wav.shape
    ta = torch.full((S, rec.shape[0], N), np.nan, dtype=torch.float64, device="cuda")
    tb = torch.full_like(ta, np.nan)
    sb.sbfwi_fem_forward(g.nx, g.ny, g.lx, g.ly, rho, 3000.0, dt, src, wav, rec, ta)
    sb.sbfwi_fem_forward_noalloc(g.nx, g.ny, g.lx, g.ly, rho, 3000.0, dt, src, wav, rec, tb)
    torch.cuda.synchronize()
    return ta.cpu().numpy(), tb.cpu().numpy()


def test_noalloc_equals_allocating_entry_two_calls():
    big = _inputs(512, 256, 0.1, 0.05, 4, 400, 31)        # the paper-sized data grid
    small = _inputs(37, 23, 0.0037, 0.0023, 2, 300, 32)   # smaller grid, fewer shots, after the big one
    for name, inp in (("512x256, 4 shots", big), ("37x23, 2 shots", small)):
        log(f"allocation-free FEM generator vs allocating one: {name}")
        ta, tb = _both(*inp)
        assert np.isfinite(ta).all() and np.abs(ta).max() > 0
        assert np.array_equal(ta, tb)


def test_noalloc_rejects_grid_beyond_scratch():
    import torch
    import paper_2501_06748_amd as sb
    nx = ny = 2048
    d = "cuda"
    rho = torch.full((nx * ny,), 2700.0, dtype=torch.float64, device=d)
    src = torch.tensor([0, 1, 2, 3], dtype=torch.int64, device=d)
    wav = torch.zeros((4, 10), dtype=torch.float64, device=d)
    rec = torch.tensor([5], dtype=torch.int64, device=d)
    tr = torch.zeros((4, 1, 10), dtype=torch.float64, device=d)
    with pytest.raises(sb.SbfwiError) as ei:
        sb.sbfwi_fem_forward_noalloc(nx, ny, 1.0, 1.0, rho, 3000.0, 1e-8, src, wav, rec, tr)
    assert ei.value.code == sb._abi.EINVAL and "scratch" in sb.sbfwi_last_error()

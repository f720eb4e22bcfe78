"""Helpers for GPU tests: run a workload through the C ABI (via the thin binding)."""

from __future__ import annotations

import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


class GpuModel:
    """Mesh + factors of a workload model on cuda:0 (by default with the library's
    default coarse solver, the direct one)."""

    def __init__(self, wl, rho, dt=None, coarse_solver=1, scheme=0):
        import torch
        import paper_2501_06748_amd as sb
        self.sb, self.torch, self.wl = sb, torch, wl
        m = wl.mesh
        self.dt = wl.dt if dt is None else dt
        self.mesh = sb.sbfwi_build_mesh(m.node_xy, m.elem_ptr, m.elem_nodes, m.n_r, xi0=wl.xi0)
        self.rho = torch.tensor(np.asarray(rho), dtype=torch.float64, device="cuda")
        self.f = sb.sbfwi_factor_elements(self.mesh, self.rho, wl.c, self.dt, wl.beta, wl.gamma, scheme=scheme,
                                          coarse_solver=coarse_solver)
        self.info = sb.sbfwi_mesh_info(self.mesh)

    def tensors(self, n_steps=None, shots=None):
        torch, wl = self.torch, self.wl
        n_steps = wl.n_steps if n_steps is None else n_steps
        idx = list(range(wl.n_shots)) if shots is None else list(shots)
        src = torch.tensor(wl.src_nodes[idx], dtype=torch.int64, device="cuda")
        wav = torch.tensor(np.ascontiguousarray(wl.wavelets[idx, :n_steps]), dtype=torch.float64, device="cuda")
        rec = torch.tensor(wl.rec_nodes, dtype=torch.int64, device="cuda")
        tr = torch.zeros((len(idx), len(wl.rec_nodes), n_steps), dtype=torch.float64, device="cuda")
        return src, wav, rec, tr

    def forward(self, n_steps=None, shots=None, n_ckpt=0):
        src, wav, rec, tr = self.tensors(n_steps, shots)
        ck = self.sb.sbfwi_forward(self.f, src, wav, rec, tr, n_ckpt=n_ckpt)
        self.torch.cuda.synchronize()
        return tr, ck

    def gradient(self, observed, n_steps=None, shots=None, n_ckpt=-1, mode=0):
        torch = self.torch
        tr, ck = self.forward(n_steps, shots, n_ckpt=n_ckpt)
        obs = torch.tensor(np.ascontiguousarray(observed), dtype=torch.float64, device="cuda")
        mis = torch.zeros(1, dtype=torch.float64, device="cuda")
        grad = torch.zeros(self.info["n_params"], dtype=torch.float64, device="cuda")
        self.sb.sbfwi_gradient(self.f, ck, obs, tr, mode, mis, grad)
        torch.cuda.synchronize()
        return tr.cpu().numpy(), float(mis.item()), grad.cpu().numpy(), ck


def fem_gpu(grid, rho_elem, c, dt, src, wavelets, rec, n_steps=None):
    """Finite element data on cuda:0 through the C ABI; returns traces [S, R, N] (numpy)."""
    import torch
    import paper_2501_06748_amd as sb
    wav = np.ascontiguousarray(np.asarray(wavelets, dtype=np.float64))
    if n_steps is not None:
        wav = np.ascontiguousarray(wav[:, :n_steps])
    S, N = wav.shape
    d = "cuda"
    tr = torch.full((S, len(rec), N), np.nan, dtype=torch.float64, device=d)
    sb.sbfwi_fem_forward(grid.nx, grid.ny, grid.lx, grid.ly,
                         torch.tensor(np.asarray(rho_elem, dtype=np.float64), device=d), c, dt,
                         torch.tensor(np.asarray(src, dtype=np.int64), device=d), torch.tensor(wav, device=d),
                         torch.tensor(np.asarray(rec, dtype=np.int64), device=d), tr)
    torch.cuda.synchronize()
    return tr.cpu().numpy()

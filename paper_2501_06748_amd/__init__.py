"""MI355X (gfx950) hot path of SBFEM full-waveform inversion with radial discretisation.

Thin Python binding of the C ABI in include/sbfwi.h.  The functions below
carry the ABI's names and only marshal arguments: host arrays are NumPy,
device arrays are torch CUDA (ROCm) tensors whose data pointers and the
current HIP stream are passed through.  Every step of the path runs in the
HIP kernels of libsbfwi.so; without the built library nothing here runs.

Higher layers in this package:
  ``autograd``  -- torch.autograd.Function over forward + adjoint gradient;
  ``lbfgs``     -- the outer L-BFGS loop with box constraints;
  ``serving``   -- continuous-batching request loop with HBM admission;
  ``batching``  -- multi-shot batched stepping and tile autotuning helpers.
"""

from __future__ import annotations

import atexit
import ctypes as C
import weakref

import numpy as np

from ._abi import SbfwiError, check, lib

SCHEME_PAPER_FD = 0
SCHEME_RADIAL_GALERKIN = 1
SCHEME_LFE = 2
SCHEME_LFE_CONDENSED = 3
GRAD_EXACT = 0
GRAD_PAPER_KERNEL = 1
GRAD_PER_SHOT = 16


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dptr(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (ROCm) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _hptr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


_live_handles = weakref.WeakSet()   # open handles, closed by sbfwi_finalize


class _Handle:
    _destroy = None
    _order = 0     # closing order at finalize: checkpoints, then factors, then meshes

    def __init__(self, ptr):
        self.ptr = ptr
        if ptr:
            _live_handles.add(self)

    def close(self):
        if self.ptr:
            getattr(lib(), self._destroy)(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def _as_parameter_(self):
        if not self.ptr:
            raise ValueError("handle is closed")
        return self.ptr


class MeshHandle(_Handle):
    _destroy = "sbfwi_destroy_mesh"
    _order = 2


class FactorsHandle(_Handle):
    _destroy = "sbfwi_destroy_factors"
    _order = 1

    def __init__(self, ptr, mesh):
        super().__init__(ptr)
        self.mesh = mesh   # the factors reference the mesh, keep it alive


class CkptHandle(_Handle):
    _destroy = "sbfwi_destroy_ckpt"

    def __init__(self, ptr, factors, n_shots=0, n_rec=0, n_steps=0, n_params=0):
        super().__init__(ptr)
        self.factors = factors
        # sizes of the run, checked against every array passed with this handle
        self.n_shots, self.n_rec, self.n_steps, self.n_params = n_shots, n_rec, n_steps, n_params


def sbfwi_last_error() -> str:
    return lib().sbfwi_last_error().decode()


def sbfwi_finalize():
    """Closes every open handle (checkpoints, factors, meshes) and releases the
    library's own streams and events (sbfwi_finalize of the C ABI).  Registered
    to run at interpreter exit; safe to call more than once."""
    from . import _abi
    if _abi._lib is None:
        return
    for h in sorted(list(_live_handles), key=lambda h: h._order):
        h.close()
    check(lib().sbfwi_finalize())


@atexit.register
def _finalize_at_exit():
    try:
        sbfwi_finalize()
    except Exception:
        pass


def sbfwi_build_mesh(node_xy, elem_ptr, elem_nodes, n_r, centre_xy=None, xi0=1e-3) -> MeshHandle:
    xy, pxy = _hptr(node_xy, np.float64)
    ep, pep = _hptr(elem_ptr, np.int64)
    en, pen = _hptr(elem_nodes, np.int64)
    nr, pnr = _hptr(n_r, np.int32)
    pc = None
    if centre_xy is not None:
        cc, pc = _hptr(centre_xy, np.float64)
    out = C.c_void_p()
    check(lib().sbfwi_build_mesh(pxy, xy.shape[0], pep, pen, ep.shape[0] - 1, pc, pnr, float(xi0), C.byref(out)))
    return MeshHandle(out.value)


def sbfwi_mesh_info(m: MeshHandle) -> dict:
    buf = np.zeros(5, dtype=np.int64)
    check(lib().sbfwi_mesh_info(m, buf.ctypes.data_as(C.c_void_p)))
    return {"n_nodes": int(buf[0]), "n_elem": int(buf[1]), "n_params": int(buf[2]), "nnz": int(buf[3]),
            "n_interior": int(buf[4])}


def sbfwi_factor_elements(m: MeshHandle, rho, c, dt, beta=0.25, gamma=0.5, scheme=SCHEME_PAPER_FD,
                          coarse_solver=1, stream=None) -> FactorsHandle:
    """Factors of one model: rho [n_params] f64 (device).  coarse_solver 1 (default): the
    direct nested-dissection LU of K_g, factored here once; 0: BiCGStab every step."""
    import torch
    out = C.c_void_p()
    check(lib().sbfwi_factor_elements(m, _dptr(rho, torch.float64, "rho"), float(c), float(dt), float(beta),
                                      float(gamma), int(scheme), int(coarse_solver), _stream(stream),
                                      C.byref(out)))
    return FactorsHandle(out.value, m)


def sbfwi_set_solver(f: FactorsHandle, rtol=1e-13, max_iter=500):
    check(lib().sbfwi_set_solver(f, float(rtol), int(max_iter)))


def sbfwi_set_launch(f: FactorsHandle, param: int, value: int):
    check(lib().sbfwi_set_launch(f, int(param), int(value)))


def sbfwi_plan_bytes(m: MeshHandle, n_shots: int, n_steps: int, n_ckpt: int = -1) -> dict:
    out = np.zeros(4, dtype=np.int64)
    check(lib().sbfwi_plan_bytes(m, int(n_shots), int(n_steps), int(n_ckpt), out.ctypes.data_as(C.c_void_p)))
    return {"factors": int(out[0]), "checkpoints": int(out[1]), "forward_work": int(out[2]),
            "backward_work": int(out[3])}


def sbfwi_direct_info(m: MeshHandle) -> dict:
    out = np.zeros(7, dtype=np.int64)
    check(lib().sbfwi_direct_info(m, out.ctypes.data_as(C.c_void_p)))
    keys = ["supernodes", "depth", "max_supernode", "sum_J2", "sum_JB", "sum_B", "max_per_level"]
    return {k: int(v) for k, v in zip(keys, out)}


def sbfwi_direct_launches(m: MeshHandle, direction: int) -> list:
    """Launches of the direct solve's forward (0) or backward (1) program, in order."""
    cap = 256
    out = np.zeros(8 * cap, dtype=np.int64)
    n = C.c_int(0)
    check(lib().sbfwi_direct_launches(m, int(direction), out.ctypes.data_as(C.c_void_p), cap, C.byref(n)))
    keys = ["blocks", "lanes", "slots", "steps", "rows", "slot_records", "max_step_rows", "subtrees"]
    return [dict(zip(keys, (int(v) for v in out[8 * k:8 * k + 8]))) for k in range(min(n.value, cap))]


def sbfwi_autotune(f: FactorsHandle, n_shots: int, stream=None) -> dict:
    """Times the sweep launch shapes for runs of n_shots shots and keeps the fastest plan."""
    out = np.zeros(24, dtype=np.float64)
    check(lib().sbfwi_autotune(f, int(n_shots), out.ctypes.data_as(C.c_void_p), _stream(stream)))
    kinds = ["condense", "recover", "adj_condense", "adj_recover"]
    return {k: {"shots_per_block": [int(v) for v in out[6 * i:6 * i + 3]], "fused": int(out[6 * i + 3]),
                "ms_per_class": float(out[6 * i + 4]), "ms_fused": float(out[6 * i + 5])}
            for i, k in enumerate(kinds)}


LAUNCH_ENQUEUED_ITERS, LAUNCH_GRAPHS, LAUNCH_RESET_PLAN = 0, 1, 2
LAUNCH_OVERLAP_BACKWARD, LAUNCH_KEEP_SOLUTIONS, LAUNCH_JOINT_SWEEPS, LAUNCH_SUBTREE_CUT = 3, 4, 5, 6
LAUNCH_ROWS_ON_THE_FLY, LAUNCH_TAIL_STORE_KIB = 7, 8


def launch_param_shots(sweep: int, cls: int) -> int:
    """sbfwi_set_launch parameter of the shots per block of sweep (0..3) and n_b class (0..2)."""
    return 10 + 3 * sweep + cls


def launch_param_fused(sweep: int) -> int:
    return 30 + sweep


def apply_plan(f: FactorsHandle, plan: dict) -> None:
    """Sets the launch plan returned by sbfwi_autotune (for the same mesh and shot count) on
    other factors, e.g. those of the next model of an inversion."""
    kinds = ["condense", "recover", "adj_condense", "adj_recover"]
    for i, k in enumerate(kinds):
        for cl, v in enumerate(plan[k]["shots_per_block"]):
            sbfwi_set_launch(f, launch_param_shots(i, cl), int(v))
        sbfwi_set_launch(f, launch_param_fused(i), int(plan[k]["fused"]))


def sbfwi_copy_factor_data(f: FactorsHandle, which: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    check(lib().sbfwi_copy_factor_data(f, int(which), out.ctypes.data_as(C.c_void_p)))
    return out


def sbfwi_coarse_pattern(m: MeshHandle):
    info = sbfwi_mesh_info(m)
    rp = np.empty(info["n_nodes"] + 1, dtype=np.int64)
    col = np.empty(info["nnz"], dtype=np.int64)
    check(lib().sbfwi_coarse_pattern(m, rp.ctypes.data_as(C.c_void_p), col.ctypes.data_as(C.c_void_p)))
    return rp, col


def sbfwi_forward(f: FactorsHandle, src_node, wavelet, rec_node, traces, n_ckpt=0, stream=None):
    """src_node [S] int64, wavelet [S, N_t] f64, rec_node [R] int64, traces [S, R, N_t] f64 (device)."""
    import torch
    n_shots, n_steps = int(wavelet.shape[0]), int(wavelet.shape[1])
    n_rec = int(rec_node.shape[0])
    if traces.shape != (n_shots, n_rec, n_steps) or src_node.shape != (n_shots,):
        raise ValueError("shape mismatch between src_node, wavelet, rec_node and traces")
    out = C.c_void_p()
    check(lib().sbfwi_forward(f, n_shots, n_steps, _dptr(src_node, torch.int64, "src_node"),
                              _dptr(wavelet, torch.float64, "wavelet"), n_rec,
                              _dptr(rec_node, torch.int64, "rec_node"), _dptr(traces, torch.float64, "traces"),
                              int(n_ckpt), C.byref(out) if n_ckpt != 0 else None, _stream(stream)))
    if n_ckpt == 0:
        return None
    return CkptHandle(out.value, f, n_shots, n_rec, n_steps, sbfwi_mesh_info(f.mesh)["n_params"])


def sbfwi_fem_forward(nx, ny, lx, ly, rho_elem, c, dt, src_node, wavelet, rec_node, traces, stream=None):
    """Finite element data: rho_elem [ny * nx] f64, src_node [S] int64, wavelet [S, N_t] f64,
    rec_node [R] int64, traces [S, R, N_t] f64 (device); grid node (i, j) is j (nx + 1) + i."""
    import torch
    n_shots, n_steps = int(wavelet.shape[0]), int(wavelet.shape[1])
    n_rec = int(rec_node.shape[0])
    if traces.shape != (n_shots, n_rec, n_steps) or src_node.shape != (n_shots,):
        raise ValueError("shape mismatch between src_node, wavelet, rec_node and traces")
    if rho_elem.numel() != int(nx) * int(ny):
        raise ValueError("rho_elem must hold nx * ny densities")
    check(lib().sbfwi_fem_forward(int(nx), int(ny), float(lx), float(ly), _dptr(rho_elem, torch.float64, "rho_elem"),
                                  float(c), float(dt), n_shots, n_steps, _dptr(src_node, torch.int64, "src_node"),
                                  _dptr(wavelet, torch.float64, "wavelet"), n_rec,
                                  _dptr(rec_node, torch.int64, "rec_node"), _dptr(traces, torch.float64, "traces"),
                                  _stream(stream)))


def sbfwi_fem_forward_noalloc(nx, ny, lx, ly, rho_elem, c, dt, src_node, wavelet, rec_node, traces, stream=None):
    """sbfwi_fem_forward without any allocation by the library (work buffers in its
    static device scratch array; calls that overlap on one GPU race)."""
    import torch
    n_shots, n_steps = int(wavelet.shape[0]), int(wavelet.shape[1])
    n_rec = int(rec_node.shape[0])
    if traces.shape != (n_shots, n_rec, n_steps) or src_node.shape != (n_shots,):
        raise ValueError("shape mismatch between src_node, wavelet, rec_node and traces")
    if rho_elem.numel() != int(nx) * int(ny):
        raise ValueError("rho_elem must hold nx * ny densities")
    check(lib().sbfwi_fem_forward_noalloc(int(nx), int(ny), float(lx), float(ly),
                                          _dptr(rho_elem, torch.float64, "rho_elem"), float(c), float(dt), n_shots,
                                          n_steps, _dptr(src_node, torch.int64, "src_node"),
                                          _dptr(wavelet, torch.float64, "wavelet"), n_rec,
                                          _dptr(rec_node, torch.int64, "rec_node"),
                                          _dptr(traces, torch.float64, "traces"), _stream(stream)))


def _check_run_shapes(ck, mode, grad, misfit=None, **series):
    """Every array passed with a checkpoint handle must have the sizes of its run:
    the library reads and writes them by the run's shot, receiver and step counts."""
    run = (ck.n_shots, ck.n_rec, ck.n_steps)
    for name, t in series.items():
        if tuple(t.shape) != run:
            raise ValueError(f"{name} has shape {tuple(t.shape)}, the checkpointed run is "
                             f"[shots, receivers, steps] = {list(run)}")
    per = ck.n_shots if (int(mode) & GRAD_PER_SHOT) else 1
    if grad.numel() != per * ck.n_params:
        raise ValueError(f"grad must hold {per} x {ck.n_params} values")
    if misfit is not None and misfit.numel() < per:
        raise ValueError(f"misfit must hold {per} values")


def sbfwi_adjoint(f: FactorsHandle, ck: CkptHandle, adj_src, mode, grad, stream=None):
    """adj_src [S, R, N_t] f64 (device); grad [n_params] or, with GRAD_PER_SHOT, [S, n_params]."""
    import torch
    _check_run_shapes(ck, mode, grad, adj_src=adj_src)
    check(lib().sbfwi_adjoint(f, ck, _dptr(adj_src, torch.float64, "adj_src"), int(mode),
                              _dptr(grad, torch.float64, "grad"), _stream(stream)))


def sbfwi_gradient(f: FactorsHandle, ck: CkptHandle, observed, traces, mode, misfit, grad, stream=None):
    """observed, traces [S, R, N_t]; misfit [1] (or [S] with GRAD_PER_SHOT); grad as in sbfwi_adjoint."""
    import torch
    _check_run_shapes(ck, mode, grad, misfit, observed=observed, traces=traces)
    check(lib().sbfwi_gradient(f, ck, _dptr(observed, torch.float64, "observed"),
                               _dptr(traces, torch.float64, "traces"), int(mode),
                               _dptr(misfit, torch.float64, "misfit"), _dptr(grad, torch.float64, "grad"),
                               _stream(stream)))


def sbfwi_misfit(observed, traces, dt, misfit, residual=None, stream=None):
    """misfit [1] = 1/2 dt sum (traces - observed)^2; residual (optional, like traces) = dt (traces - observed)."""
    import torch
    if observed.shape != traces.shape or (residual is not None and residual.shape != traces.shape):
        raise ValueError("observed, traces and residual must have the same shape")
    if misfit.numel() < 1:
        raise ValueError("misfit must hold one value")
    check(lib().sbfwi_misfit(_dptr(observed, torch.float64, "observed"), _dptr(traces, torch.float64, "traces"),
                             int(traces.numel()), float(dt),
                             _dptr(residual, torch.float64, "residual") if residual is not None else None,
                             _dptr(misfit, torch.float64, "misfit"), _stream(stream)))


def sbfwi_ckpt_info(ck: CkptHandle) -> dict:
    buf = np.zeros(6, dtype=np.int64)
    check(lib().sbfwi_ckpt_info(ck, buf.ctypes.data_as(C.c_void_p)))
    return {"bytes": int(buf[0]), "interval": int(buf[1]), "n_shots": int(buf[2]), "n_rec": int(buf[3]),
            "n_steps": int(buf[4]), "tail_steps": int(buf[5])}


def sbfwi_solver_stats(f: FactorsHandle, reset=False) -> dict:
    buf = np.zeros(3, dtype=np.int64)
    check(lib().sbfwi_solver_stats(f, buf.ctypes.data_as(C.c_void_p), int(bool(reset))))
    return {"solves": int(buf[0]), "iterations": int(buf[1]), "max_iterations": int(buf[2])}


PROFILE_KERNELS = ["condense", "recover", "coarse_solve", "source_gather", "nodal_update", "adj_condense",
                   "adj_recover", "adj_gather", "adj_nodal_update", "grad_exact", "grad_paper", "factor",
                   "solve_v", "solve_t", "solve_x", "solve_init", "recover_store", "fem_step", "joint",
                   "joint_store", "adj_joint"]


def sbfwi_profile(kernels):
    """Enable live event timing for the named kernels (or an int mask)."""
    mask = kernels if isinstance(kernels, int) else sum(1 << PROFILE_KERNELS.index(k) for k in kernels)
    check(lib().sbfwi_profile(mask))


def sbfwi_profile_read(reset=False) -> dict:
    buf = np.zeros(2 * len(PROFILE_KERNELS), dtype=np.float64)
    check(lib().sbfwi_profile_read(buf.ctypes.data_as(C.c_void_p), int(bool(reset))))
    return {name: {"launches": int(buf[2 * i]), "ms": float(buf[2 * i + 1])}
            for i, name in enumerate(PROFILE_KERNELS) if buf[2 * i] > 0}


def sbfwi_factors_info(f: FactorsHandle) -> dict:
    buf = np.zeros(1, dtype=np.int64)
    check(lib().sbfwi_factors_info(f, buf.ctypes.data_as(C.c_void_p)))
    return {"bytes": int(buf[0])}


__all__ = [n for n in dir() if n.startswith("sbfwi_")] + ["SbfwiError", "MeshHandle", "FactorsHandle",
                                                          "CkptHandle", "GRAD_EXACT", "GRAD_PAPER_KERNEL",
                                                          "GRAD_PER_SHOT"]

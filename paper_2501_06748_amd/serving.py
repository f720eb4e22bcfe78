"""Continuous-batching server of forward + adjoint shot requests (one GPU).

A request is one shot on one model: the forward run with sqrt(T)
checkpoints, the misfit of its traces against observed data and the exact
gradient of that misfit (the adjoint run), i.e. one shot's share of a
full-waveform-inversion gradient evaluation.

How requests flow:

* ``submit`` queues a request as it arrives.  The dispatcher forms *batches*:
  the oldest waiting request together with every other waiting request for
  the same model, step count and receivers (up to 16 shots) -- they run as
  one multi-shot launch sequence with one gradient per shot.
* Admission is by device-memory footprint: a batch is started only when its
  checkpoint store and work buffers (and the model's factors, unless they are
  already resident) fit in the memory budget next to the runs in flight and
  the cached factors.  Idle cached factors are evicted, least recently used
  first, when a new batch needs the room.
* Factored models stay on the device between requests (a model is factored
  once while it stays in the cache).
* ``slots`` worker threads each own a HIP stream; batches that are admitted
  while others run overlap on the device.  A batch whose model is already in
  use by another slot waits (the factors of one model serve one run at a
  time), so new requests for it join the next batch.
* Device memory of the library comes from PyTorch's caching allocator
  (``sbfwi_set_allocator``), so no run frees memory with a device-wide
  synchronisation.

Latency of a request = completion time - arrival time; throughput = shots
completed per second of the stream.
"""

from __future__ import annotations

import ctypes as C
import queue
import sys
import threading
import time
from collections import OrderedDict
from dataclasses import dataclass

import numpy as np
import torch

from . import (GRAD_EXACT, GRAD_PER_SHOT, LAUNCH_GRAPHS, sbfwi_build_mesh, sbfwi_factor_elements,
               sbfwi_forward, sbfwi_gradient, sbfwi_mesh_info, sbfwi_plan_bytes, sbfwi_set_launch)
from ._abi import check, lib

MAX_SHOTS = 16


# ---------------------------------------------------------------- planning (host logic only)

@dataclass
class Batch:
    key: tuple                    # (model key, n_steps, receiver count)
    requests: list
    factor_bytes: int             # bytes added to the cache by this batch (0 if the model was resident)
    run_bytes: int


@dataclass
class _CacheEntry:
    bytes: int
    busy: int = 0
    value: object = None          # the factored model once built


class BatchPlanner:
    """Batch formation, admission by footprint and the factor cache (no device calls).

    footprint(model_key, n_shots, n_steps) -> (factor_bytes, run_bytes)."""

    def __init__(self, budget_bytes: int, footprint, max_shots: int = MAX_SHOTS, batching: bool = True,
                 cache: bool = True):
        self.budget = int(budget_bytes)
        self.footprint = footprint
        self.max_shots = max_shots if batching else 1
        self.cache_on = cache
        self.pending = []
        self.cache = OrderedDict()            # model key -> _CacheEntry (LRU order)
        self.used = 0                         # cached factors + runs in flight
        self.running = 0

    @staticmethod
    def batch_key(req):
        return (req.model.key, req.n_steps, req.n_rec)

    def add(self, req):
        self.pending.append(req)

    def _evict_for(self, need, keep):
        for k in list(self.cache.keys()):
            if self.used + need <= self.budget:
                break
            e = self.cache[k]
            if e.busy == 0 and k != keep:
                self.used -= e.bytes
                del self.cache[k]
                yield e

    def next_batch(self):
        """The next admissible batch (removed from the queue), evicted cache entries, or (None, [])."""
        for i, r in enumerate(self.pending):
            mk = r.model.key
            ent = self.cache.get(mk)
            if ent is not None and ent.busy:
                continue                                  # model in use: its requests join a later batch
            key = self.batch_key(r)
            group = [q for q in self.pending[i:] if self.batch_key(q) == key][: self.max_shots]
            fb, rb = self.footprint(mk, len(group), r.n_steps)
            need = rb + (0 if ent is not None else fb)
            evicted = list(self._evict_for(need, mk)) if self.used + need > self.budget else []
            if self.used + need > self.budget and self.running > 0:
                return None, evicted                      # wait for memory (first-come order is kept)
            # alone on the device it runs even above the budget (nothing else can free memory)
            ids = {id(q) for q in group}
            self.pending = [q for q in self.pending if id(q) not in ids]
            if ent is None:
                ent = _CacheEntry(bytes=fb)
                self.cache[mk] = ent
                self.used += fb
            self.cache.move_to_end(mk)
            ent.busy += 1
            self.used += rb
            self.running += 1
            return Batch(key, group, fb if ent.value is None else 0, rb), evicted
        return None, []

    def finish(self, batch):
        """Releases a batch's run memory; without caching, its factors too (returns the entry to close)."""
        self.used -= batch.run_bytes
        self.running -= 1
        ent = self.cache[batch.key[0]]
        ent.busy -= 1
        if not self.cache_on and ent.busy == 0:
            self.used -= ent.bytes
            del self.cache[batch.key[0]]
            return ent
        return None


# ---------------------------------------------------------------- device memory from torch

_ALLOC_T = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_T = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
_callbacks = []


def use_torch_allocator(enable: bool = True):
    """Routes the library's device allocations through PyTorch's caching allocator
    (on the calling thread's current stream), or back to hipMalloc."""
    if not enable:
        check(lib().sbfwi_set_allocator(None, None, None))
        return

    def _alloc(nbytes, ctx):
        # the block comes from the current stream's pool; waiting for that stream makes it idle,
        # so the library may also use it on its own streams
        try:
            st = torch.cuda.current_stream()
            p = torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), st)
            st.synchronize()
            return p
        except Exception:
            return None

    def _free(ptr, ctx):
        if ptr:
            torch.cuda.caching_allocator_delete(ptr)

    cbs = (_ALLOC_T(_alloc), _FREE_T(_free))
    _callbacks.append(cbs)
    check(lib().sbfwi_set_allocator(C.cast(cbs[0], C.c_void_p), C.cast(cbs[1], C.c_void_p), None))


# ---------------------------------------------------------------- the server

@dataclass
class Result:
    rid: int
    traces: np.ndarray
    misfit: float
    grad: np.ndarray
    arrival: float
    start: float
    done: float
    batch_shots: int
    error: str = ""

    @property
    def latency(self):
        return self.done - self.arrival


@dataclass
class _Model:
    factors: object
    n_params: int


@dataclass
class _Host:
    """Host side of a model: mesh arrays, densities, recipe and the mesh handle
    (built once when its first request arrives; small next to the factors)."""
    mesh: object
    rho: np.ndarray
    recipe: object
    handle: object


class ShotServer:
    """slots: concurrent batches; budget_bytes: device memory budget (default 80 % of free);
    batching / cache / graphs: continuous batching, factor cache, graph replay of forward steps."""

    def __init__(self, slots=4, budget_bytes=None, batching=True, cache=True, graphs=True, keep_grad=True,
                 coarse_solver=1):
        self.coarse_solver = coarse_solver
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(0.8 * free)
        self.slots, self.graphs, self.keep_grad = slots, graphs, keep_grad
        self._fp_cache = {}
        self.planner = BatchPlanner(budget_bytes, self._footprint, batching=batching, cache=cache)
        self._lock = threading.Condition()
        self._work = queue.Queue()
        self._free_slots = slots
        self._results = {}
        self._t0 = None
        self._stop = False
        self._threads = []
        self._hosts = {}                      # model key -> (mesh arrays, rho) built on the host
        self.log = None                       # optional callable(str): a line per batch started and finished

    # footprint of (model, shots, steps): factors and run bytes from the library's plan
    def _footprint(self, mk, n_shots, n_steps):
        key = (mk, n_shots, n_steps)
        if key not in self._fp_cache:
            pb = sbfwi_plan_bytes(self._hosts[mk].handle, n_shots, n_steps, -1)
            self._fp_cache[key] = (pb["factors"], pb["checkpoints"] + max(pb["forward_work"], pb["backward_work"]))
        return self._fp_cache[key]

    def start(self):
        use_torch_allocator(True)
        self._t0 = time.perf_counter()
        for i in range(self.slots):
            t = threading.Thread(target=self._worker, name=f"slot{i}", daemon=True)
            t.start()
            self._threads.append(t)
        d = threading.Thread(target=self._dispatcher, name="dispatcher", daemon=True)
        d.start()
        self._threads.append(d)

    def now(self):
        return time.perf_counter() - self._t0

    def submit(self, req, arrival=None):
        if req.model.key not in self._hosts:
            mesh, rho = req.model.build()
            handle = sbfwi_build_mesh(mesh.node_xy, mesh.elem_ptr, mesh.elem_nodes, mesh.n_r)
            self._hosts[req.model.key] = _Host(mesh, rho, req.model, handle)
        req.t_arrival = self.now() if arrival is None else arrival
        with self._lock:
            self.planner.add(req)
            self._lock.notify_all()

    def _dispatcher(self):
        while True:
            with self._lock:
                while not self._stop:
                    batch = None
                    if self._free_slots > 0:
                        batch, evicted = self.planner.next_batch()
                        for e in evicted:
                            self._close_entry(e)
                    if batch is not None:
                        self._free_slots -= 1
                        self._work.put(batch)
                        continue
                    self._lock.wait(0.05)
                if self._stop:
                    return

    def _close_entry(self, ent):
        if ent.value is not None:
            ent.value.factors.close()
            ent.value = None

    def _build_model(self, mk, stream):
        h = self._hosts[mk]
        r = torch.tensor(h.rho, dtype=torch.float64, device="cuda")
        f = sbfwi_factor_elements(h.handle, r, h.recipe.c, h.recipe.dt, 0.25, 0.5, coarse_solver=self.coarse_solver,
                                  stream=stream)
        if self.graphs:
            sbfwi_set_launch(f, LAUNCH_GRAPHS, 1)
        return _Model(f, sbfwi_mesh_info(h.handle)["n_params"])

    def _cache_entry(self, mk):
        with self._lock:
            return self.planner.cache[mk]

    def _worker(self):
        stream = torch.cuda.Stream()
        while True:
            batch = self._work.get()
            if batch is None:
                return
            with torch.cuda.stream(stream):
                self._run_batch(batch, stream)
            with self._lock:
                closed = self.planner.finish(batch)
                if closed is not None:
                    self._close_entry(closed)
                self._free_slots += 1
                self._lock.notify_all()

    def _run_batch(self, batch, stream):
        start = self.now()
        reqs = batch.requests
        mk = reqs[0].model.key
        if self.log:
            self.log(f"[serving] batch of {len(reqs)} shot(s), {reqs[0].n_steps} steps, model {mk}: "
                     f"started at {start:.1f} s")
        ent = self._cache_entry(mk)
        err = ""
        try:
            if ent.value is None:
                ent.value = self._build_model(mk, stream)
            mdl = ent.value
            ins = [r.inputs(self._hosts[mk].mesh) for r in reqs]
            S, N, R = len(reqs), reqs[0].n_steps, len(ins[0][2])
            dev = "cuda"
            src = torch.tensor([i[0] for i in ins], dtype=torch.int64, device=dev)
            wav = torch.tensor(np.stack([i[1] for i in ins]), dtype=torch.float64, device=dev)
            rec = torch.tensor(ins[0][2], dtype=torch.int64, device=dev)
            obs = torch.tensor(np.stack([i[3] for i in ins]), dtype=torch.float64, device=dev)
            tr = torch.zeros((S, R, N), dtype=torch.float64, device=dev)
            ck = sbfwi_forward(mdl.factors, src, wav, rec, tr, n_ckpt=-1, stream=stream)
            mis = torch.zeros(S, dtype=torch.float64, device=dev)
            grad = torch.zeros((S, mdl.n_params), dtype=torch.float64, device=dev)
            sbfwi_gradient(mdl.factors, ck, obs, tr, GRAD_EXACT | GRAD_PER_SHOT, mis, grad, stream=stream)
            ck.close()
            tr_h, mis_h = tr.cpu().numpy(), mis.cpu().numpy()
            grad_h = grad.cpu().numpy() if self.keep_grad else None
        except Exception as e:          # reported per request; the server keeps running
            err = f"{type(e).__name__}: {e}"
        done = self.now()
        if self.log:
            self.log(f"[serving] batch of {len(reqs)} shot(s), model {mk}: finished at {done:.1f} s"
                     + (f" ({err})" if err else ""))
        with self._lock:
            for i, r in enumerate(reqs):
                if err:
                    self._results[r.rid] = Result(r.rid, None, float("nan"), None, r.t_arrival, start, done, len(reqs),
                                                  err)
                else:
                    self._results[r.rid] = Result(r.rid, tr_h[i], float(mis_h[i]),
                                                  grad_h[i] if grad_h is not None else None, r.t_arrival, start,
                                                  done, len(reqs))
            self._lock.notify_all()

    def wait(self, n, timeout=None):
        """Blocks until n results exist; returns them by request id."""
        end = None if timeout is None else time.perf_counter() + timeout
        with self._lock:
            while len(self._results) < n:
                left = None if end is None else end - time.perf_counter()
                if left is not None and left <= 0:
                    raise TimeoutError(f"{len(self._results)} of {n} results")
                self._lock.wait(0.05 if left is None else min(0.05, left))
            return dict(self._results)

    def stop(self):
        with self._lock:
            self._stop = True
            self._lock.notify_all()
        for _ in range(self.slots):
            self._work.put(None)
        for t in self._threads:
            t.join(timeout=60)
        torch.cuda.synchronize()
        for ent in list(self.planner.cache.values()):
            self._close_entry(ent)
        for h in self._hosts.values():
            h.handle.close()
        use_torch_allocator(False)


def run_stream(server, requests, time_scale=1.0):
    """Submits requests at their arrival times (scaled) and waits for all results."""
    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if len(requests) <= 64:      # a line per arrival and per batch while the stream runs
        server.log = log
    server.start()
    t0 = server.now()
    for r in sorted(requests, key=lambda q: q.arrival):
        delay = t0 + r.arrival * time_scale - server.now()
        if delay > 0:
            time.sleep(delay)
        server.submit(r)
        if server.log:
            log(f"[serving] request {r.rid} arrived at {server.now():.1f} s")
    res = {}
    step = 1 if len(requests) <= 64 else len(requests) // 8
    for k in range(step, len(requests) + step, step):     # progress lines while waiting
        res = server.wait(min(k, len(requests)))
        log(f"[serving] {len(res)}/{len(requests)} requests done at {server.now():.1f} s")
    server.stop()
    return res


def summarize(results, requests):
    lat = np.array([results[r.rid].latency for r in requests])
    first = min(results[r.rid].arrival for r in requests)
    last = max(results[r.rid].done for r in requests)
    return {"requests": len(requests), "errors": sum(1 for r in requests if results[r.rid].error),
            "shots_per_s": len(requests) / (last - first), "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_batch_shots": float(np.mean(
                [results[r.rid].batch_shots for r in requests])), "span_s": last - first}


def main(argv=None):
    """Serving measurement: plain serial capacity, then the server at 0.5x and
    0.9x of it (Poisson arrivals) and saturated; prints progress and one JSON line.
    --phases selects the parts (plain, 0.5, 0.9, saturated); without the plain
    phase --capacity gives the plain path's shots/s that sets the arrival rates."""
    import argparse
    import json
    import os
    import sys
    ap = argparse.ArgumentParser(description="continuous-batching shot server measurement")
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--scale", default="reduced")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--phases", default="plain,0.5,0.9,saturated")
    ap.add_argument("--capacity", type=float, default=0.0, help="plain-path shots/s (when plain is not run)")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from workloads.serving import serving_requests

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    phases = [p.strip() for p in args.phases.split(",") if p.strip()]
    base = serving_requests(args.requests, scale=args.scale, rate=1.0)
    out = {"requests": args.requests, "scale": args.scale, "slots": args.slots}
    cap = args.capacity
    if "plain" in phases:
        # plain path: one request at a time, no batching, no cache, ordinary launches
        srv = ShotServer(slots=1, batching=False, cache=False, graphs=False, keep_grad=False)
        res = run_stream(srv, [_at(r, 0.0) for r in base])
        plain = summarize(res, base)
        out["plain_serial"] = plain
        cap = plain["shots_per_s"]
        log(f"[serving] plain serial: {plain}")
    for frac in (0.5, 0.9):
        if str(frac) not in phases:
            continue
        if not cap > 0:
            raise SystemExit("the load phases need the plain capacity (--capacity or the plain phase)")
        reqs = serving_requests(args.requests, scale=args.scale, rate=frac * cap)
        srv = ShotServer(slots=args.slots, keep_grad=False)
        res = run_stream(srv, reqs)
        out[f"server_at_{frac}x_plain"] = dict(summarize(res, reqs), arrival_rate=frac * cap)
        log(f"[serving] server at {frac} x plain capacity: {out[f'server_at_{frac}x_plain']}")
    if "saturated" in phases:
        srv = ShotServer(slots=args.slots, keep_grad=False)
        res = run_stream(srv, [_at(r, 0.0) for r in base])
        out["server_saturated"] = summarize(res, base)
        log(f"[serving] saturated: {out['server_saturated']}")
    out["plain_capacity_shots_per_s"] = cap
    print(json.dumps(out))


def _at(req, t):
    import copy
    q = copy.copy(req)
    q.arrival = t
    return q


if __name__ == "__main__":
    main()

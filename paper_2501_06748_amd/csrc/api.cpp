// Exported C ABI: argument checks, handle lifetimes, the forward driver with
// checkpointing, and error reporting.  Every computation runs in the HIP
// kernels of factor.hip, step.hip, coarse.hip and adjoint.hip.
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "sbfwi_internal.h"

static thread_local char g_err[1024] = "";

// The registered allocator, and for every live allocation the deallocator of
// the allocator that made it (so that switching allocators while handles are
// alive frees each block where it came from).
struct Allocator {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free)(void*, void*) = nullptr;
  void* ctx = nullptr;
};
static std::mutex g_alloc_mu;
static Allocator g_allocator;
static std::unordered_map<void*, Allocator> g_owner;

int sbfwi_fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

void* sbfwi_dev_alloc(size_t bytes) {
  Allocator a;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    a = g_allocator;
  }
  void* p = nullptr;
  if (a.alloc) {
    p = a.alloc(bytes, a.ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (p) {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_owner[p] = a;
  }
  return p;
}

void sbfwi_dev_free(void* p) {
  if (!p) return;
  Allocator a;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    auto it = g_owner.find(p);
    if (it != g_owner.end()) {
      a = it->second;
      g_owner.erase(it);
    }
  }
  if (a.free)
    a.free(p, a.ctx);
  else
    (void)hipFree(p);
}

void sbfwi_factors_free(sbfwi_factors_s* f);

// The tail store of a checkpointed run (hundreds of GiB: an allocation of that size
// takes seconds) is kept when its run is destroyed and handed to the next run on the
// same device that fits in it; sbfwi_finalize releases it.
static std::mutex g_tail_mu;
static struct {
  void* p = nullptr;
  size_t bytes = 0;
  int device = -1;
} g_tail;

static void* tail_take(size_t bytes) {
  int dev = -1;
  (void)hipGetDevice(&dev);
  {
    std::lock_guard<std::mutex> lk(g_tail_mu);
    if (g_tail.p && g_tail.device == dev && g_tail.bytes >= bytes) {
      void* p = g_tail.p;
      g_tail = {};
      return p;
    }
  }
  return sbfwi_dev_alloc(bytes);
}

static void tail_give(void* p, size_t bytes) {
  if (!p) return;
  int dev = -1;
  (void)hipGetDevice(&dev);
  void* drop = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_tail_mu);
    if (g_tail.p && g_tail.bytes >= bytes && g_tail.device == dev) {
      drop = p;   // keep the larger one
    } else {
      drop = g_tail.p;
      g_tail.p = p;
      g_tail.bytes = bytes;
      g_tail.device = dev;
    }
  }
  sbfwi_dev_free(drop);
}

static void tail_release() {
  void* p = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_tail_mu);
    p = g_tail.p;
    g_tail = {};
  }
  sbfwi_dev_free(p);
}

// One non-blocking stream per host thread for the library's synchronous copies,
// created on first use and registered so that sbfwi_finalize can destroy them
// all; a thread's cached stream is recreated after a finalize (generation count).
static std::mutex g_aux_mu;
static std::vector<hipStream_t> g_aux_streams;
static std::atomic<int> g_aux_gen{0};

static hipStream_t aux_stream() {
  thread_local hipStream_t s = nullptr;
  thread_local int gen = -1;
  const int cur = g_aux_gen.load();
  if (s && gen == cur) return s;
  s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return s = nullptr;
  gen = cur;
  std::lock_guard<std::mutex> lk(g_aux_mu);
  g_aux_streams.push_back(s);
  return s;
}

int sbfwi_prof_release();

static void tail_release();

extern "C" int sbfwi_finalize(void) {
  SBFWI_HIP(hipDeviceSynchronize());
  tail_release();
  int rc = sbfwi_prof_release();
  std::lock_guard<std::mutex> lk(g_aux_mu);
  g_aux_gen.fetch_add(1);
  for (hipStream_t st : g_aux_streams)
    if (hipStreamDestroy(st) != hipSuccess && rc == SBFWI_OK) rc = sbfwi_fail(SBFWI_EHIP, "hipStreamDestroy failed");
  g_aux_streams.clear();
  return rc;
}

int sbfwi_copy_sync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  hipStream_t s = aux_stream();
  if (!s) return sbfwi_fail(SBFWI_EHIP, "cannot create the copy stream");
  SBFWI_HIP(hipMemcpyAsync(dst, src, bytes, kind, s));
  SBFWI_HIP(hipStreamSynchronize(s));
  return SBFWI_OK;
}

int sbfwi_zero_sync(void* dst, size_t bytes) {
  hipStream_t s = aux_stream();
  if (!s) return sbfwi_fail(SBFWI_EHIP, "cannot create the copy stream");
  SBFWI_HIP(hipMemsetAsync(dst, 0, bytes, s));
  SBFWI_HIP(hipStreamSynchronize(s));
  return SBFWI_OK;
}

extern "C" const char* sbfwi_last_error(void) { return g_err; }

extern "C" int sbfwi_set_allocator(void* (*alloc_fn)(size_t, void*), void (*free_fn)(void*, void*), void* ctx) {
  if ((alloc_fn == nullptr) != (free_fn == nullptr))
    return sbfwi_fail(SBFWI_EINVAL, "allocator and deallocator must be given together");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_allocator.alloc = alloc_fn;
  g_allocator.free = free_fn;
  g_allocator.ctx = ctx;
  return SBFWI_OK;
}

extern "C" int sbfwi_factor_elements(sbfwi_mesh m, const double* rho, double c, double dt, double beta,
                                     double gamma, int scheme, int coarse_solver, hipStream_t s,
                                     sbfwi_factors* out) {
  if (!out) return sbfwi_fail(SBFWI_EINVAL, "out is NULL");
  *out = nullptr;
  if (!m || !rho) return sbfwi_fail(SBFWI_EINVAL, "NULL mesh or density");
  if (!(c > 0) || !(dt > 0) || !(beta > 0) || !(gamma > 0))
    return sbfwi_fail(SBFWI_EINVAL, "c, dt, beta and gamma must be positive");
  if (scheme != SBFWI_SCHEME_PAPER_FD && scheme != SBFWI_SCHEME_RADIAL_GALERKIN && !sbfwi_is_lfe(scheme))
    return sbfwi_fail(SBFWI_EINVAL, "unknown radial scheme %d", scheme);
  if (coarse_solver != 0 && coarse_solver != 1)
    return sbfwi_fail(SBFWI_EINVAL, "unknown coarse solver %d", coarse_solver);
  return sbfwi_factor_impl(m, rho, c, dt, beta, gamma, scheme, coarse_solver, s, out);
}

extern "C" int sbfwi_set_solver(sbfwi_factors f, double rtol, int max_iter) {
  if (!f || !(rtol > 0) || max_iter <= 0) return sbfwi_fail(SBFWI_EINVAL, "bad solver controls");
  f->rtol = rtol;
  f->max_iter = max_iter;
  return SBFWI_OK;
}

int sbfwi_device_cus() {
  static std::atomic<int> cached{0};
  int cus = cached.load();
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 1;
    cached.store(cus);
  }
  return cus;
}

static bool valid_shots_per_block(int v) { return v == 0 || v == 1 || v == 2 || v == 4 || v == 8 || v == 16; }

extern "C" int sbfwi_set_launch(sbfwi_factors f, int param, int value) {
  if (!f) return sbfwi_fail(SBFWI_EINVAL, "NULL factors");
  if (param == 0) {
    if (value < 1 || value > 1000) return sbfwi_fail(SBFWI_EINVAL, "enqueued iterations must be in 1..1000");
    f->enqueued_iters = value;
    return SBFWI_OK;
  }
  if (param == 1) {
    if (value != 0 && value != 1) return sbfwi_fail(SBFWI_EINVAL, "graph replay flag must be 0 or 1");
    f->use_graphs = value;
    return SBFWI_OK;
  }
  if (param == 2) {
    f->plan = SweepPlan();
    return SBFWI_OK;
  }
  if (param == 3) {
    if (value != 0 && value != 1) return sbfwi_fail(SBFWI_EINVAL, "overlap flag must be 0 or 1");
    f->overlap_adjoint = value;
    return SBFWI_OK;
  }
  if (param == 4) {
    if (value != 0 && value != 1) return sbfwi_fail(SBFWI_EINVAL, "solution store flag must be 0 or 1");
    f->keep_solutions = value;
    return SBFWI_OK;
  }
  if (param == 6) {
    if (value < 1) return sbfwi_fail(SBFWI_EINVAL, "the subtree cut needs at least 1 supernode per level");
    if (!f->dnum) return sbfwi_fail(SBFWI_EINVAL, "the subtree cut applies to the direct coarse solver");
    SBFWI_HIP(hipDeviceSynchronize());   // no solve may be reading the programs being replaced
    return sbfwi_direct_programs(f->m, value);
  }
  if (param == 5) {
    if (value != 0 && value != 1) return sbfwi_fail(SBFWI_EINVAL, "joint sweep flag must be 0 or 1");
    f->joint_sweeps = value;
    return SBFWI_OK;
  }
  if (param == 8) {
    if (value < 0) return sbfwi_fail(SBFWI_EINVAL, "tail store budget must be >= 0 KiB");
    f->tail_kib = value;
    return SBFWI_OK;
  }
  if (param == 7) {
    if (value != 0 && value != 1) return sbfwi_fail(SBFWI_EINVAL, "row formation flag must be 0 or 1");
    f->d.fly = value;
    return SBFWI_OK;
  }

  if (param >= 10 && param < 10 + 3 * SW_N) {
    if (!valid_shots_per_block(value)) return sbfwi_fail(SBFWI_EINVAL, "shots per block must be 0, 1, 2, 4, 8 or 16");
    f->plan.S[(param - 10) / 3][(param - 10) % 3] = value;
    return SBFWI_OK;
  }
  if (param >= 30 && param < 30 + SW_N) {
    if (!valid_shots_per_block(value)) return sbfwi_fail(SBFWI_EINVAL, "shots per block must be 0, 1, 2, 4, 8 or 16");
    f->plan.fusedS[param - 30] = value;
    return SBFWI_OK;
  }
  return sbfwi_fail(SBFWI_EINVAL, "unknown launch parameter %d", param);
}

extern "C" int sbfwi_plan_bytes(sbfwi_mesh m, int n_shots, int64_t n_steps, int n_ckpt, int64_t* out) {
  if (!m || !out) return sbfwi_fail(SBFWI_EINVAL, "NULL argument");
  if (n_shots <= 0 || n_shots > 16 || n_steps <= 0 || n_ckpt < -1)
    return sbfwi_fail(SBFWI_EINVAL, "bad shot, step or checkpoint count");
  const int64_t NS = n_shots;
  const int64_t n_slices = (m->n_nodes + ELL_SLICE - 1) / ELL_SLICE;
  // the allocations of factor.hip, step.hip, coarse.hip, adjoint.hip and api.cpp
  // (the central-difference scheme's kappa and density copy: 27 n_loop + n_params)
  const int64_t factors = 8 * (m->n_finv + 10 * m->n_params + 36 * m->n_loop + 6 * m->n_dense + 32 * m->n_loop +
                               2 * m->nnz + 2 * m->d.n_ell + m->n_nodes) + 32;
  const int64_t coarse = 8 * (9 * m->n_nodes * NS + 4 * n_slices * 3 * NS + 3 * 11 * 16) +
                         4 * (64 + 32 * (n_slices / 16 + 2));
  const int64_t state = 8 * sbfwi_state_size(m, (int)NS);
  const int64_t fwd_work = state + 8 * NS * (m->n_int + 2 * m->n_loop + 2 * m->n_nodes) + coarse + 8 +
                           8 * NS * n_steps;   // the growth envelope
  int64_t ckpt = 8 * NS * n_steps + 16 * NS + 8 * 64;   // copies of sources, wavelets, receivers (bounded)
  int64_t interval = 1;
  if (n_ckpt >= n_steps) {
    ckpt += 8 * n_steps * (m->n_x + 2 * m->n_params) * NS;
  } else if (n_ckpt != 0) {
    int64_t cnt = n_ckpt > 0 ? n_ckpt : (int64_t)std::ceil(std::sqrt((double)n_steps));
    interval = (n_steps + cnt - 1) / cnt;
    ckpt += ((n_steps + interval - 1) / interval) * state;
    ckpt += 8 * n_steps * m->n_nodes * NS;   // the coarse solutions kept for the recompute
  }
  int64_t bwd = 0;
  if (n_ckpt != 0) {
    // (+ the paper kernel's back-propagated velocity field, n_params per shot)
    bwd = 8 * NS * (3 * m->n_int + 3 * m->n_nodes + m->n_int + 2 * m->n_loop + 2 * m->n_nodes + m->n_x +
                    m->n_params) +
          coarse + 4 * m->n_params;
    // the segment recompute: its work buffers and two segment stores (the second one
    // when the recompute of the next segment overlaps the adjoint of the current one)
    if (n_ckpt < n_steps) bwd += fwd_work + 2 * 8 * interval * NS * (m->n_x + m->n_params);
    bwd += 8 * NS * n_steps * 64;   // residual of sbfwi_gradient, receivers bounded by 64 per shot
  }
  out[0] = factors;
  out[1] = ckpt;
  out[2] = fwd_work;
  out[3] = bwd;
  return SBFWI_OK;
}

extern "C" int sbfwi_autotune(sbfwi_factors f, int n_shots, double* host_out, hipStream_t s) {
  if (!f) return sbfwi_fail(SBFWI_EINVAL, "NULL factors");
  if (n_shots <= 0 || n_shots > 16) return sbfwi_fail(SBFWI_EINVAL, "n_shots must be in 1..16");
  SBFWI_CHECK(sbfwi_tune_step_sweeps(f, n_shots, s, host_out));
  return sbfwi_tune_adj_sweeps(f, n_shots, s, host_out);
}

extern "C" int sbfwi_copy_factor_data(sbfwi_factors f, int which, double* dst) {
  if (!f || !dst) return sbfwi_fail(SBFWI_EINVAL, "NULL argument");
  const double* src = nullptr;
  int64_t n = 0;
  switch (which) {
    case 0: src = f->d.S; n = f->m->n_dense; break;
    case 1: src = f->d.Kval; n = f->m->nnz; break;
    case 2: src = f->d.finv; n = f->m->n_finv; break;
    case 3: src = f->d.G; n = f->m->n_dense; break;
    case 4:
    case 5:
      if (!sbfwi_is_lfe(f->scheme))
        return sbfwi_fail(SBFWI_EINVAL, "factor data %d exists for the expansion schemes only", which);
      src = which == 4 ? f->d.Me : f->d.Mval;
      n = which == 4 ? f->m->n_dense : f->m->nnz;
      break;
    default: return sbfwi_fail(SBFWI_EINVAL, "unknown factor data %d", which);
  }
  SBFWI_CHECK(sbfwi_copy_sync(dst, src, n * sizeof(double), hipMemcpyDeviceToHost));
  return SBFWI_OK;
}

extern "C" int sbfwi_solver_stats(sbfwi_factors f, int64_t* out, int reset) {
  if (!f || !out) return sbfwi_fail(SBFWI_EINVAL, "NULL argument");
  int st[8];
  SBFWI_CHECK(sbfwi_copy_sync(st, f->d.status, sizeof(st), hipMemcpyDeviceToHost));
  out[0] = st[5];
  out[1] = st[4];
  out[2] = st[3];
  if (reset) {
    int z[3] = {0, 0, 0};
    SBFWI_CHECK(sbfwi_copy_sync(f->d.status + 3, z, sizeof(z), hipMemcpyHostToDevice));
  }
  return SBFWI_OK;
}

extern "C" int sbfwi_factors_info(sbfwi_factors f, int64_t* out) {
  if (!f || !out) return sbfwi_fail(SBFWI_EINVAL, "NULL argument");
  out[0] = f->bytes;
  return SBFWI_OK;
}

extern "C" void sbfwi_destroy_factors(sbfwi_factors f) { sbfwi_factors_free(f); }

static void ckpt_free(sbfwi_ckpt_s* ck) {
  if (!ck) return;
  sbfwi_dev_free(ck->src_node);
  sbfwi_dev_free(ck->wavelet);
  sbfwi_dev_free(ck->rec_node);
  sbfwi_dev_free(ck->states);
  sbfwi_dev_free(ck->xstore);
  tail_give(ck->tail_x, ck->tail_bytes);   // tail_f lies in the same allocation
  sbfwi_dev_free(ck->fstore);
  sbfwi_dev_free(ck->vstore);
  sbfwi_dev_free(ck->ustore);
  delete ck;
}

extern "C" void sbfwi_destroy_ckpt(sbfwi_ckpt ck) { ckpt_free(ck); }

extern "C" int sbfwi_ckpt_info(sbfwi_ckpt ck, int64_t* out) {
  if (!ck || !out) return sbfwi_fail(SBFWI_EINVAL, "NULL argument");
  out[0] = ck->bytes;
  out[1] = ck->interval;
  out[2] = ck->n_shots;
  out[3] = ck->n_rec;
  out[4] = ck->n_steps;
  out[5] = ck->n_steps - (ck->tail_x ? ck->tail_k0 : ck->n_steps);
  return SBFWI_OK;
}

static int read_status(sbfwi_factors_s* f, hipStream_t s, const char* what) {
  int flags[4] = {0, -1, 0, 0};
  SBFWI_HIP(hipMemcpyAsync(flags, f->d.status, sizeof(flags), hipMemcpyDeviceToHost, s));
  SBFWI_HIP(hipStreamSynchronize(s));
  if (flags[0] & 8) return sbfwi_fail(SBFWI_EHIP, "%s: coarse-solve grid barrier timed out", what);
  if (flags[0] & 32)
    return sbfwi_fail(SBFWI_ENONFINITE, "%s: non-finite nodal displacement at step %d", what, flags[1]);
  if (flags[0] & 16)
    return sbfwi_fail(SBFWI_EUNSTABLE, "%s: nodal displacement beyond the growth envelope at step %d", what,
                      flags[1]);
  if (flags[0] & 4) return sbfwi_fail(SBFWI_ENONFINITE, "%s: non-finite coarse residual at step %d", what, flags[1]);
  if (flags[0] & 2) return sbfwi_fail(SBFWI_ENOCONV, "%s: coarse solve did not converge at step %d", what, flags[1]);
  return SBFWI_OK;
}

static int forward_run(sbfwi_factors_s* f, int n_shots, int64_t n_steps, const int64_t* src_node,
                       const double* wavelet, int n_rec, const int64_t* rec_node, double* traces, int n_ckpt,
                       sbfwi_ckpt_s* ck, hipStream_t s, StepWork& w) {
  sbfwi_mesh_s* m = f->m;
  SBFWI_CHECK(sbfwi_step_work_alloc(&w, m, n_shots));
  SBFWI_CHECK(sbfwi_step_zero(m, &w, s));
  {
    // growth envelope of the nodal displacement: kEnvelopeSafety * 4 k r F_k per shot and step
    // (the wavelet was made ready on s by the caller; s was synchronised by the node checks)
    std::vector<double> wav((size_t)n_shots * n_steps), env((size_t)n_shots * n_steps);
    SBFWI_HIP(hipMemcpyAsync(wav.data(), wavelet, wav.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    SBFWI_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < n_shots; ++q) {
      double F = 0.0;
      for (int64_t k = 1; k <= n_steps; ++k) {
        F += std::fabs(wav[(size_t)q * n_steps + k - 1]);
        env[(size_t)(k - 1) * n_shots + q] = kEnvelopeSafety * 4.0 * (double)k * f->env_r * F;
      }
    }
    SBFWI_CHECK(sbfwi_upload(&w.env, env));
  }
  int flags0[4] = {0, -1, 0, 0};
  SBFWI_HIP(hipMemcpyAsync(f->d.status, flags0, 2 * sizeof(int), hipMemcpyHostToDevice, s));
  const int64_t ssz = sbfwi_state_size(m, n_shots);
  if (ck) {
    ck->f = f;
    ck->n_shots = n_shots;
    ck->n_rec = n_rec;
    ck->n_steps = n_steps;
    SBFWI_CHECK(sbfwi_alloc(&ck->src_node, n_shots));
    SBFWI_CHECK(sbfwi_alloc(&ck->wavelet, (int64_t)n_shots * n_steps));
    SBFWI_CHECK(sbfwi_alloc(&ck->rec_node, n_rec > 0 ? n_rec : 1));
    SBFWI_HIP(hipMemcpyAsync(ck->src_node, src_node, n_shots * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    SBFWI_HIP(hipMemcpyAsync(ck->wavelet, wavelet, (size_t)n_shots * n_steps * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    if (n_rec > 0)
      SBFWI_HIP(hipMemcpyAsync(ck->rec_node, rec_node, n_rec * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    if (n_ckpt >= n_steps) {
      ck->full_store = true;
      ck->interval = 1;
      SBFWI_CHECK(sbfwi_alloc(&ck->xstore, n_steps * m->n_x * n_shots));
      SBFWI_CHECK(sbfwi_alloc(&ck->fstore, n_steps * m->n_params * n_shots));
      SBFWI_CHECK(sbfwi_alloc(&ck->vstore, n_steps * m->n_params * n_shots));
      ck->bytes = 8 * n_steps * (m->n_x + 2 * m->n_params) * n_shots;
    } else {
      int64_t cnt = n_ckpt > 0 ? n_ckpt : (int64_t)std::ceil(std::sqrt((double)n_steps));
      ck->interval = (n_steps + cnt - 1) / cnt;
      ck->n_saved = (n_steps + ck->interval - 1) / ck->interval;
      SBFWI_CHECK(sbfwi_alloc(&ck->states, ck->n_saved * ssz));
      ck->bytes = 8 * ck->n_saved * ssz;
      // every step's coarse solution, for a recompute without coarse solves (skipped if it does not fit)
      if (f->keep_solutions && n_steps > ck->interval) {
        if (sbfwi_alloc(&ck->ustore, n_steps * m->n_nodes * n_shots) == SBFWI_OK)
          ck->bytes += 8 * n_steps * m->n_nodes * n_shots;
        else
          (void)hipGetLastError();
      }
      // the tail store: as many whole segments at the end of the run as the budget holds
      // (skipped if it does not fit)
      ck->tail_k0 = n_steps;
      const int64_t per_step = 8 * (m->n_x + m->n_params) * n_shots;
      const int64_t segs = std::min(f->tail_kib * 1024 / per_step / ck->interval, ck->n_saved);
      if (segs > 0) {
        const int64_t k0 = std::max<int64_t>(0, (ck->n_saved - segs) * ck->interval), ns = n_steps - k0;
        ck->tail_x = (double*)tail_take((size_t)(ns * per_step));
        if (ck->tail_x) {
          ck->tail_f = ck->tail_x + ns * m->n_x * n_shots;
          ck->tail_bytes = (size_t)(ns * per_step);
          ck->tail_k0 = k0;
          ck->bytes += ns * per_step;
        } else {
          (void)hipGetLastError();
        }
      }
    }
  }
  w.ustore = ck ? ck->ustore : nullptr;
  SourceTable src;
  src.n_src = 1;
  src.node = src_node;
  src.node_stride = 1;
  src.amp = wavelet;
  src.amp_steps = n_steps;
  const bool graphs = f->use_graphs && !(ck && (ck->full_store || ck->tail_x));
  if (graphs) SBFWI_CHECK(sbfwi_graph_step_reset(&w, 1, s));
  for (int64_t k = 1; k <= n_steps; ++k) {
    double *xs = nullptr, *fs = nullptr, *vs = nullptr;
    if (ck && !ck->full_store && (k - 1) % ck->interval == 0)
      SBFWI_CHECK(sbfwi_state_copy(m, &w, ck->states + ((k - 1) / ck->interval) * ssz, 1, s));
    if (graphs) {
      SBFWI_CHECK(sbfwi_forward_step_graph(f, &w, src, n_rec, rec_node, traces, n_steps, s));
      continue;
    }
    if (ck && ck->full_store) {
      xs = ck->xstore + (k - 1) * m->n_x * n_shots;
      fs = ck->fstore + (k - 1) * m->n_params * n_shots;
      vs = ck->vstore + (k - 1) * m->n_params * n_shots;
    } else if (ck && ck->tail_x && k > ck->tail_k0) {
      xs = ck->tail_x + (k - ck->tail_k0 - 1) * m->n_x * n_shots;
      fs = ck->tail_f + (k - ck->tail_k0 - 1) * m->n_params * n_shots;
    }
    SBFWI_CHECK(sbfwi_forward_step(f, &w, k, src, n_rec, rec_node, traces, n_steps, xs, fs, 0, s, vs, nullptr,
                                   k < n_steps));
  }
  return read_status(f, s, "forward");
}

extern "C" int sbfwi_forward(sbfwi_factors f, int n_shots, int64_t n_steps, const int64_t* src_node,
                             const double* wavelet, int n_rec, const int64_t* rec_node, double* traces,
                             int n_ckpt, sbfwi_ckpt* ckpt_out, hipStream_t s) {
  if (ckpt_out) *ckpt_out = nullptr;
  if (!f) return sbfwi_fail(SBFWI_EINVAL, "NULL factors");
  if (n_shots <= 0 || n_shots > 16) return sbfwi_fail(SBFWI_EINVAL, "n_shots must be in 1..16");
  if (n_steps <= 0) return sbfwi_fail(SBFWI_EINVAL, "n_steps must be positive");
  if (!src_node || !wavelet) return sbfwi_fail(SBFWI_EINVAL, "NULL source arrays");
  if (n_rec < 0 || (n_rec > 0 && (!rec_node || !traces))) return sbfwi_fail(SBFWI_EINVAL, "bad receivers");
  if (n_ckpt != 0 && !ckpt_out) return sbfwi_fail(SBFWI_EINVAL, "checkpoints requested but ckpt_out is NULL");
  if (n_ckpt < -1) return sbfwi_fail(SBFWI_EINVAL, "n_ckpt must be >= -1");

  // node ids are checked on the host (small arrays)
  {
    std::vector<int64_t> h(n_shots);
    SBFWI_HIP(hipMemcpyAsync(h.data(), src_node, n_shots * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SBFWI_HIP(hipStreamSynchronize(s));
    for (int64_t v : h)
      if (v < 0 || v >= f->m->n_nodes) return sbfwi_fail(SBFWI_EINVAL, "source node %lld out of range", (long long)v);
    std::vector<int64_t> r(n_rec);
    if (n_rec > 0)
      SBFWI_HIP(hipMemcpyAsync(r.data(), rec_node, n_rec * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (n_rec > 0) SBFWI_HIP(hipStreamSynchronize(s));
    for (int64_t v : r)
      if (v < 0 || v >= f->m->n_nodes) return sbfwi_fail(SBFWI_EINVAL, "receiver node %lld out of range", (long long)v);
  }
  if (sbfwi_is_lfe(f->scheme)) {
    // any n_ckpt != 0 keeps every step's nodal velocity (the paper-kernel gradient needs them all)
    sbfwi_ckpt_s* ck = nullptr;
    double* vstore = nullptr;
    if (n_ckpt != 0) {
      ck = new sbfwi_ckpt_s();
      ck->f = f;
      ck->n_shots = n_shots;
      ck->n_rec = n_rec;
      ck->n_steps = n_steps;
      ck->interval = 1;
      ck->full_store = true;
      int rc = sbfwi_alloc(&ck->rec_node, n_rec > 0 ? n_rec : 1);
      if (rc == SBFWI_OK) rc = sbfwi_alloc(&ck->vstore, n_steps * f->m->n_nodes * n_shots);
      if (rc == SBFWI_OK && n_rec > 0 &&
          hipMemcpyAsync(ck->rec_node, rec_node, n_rec * sizeof(int64_t), hipMemcpyDeviceToDevice, s) != hipSuccess)
        rc = sbfwi_fail(SBFWI_EHIP, "hipMemcpyAsync failed");
      if (rc != SBFWI_OK) {
        ckpt_free(ck);
        return rc;
      }
      ck->bytes = 8 * n_steps * f->m->n_nodes * n_shots;
      vstore = ck->vstore;
    }
    int rc = sbfwi_lfe_forward(f, n_shots, n_steps, src_node, wavelet, n_rec, rec_node, traces, vstore, s);
    if (rc != SBFWI_OK) {
      ckpt_free(ck);
      return rc;
    }
    if (ckpt_out) *ckpt_out = ck;
    return SBFWI_OK;
  }
  sbfwi_ckpt_s* ck = n_ckpt != 0 ? new sbfwi_ckpt_s() : nullptr;
  StepWork w;
  // graph replay needs a stream that can be captured: the run goes to a
  // library stream (default priority) ordered after the caller's work
  hipStream_t rs = s;
  hipStream_t own = nullptr;
  if (f->use_graphs) {
    SBFWI_HIP(hipStreamSynchronize(s));
    SBFWI_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
    rs = own;
  }
  int rc = forward_run(f, n_shots, n_steps, src_node, wavelet, n_rec, rec_node, traces, n_ckpt, ck, rs, w);
  (void)hipStreamSynchronize(rs);
  sbfwi_step_work_free(&w);
  if (own) (void)hipStreamDestroy(own);
  if (rc != SBFWI_OK) {
    ckpt_free(ck);
    return rc;
  }
  if (ckpt_out) *ckpt_out = ck;
  return SBFWI_OK;
}

extern "C" int sbfwi_adjoint(sbfwi_factors f, sbfwi_ckpt ck, const double* adj_src, int mode, double* grad,
                             hipStream_t s) {
  if (!f || !ck || !grad || (!adj_src && ck->n_rec > 0)) return sbfwi_fail(SBFWI_EINVAL, "NULL argument");
  if (ck->f != f) return sbfwi_fail(SBFWI_EINVAL, "checkpoints belong to other factors");
  const int base = mode & ~SBFWI_GRAD_PER_SHOT;
  if (base != SBFWI_GRAD_EXACT && base != SBFWI_GRAD_PAPER_KERNEL) return sbfwi_fail(SBFWI_EINVAL, "unknown mode");
  if (sbfwi_is_lfe(f->scheme) && base != SBFWI_GRAD_PAPER_KERNEL)
    return sbfwi_fail(SBFWI_EINVAL, "the expansion schemes provide the paper-kernel gradient only");
  if (ck->n_rec == 0) {   // no receivers, no adjoint sources: the adjoint state and the gradient vanish
    (void)hipStreamSynchronize(s);
    return sbfwi_zero_sync(grad, sizeof(double) * f->m->n_params * ((mode & SBFWI_GRAD_PER_SHOT) ? ck->n_shots : 1));
  }
  if (sbfwi_is_lfe(f->scheme)) {
    SBFWI_CHECK(sbfwi_zero_sync(grad, sizeof(double) * f->m->n_params *
                                          ((mode & SBFWI_GRAD_PER_SHOT) ? ck->n_shots : 1)));
    return sbfwi_lfe_adjoint(f, ck, adj_src, (mode & SBFWI_GRAD_PER_SHOT) != 0, grad, s);
  }
  return sbfwi_adjoint_impl(f, ck, adj_src, mode, grad, s);
}

extern "C" int sbfwi_gradient(sbfwi_factors f, sbfwi_ckpt ck, const double* observed, const double* traces,
                              int mode, double* misfit, double* grad, hipStream_t s) {
  if (!f || !ck || !misfit || !grad || ((!observed || !traces) && ck->n_rec > 0))
    return sbfwi_fail(SBFWI_EINVAL, "NULL argument");
  int64_t count = (int64_t)ck->n_shots * ck->n_rec * ck->n_steps;
  if (ck->n_rec == 0) {   // no data: the misfit is zero, and so is its gradient (checked and set by sbfwi_adjoint)
    SBFWI_CHECK(sbfwi_adjoint(f, ck, nullptr, mode, grad, s));
    return sbfwi_zero_sync(misfit, sizeof(double) * ((mode & SBFWI_GRAD_PER_SHOT) ? ck->n_shots : 1));
  }
  double* res = nullptr;
  SBFWI_CHECK(sbfwi_alloc(&res, count));
  int rc = SBFWI_OK;
  if (mode & SBFWI_GRAD_PER_SHOT) {
    const int64_t per = (int64_t)ck->n_rec * ck->n_steps;
    for (int q = 0; q < ck->n_shots && rc == SBFWI_OK; ++q)
      rc = sbfwi_misfit_residual(traces + q * per, observed + q * per, per, f->dt, res + q * per, misfit + q, s);
  } else {
    rc = sbfwi_misfit_residual(traces, observed, count, f->dt, res, misfit, s);
  }
  if (rc == SBFWI_OK) rc = sbfwi_adjoint(f, ck, res, mode, grad, s);
  (void)hipStreamSynchronize(s);
  sbfwi_dev_free(res);
  return rc;
}

// Coarse nodal solve K_g U = F (or K_g^T lambda = r for the adjoint).
//
// The paper assembles the element dynamic stiffnesses S_e into one global
// system on the boundary nodes and leaves the solver open.  S_e of the radial
// finite-difference scheme is not symmetric, so the solver is BiCGStab with a
// Jacobi preconditioner, warm-started by the caller.
//
// Design (measured on MI355X): a device-wide barrier inside one persistent
// kernel writes back and invalidates L2 on every arrival, which leaves the
// following gathers latency-bound; ordinary kernel boundaries are cheaper.
// So every phase of an iteration is its own full-grid kernel covering all
// shots of the run together.  A block takes one slice of ELL_SLICE rows at a
// time with ELL_LPR lanes per row: the lanes of a row split its entries for
// the product (so a row costs one round of loads, not a chain of them) and
// then split its shots for the vector updates.  A phase writes per-block partial
// sums; the next phase's blocks each reduce all of them in the same fixed
// order, so every block derives identical scalars without atomics or
// barriers, and results are bit-reproducible.  Scalars rotate through three
// small device buffers: each phase reads the buffer the previous phase wrote
// and block 0 writes a different one (v: A -> B, t: B -> C, x: C -> A), so no
// block can see a buffer that is being rewritten.  A fixed number of
// iterations is enqueued up front (phases only forward the scalars once every
// shot has converged); a solve that needs more continues in one cooperative
// kernel that runs the same phases separated by grid barriers.
//
// BiCGStab is arranged with three phases per iteration: with w = K^T rhat
// (rhat = r_0 fixed for the solve), (rhat, K phat) = (w, phat) and
// (rhat, K shat) = (w, shat) are formed together with phat and shat, and
// rho_{i+1} = (rhat, s) - omega (w, shat) = (rhat, r_{i+1}).
#include <atomic>

#include "sbfwi_internal.h"

namespace {

constexpr int LPR = ELL_LPR;          // lanes per row
constexpr int CT = ELL_SLICE * LPR;   // threads per block: one slice of rows at a time
static_assert(CT == 1024 && (LPR & (LPR - 1)) == 0, "block shape");
constexpr int MAXS = 16;    // shots of a run
constexpr int NQ = 3;       // max quantities per reduction

enum { SC_BN2, SC_RHO, SC_ALPHA, SC_OMEGA, SC_RS, SC_WS, SC_BETA, SC_ACTIVE, SC_SDONE, SC_ANY, SC_ITERS, SC_N };

struct SolveArgs {
  int64_t n;
  int64_t n_slices;
  int NS;
  const int64_t* ell_off;
  const int32_t* ell_w;
  const int32_t* ell_col;
  const double* val;   // K (sliced ELL)
  const double* valT;  // K^T on the same (symmetric) pattern
  const double* dinv;
  const double* b;
  double* x;
  double *r, *rhat, *p, *v, *sv, *t, *phat, *shat, *w;
  double* partial;     // [slot][nblocks][NQ][NS]
  double* scal;        // [3][SC_N][MAXS] rotating scalar buffers
  unsigned* bar;       // grid-barrier words of the rescue kernel
  double rtol;
  int* status;         // [0] flags (2 no convergence, 4 non-finite), [1] step, [2] last, [3] max, [4] total iterations, [5] solves
  int64_t step;
  const int64_t* step_ptr;  // when set, the step number is read here (graph replays)
};

enum { SLOT_A = 0, SLOT_X = 1, SLOT_V = 2, SLOT_T = 3 };

__device__ __forceinline__ int step_of(const SolveArgs& a) { return (int)(a.step_ptr ? *a.step_ptr : a.step); }

// y = K x for the row of this thread's lane group and all shots, from the
// sliced ELL layout: chunk c of a slice holds entries k = c*LPR .. c*LPR+LPR-1
// of every row, lane-contiguous, so thread t of the block loads word c * CT + t
// (coalesced) and the LPR lanes of a row hold LPR different entries.  Chunks
// are loaded U at a time before their x gathers; a butterfly over the row's
// lanes then leaves the full sums in every lane (the same bits in each, as
// IEEE addition is commutative).  Padding entries have value 0 and a valid
// column.  Must be called by all threads of the block (uniform control flow).
template <int NSM>
__device__ __forceinline__ void spmv_slice(const SolveArgs& a, const double* __restrict__ val, int64_t sl,
                                           const double* __restrict__ xin, double (&out)[NSM]) {
  constexpr int U = NSM <= 4 ? 16 : (NSM <= 8 ? 8 : 4);
#pragma unroll
  for (int s = 0; s < NSM; ++s) out[s] = 0.0;
  const int nc = a.ell_w[sl];
  const double* vp = val + a.ell_off[sl] + threadIdx.x;
  const int32_t* cp = a.ell_col + a.ell_off[sl] + threadIdx.x;
  for (int c0 = 0; c0 < nc; c0 += U) {
    double kv[U];
    int c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      bool ok = c0 + u < nc;
      kv[u] = ok ? vp[(int64_t)(c0 + u) * CT] : 0.0;
      c[u] = ok ? cp[(int64_t)(c0 + u) * CT] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double* xc = xin + (int64_t)c[u] * a.NS;
#pragma unroll
      for (int s = 0; s < NSM; ++s)
        if (s < a.NS) out[s] += kv[u] * xc[s];
    }
  }
#pragma unroll
  for (int m = 1; m < LPR; m <<= 1)
#pragma unroll
    for (int s = 0; s < NSM; ++s) out[s] += __shfl_xor(out[s], m, 64);
}

constexpr int PG = 32;      // groups of the partial-slot reduction

struct Shared {
  double wsum[(CT / 64) * NQ * MAXS];
  double red[PG * NQ * MAXS];
  double tot[NQ * MAXS];     // tot[q * MAXS + s]
  double sc[SC_N][MAXS];
};

// Partial sums owned by a lane: quantity q of shot s lives in loc[q][s / LPR]
// of lane s % LPR (each lane of a row handles the shots s = j, j + LPR, ...).
template <int NSM>
struct Loc {
  static constexpr int OWNS = (NSM + LPR - 1) / LPR;
  double v[NQ][OWNS];
  __device__ Loc() {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int i = 0; i < OWNS; ++i) v[q][i] = 0.0;
  }
  __device__ double& operator()(int q, int s) { return v[q][s / LPR]; }
};

// Block totals of lane-owned partial sums, stored as this block's entry of a
// partial slot [slot][block][NQ * NS].  Fixed order: xor butterfly over the
// lanes of a wavefront that own the same shots, then the waves in index order.
template <int NSM>
__device__ void write_partials(Loc<NSM>& loc, int nq, const SolveArgs& a, int slot, Shared& L) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, NS = a.NS;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int i = 0; i < Loc<NSM>::OWNS; ++i) {
      double x = loc.v[q][i];
#pragma unroll
      for (int m = LPR; m < 64; m <<= 1) x += __shfl_xor(x, m, 64);
      const int s = lane + i * LPR;
      if (lane < LPR && q < nq && s < NS) L.wsum[(wave * NQ + q) * MAXS + s] = x;
    }
  __syncthreads();
  if (threadIdx.x < nq * NS) {
    const int q = threadIdx.x / NS, s = threadIdx.x - q * NS;
    double t = 0.0;
    for (int w = 0; w < CT / 64; ++w) t += L.wsum[(w * NQ + q) * MAXS + s];
    a.partial[((int64_t)slot * gridDim.x + blockIdx.x) * (NQ * NS) + q * NS + s] = t;
  }
}

// Sum over all blocks of a partial slot written by the previous phase (same
// grid), identical in every block.  With nv = nq * NS values per block and
// G = min(PG, CT / nv) groups, fetch_partials issues this thread's loads
// (value v = t % nv of blocks g, g + G, ... for group g = t / nv < G) early, so
// that they overlap the scalar loads; finish_partials adds the groups in index
// order into L.tot[q * MAXS + s].
__device__ __forceinline__ int partial_groups(int nv) { return min(PG, CT / nv); }

__device__ __forceinline__ double fetch_partials(int nq, const SolveArgs& a, int slot) {
  const int nv = nq * a.NS, G = partial_groups(nv), g = threadIdx.x / nv, v = threadIdx.x - g * nv;
  double acc = 0.0;
  if (g < G)
    for (int b = g; b < (int)gridDim.x; b += G)
      acc += a.partial[((int64_t)slot * gridDim.x + b) * (NQ * a.NS) + v];
  return acc;
}

__device__ void finish_partials(double acc, int nq, const SolveArgs& a, Shared& L) {
  const int nv = nq * a.NS, G = partial_groups(nv), g = threadIdx.x / nv, v = threadIdx.x - g * nv;
  if (g < G) L.red[g * nv + v] = acc;
  __syncthreads();
  if (threadIdx.x < nv) {
    double t = 0.0;
    for (int k = 0; k < G; ++k) t += L.red[k * nv + threadIdx.x];
    const int q = threadIdx.x / a.NS, s = threadIdx.x - q * a.NS;
    L.tot[q * MAXS + s] = t;
  }
  __syncthreads();
}

__device__ void load_scalars(const SolveArgs& a, int buf, Shared& L) {
  for (int q = threadIdx.x; q < SC_N * MAXS; q += CT) (&L.sc[0][0])[q] = a.scal[buf * SC_N * MAXS + q];
  __syncthreads();
}

__device__ void store_scalars(const SolveArgs& a, int buf, Shared& L) {
  __syncthreads();
  if (blockIdx.x == 0)
    for (int q = threadIdx.x; q < SC_N * MAXS; q += CT) a.scal[buf * SC_N * MAXS + q] = (&L.sc[0][0])[q];
}

// all shots converged: forward the scalars unchanged and report that the phase is idle
__device__ bool idle_forward(const SolveArgs& a, int out_buf, Shared& L) {
  if (L.sc[SC_ANY][0] != 0.0) return false;
  if (blockIdx.x == 0)
    for (int q = threadIdx.x; q < SC_N * MAXS; q += CT) a.scal[out_buf * SC_N * MAXS + q] = (&L.sc[0][0])[q];
  return true;
}

__device__ void update_any(Shared& L, int NS) {
  if (threadIdx.x == 0) {
    double any = 0.0;
    for (int s = 0; s < NS; ++s) any = (L.sc[SC_ACTIVE][s] != 0.0) ? 1.0 : any;
    L.sc[SC_ANY][0] = any;
  }
  __syncthreads();
}

// Slice loop of a block (uniform over the block): row r of lane group
// threadIdx.x / LPR, lane j; OWN(s) selects the shots s = j, j + LPR, ... of
// this lane (compile-time s, so per-shot registers stay registers).
#define SLICES_BEGIN                                                              \
  const int lane_j = threadIdx.x & (LPR - 1);                                     \
  for (int64_t sl = blockIdx.x; sl < a.n_slices; sl += gridDim.x) {               \
    const int64_t r = sl * ELL_SLICE + (threadIdx.x / LPR);                       \
    const bool row_ok = r < a.n;
#define SLICES_END }
#define OWN(s) if ((s & (LPR - 1)) == lane_j && s < NS && row_ok)

// r = b - K x ; rhat = r ; partials |b|^2, |r|^2
template <int NSM>
__global__ void __launch_bounds__(CT) k_init1(SolveArgs a) {
  __shared__ Shared L;
  Loc<NSM> loc;
  const int NS = a.NS;
  SLICES_BEGIN {
    double kx[NSM];
    spmv_slice<NSM>(a, a.val, sl, a.x, kx);
#pragma unroll
    for (int s = 0; s < NSM; ++s) {
      OWN(s) {
        int64_t g = r * NS + s;
        double bv = a.b[g], rv = bv - kx[s];
        a.r[g] = rv;
        a.rhat[g] = rv;
        loc(0, s) += bv * bv;
        loc(1, s) += rv * rv;
      }
    }
  } SLICES_END
  write_partials<NSM>(loc, 2, a, SLOT_A, L);
}

// scalars from slot A; w = K^T rhat ; p = r ; phat = D^-1 p ; partials |r|^2, (w, phat)
template <int NSM>
__global__ void __launch_bounds__(CT) k_init2(SolveArgs a) {
  __shared__ Shared L;
  const int NS = a.NS;
  finish_partials(fetch_partials(2, a, SLOT_A), 2, a, L);
  const double tol2 = a.rtol * a.rtol;
  if (threadIdx.x < MAXS) {
    const int s = threadIdx.x;
    double bn2 = s < NS ? L.tot[s] : 0.0, rn2 = s < NS ? L.tot[MAXS + s] : 0.0;
    for (int k = 0; k < SC_N; ++k) L.sc[k][s] = 0.0;
    L.sc[SC_BN2][s] = bn2;
    L.sc[SC_RHO][s] = rn2;
    L.sc[SC_ALPHA][s] = 1.0;
    L.sc[SC_OMEGA][s] = 1.0;
    L.sc[SC_ACTIVE][s] = (s < NS && bn2 > 0.0 && rn2 > tol2 * bn2 && isfinite(rn2)) ? 1.0 : 0.0;
  }
  __syncthreads();
  update_any(L, NS);
  Loc<NSM> loc;
  SLICES_BEGIN {
    double kx[NSM];
    spmv_slice<NSM>(a, a.valT, sl, a.rhat, kx);
#pragma unroll
    for (int s = 0; s < NSM; ++s) {
      OWN(s) {
        int64_t g = r * NS + s;
        if (L.sc[SC_BN2][s] == 0.0) a.x[g] = 0.0;
        double pv = a.r[g];
        double ph = a.dinv[r] * pv;
        a.w[g] = kx[s];
        a.p[g] = pv;
        a.phat[g] = ph;
        loc(0, s) += pv * pv;
        loc(1, s) += kx[s] * ph;
      }
    }
  } SLICES_END
  write_partials<NSM>(loc, 2, a, SLOT_X, L);
  store_scalars(a, 0, L);
}

// convergence / alpha from slot X ; v = K phat ; s = r - alpha v ; shat = D^-1 s ;
// partials |s|^2, (rhat, s), (w, shat).  Buffer A -> B.  Returns false when idle.
template <int NSM>
__device__ bool phase_v(const SolveArgs& a, Shared& L) {
  const int NS = a.NS;
  const double part = fetch_partials(2, a, SLOT_X);
  load_scalars(a, 0, L);
  if (idle_forward(a, 1, L)) return false;
  // with one slice per block, v = K phat (independent of this phase's scalars) starts first
  const bool single = (int64_t)gridDim.x >= a.n_slices;
  double kx0[NSM];
  if (single) spmv_slice<NSM>(a, a.val, blockIdx.x, a.phat, kx0);
  finish_partials(part, 2, a, L);
  const double tol2 = a.rtol * a.rtol;
  if (threadIdx.x < NS) {
    const int s = threadIdx.x;
    if (L.sc[SC_ACTIVE][s] != 0.0) {
      double rn2 = L.tot[s], wp = L.tot[MAXS + s], rho = L.sc[SC_RHO][s];
      if (!isfinite(rn2) || !isfinite(rho) || !isfinite(wp)) {
        L.sc[SC_ACTIVE][s] = 0.0;
        if (blockIdx.x == 0) {
          atomicOr(&a.status[0], 4);
          atomicCAS(&a.status[1], -1, step_of(a));
        }
      } else if (rn2 <= tol2 * L.sc[SC_BN2][s]) {
        L.sc[SC_ACTIVE][s] = 0.0;
      } else if (rho == 0.0 || wp == 0.0) {  // breakdown
        L.sc[SC_ACTIVE][s] = 0.0;
        if (blockIdx.x == 0) {
          atomicOr(&a.status[0], 2);
          atomicCAS(&a.status[1], -1, step_of(a));
        }
      } else {
        L.sc[SC_ALPHA][s] = rho / wp;
      }
    }
  }
  __syncthreads();
  update_any(L, NS);
  store_scalars(a, 1, L);
  if (L.sc[SC_ANY][0] == 0.0) return false;
  Loc<NSM> loc;
  SLICES_BEGIN {
    double kx[NSM];
    if (single) {
#pragma unroll
      for (int s = 0; s < NSM; ++s) kx[s] = kx0[s];
    } else {
      spmv_slice<NSM>(a, a.val, sl, a.phat, kx);
    }
#pragma unroll
    for (int s = 0; s < NSM; ++s) {
      OWN(s) {
        if (L.sc[SC_ACTIVE][s] == 0.0) continue;
        int64_t g = r * NS + s;
        double sv = a.r[g] - L.sc[SC_ALPHA][s] * kx[s];
        double sh = a.dinv[r] * sv;
        a.v[g] = kx[s];
        a.sv[g] = sv;
        a.shat[g] = sh;
        loc(0, s) += sv * sv;
        loc(1, s) += a.rhat[g] * sv;
        loc(2, s) += a.w[g] * sh;
      }
    }
  } SLICES_END
  write_partials<NSM>(loc, 3, a, SLOT_V, L);
  return true;
}

// half-step convergence from slot V ; t = K shat ; partials (t, s), (t, t).
// Shots converged on the half step take x += alpha phat.  Buffer B -> C.
template <int NSM>
__device__ void phase_t(const SolveArgs& a, Shared& L) {
  const int NS = a.NS;
  const double part = fetch_partials(3, a, SLOT_V);
  load_scalars(a, 1, L);
  if (idle_forward(a, 2, L)) return;
  const bool single = (int64_t)gridDim.x >= a.n_slices;
  double kx0[NSM];
  if (single) spmv_slice<NSM>(a, a.val, blockIdx.x, a.shat, kx0);
  finish_partials(part, 3, a, L);
  const double tol2 = a.rtol * a.rtol;
  if (threadIdx.x < NS) {
    const int s = threadIdx.x;
    L.sc[SC_SDONE][s] = (L.sc[SC_ACTIVE][s] != 0.0 && L.tot[s] <= tol2 * L.sc[SC_BN2][s]) ? 1.0 : 0.0;
    L.sc[SC_RS][s] = L.tot[MAXS + s];
    L.sc[SC_WS][s] = L.tot[2 * MAXS + s];
  }
  __syncthreads();
  store_scalars(a, 2, L);
  Loc<NSM> loc;
  SLICES_BEGIN {
    double kx[NSM];
    if (single) {
#pragma unroll
      for (int s = 0; s < NSM; ++s) kx[s] = kx0[s];
    } else {
      spmv_slice<NSM>(a, a.val, sl, a.shat, kx);
    }
#pragma unroll
    for (int s = 0; s < NSM; ++s) {
      OWN(s) {
        if (L.sc[SC_ACTIVE][s] == 0.0) continue;
        int64_t g = r * NS + s;
        if (L.sc[SC_SDONE][s] != 0.0) {
          a.x[g] += L.sc[SC_ALPHA][s] * a.phat[g];
          continue;
        }
        a.t[g] = kx[s];
        loc(0, s) += kx[s] * a.sv[g];
        loc(1, s) += kx[s] * kx[s];
      }
    }
  } SLICES_END
  write_partials<NSM>(loc, 2, a, SLOT_T, L);
}

// omega, rho, beta from slot T ; x += alpha phat + omega shat ; r = s - omega t ;
// p = r + beta (p - omega v) ; phat = D^-1 p ; partials |r|^2, (w, phat).  Buffer C -> A.
template <int NSM>
__device__ void phase_x(const SolveArgs& a, Shared& L) {
  const int NS = a.NS;
  const double part = fetch_partials(2, a, SLOT_T);
  load_scalars(a, 2, L);
  if (idle_forward(a, 0, L)) return;
  finish_partials(part, 2, a, L);
  if (threadIdx.x < NS) {
    const int s = threadIdx.x;
    if (L.sc[SC_SDONE][s] != 0.0) L.sc[SC_ACTIVE][s] = 0.0;
    L.sc[SC_SDONE][s] = 0.0;
    L.sc[SC_BETA][s] = 0.0;
    if (L.sc[SC_ACTIVE][s] != 0.0) {
      double om = L.tot[s] / L.tot[MAXS + s];
      double rho_new = L.sc[SC_RS][s] - om * L.sc[SC_WS][s];
      L.sc[SC_BETA][s] = (rho_new / L.sc[SC_RHO][s]) * (L.sc[SC_ALPHA][s] / om);
      L.sc[SC_OMEGA][s] = om;
      L.sc[SC_RHO][s] = rho_new;
    }
  }
  __syncthreads();
  update_any(L, NS);
  if (blockIdx.x == 0 && threadIdx.x == 0) L.sc[SC_ITERS][0] += 1.0;
  Loc<NSM> loc;
  SLICES_BEGIN {
#pragma unroll
    for (int s = 0; s < NSM; ++s) {
      OWN(s) {
        if (L.sc[SC_ACTIVE][s] == 0.0) continue;
        int64_t g = r * NS + s;
        const double al = L.sc[SC_ALPHA][s], om = L.sc[SC_OMEGA][s];
        a.x[g] += al * a.phat[g] + om * a.shat[g];
        double rv = a.sv[g] - om * a.t[g];
        double pv = rv + L.sc[SC_BETA][s] * (a.p[g] - om * a.v[g]);
        double ph = a.dinv[r] * pv;
        a.r[g] = rv;
        a.p[g] = pv;
        a.phat[g] = ph;
        loc(0, s) += rv * rv;
        loc(1, s) += a.w[g] * ph;
      }
    }
  } SLICES_END
  write_partials<NSM>(loc, 2, a, SLOT_X, L);
  store_scalars(a, 0, L);
}

template <int NSM>
__global__ void __launch_bounds__(CT) k_phase_v(SolveArgs a) {
  __shared__ Shared L;
  phase_v<NSM>(a, L);
}

template <int NSM>
__global__ void __launch_bounds__(CT) k_phase_t(SolveArgs a) {
  __shared__ Shared L;
  phase_t<NSM>(a, L);
}

template <int NSM>
__global__ void __launch_bounds__(CT) k_phase_x(SolveArgs a) {
  __shared__ Shared L;
  phase_x<NSM>(a, L);
}

// Grid barrier for the rescue kernel (all blocks co-resident by cooperative
// launch): arrival counters in groups of 16 blocks, one counter for the
// groups, and a generation word the others poll.  The poll is bounded: after
// about two seconds it flags an error and stops waiting, so a broken barrier
// ends the kernel instead of hanging it.
__device__ __forceinline__ unsigned ld_acquire(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ void grid_barrier(unsigned* bar, unsigned& gen_seen, int* status) {
  __syncthreads();
  if (threadIdx.x == 0 && gen_seen != 0xFFFFFFFFu) {
    const int G = 16;
    const int nb = gridDim.x, ng = (nb + G - 1) / G, grp = blockIdx.x / G;
    const int gsize = min(G, nb - grp * G);
    unsigned* gen = bar;
    unsigned* top = bar + 32;
    unsigned* ctr = bar + 64 + 32 * grp;
    const unsigned g = gen_seen;
    __threadfence();
    unsigned old = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (old == (unsigned)(gsize - 1)) {
      __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      unsigned o2 = __hip_atomic_fetch_add(top, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (o2 == (unsigned)(ng - 1)) {
        __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    long spins = 0;
    bool timed_out = false;
    while (ld_acquire(gen) == g) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > 2000000L) {
        atomicOr(&status[0], 8);
        timed_out = true;
        break;
      }
    }
    gen_seen = timed_out ? 0xFFFFFFFFu : g + 1;
    __threadfence();
  }
  __syncthreads();
}

// Continues the iteration for solves that the enqueued phases did not finish,
// with the same grid, row mapping and partial slots (so the same arithmetic);
// leaves at once when every shot has converged.
template <int NSM>
__global__ void __launch_bounds__(CT) k_rescue(SolveArgs a, int max_more) {
  __shared__ Shared L;
  unsigned gen_seen = 0;
  if (threadIdx.x == 0) gen_seen = ld_acquire(a.bar);
  for (int i = 0; i < max_more; ++i) {
    // go is the same in every block (identical scalars), so all blocks leave together
    if (!phase_v<NSM>(a, L)) break;
    grid_barrier(a.bar, gen_seen, a.status);
    phase_t<NSM>(a, L);
    grid_barrier(a.bar, gen_seen, a.status);
    phase_x<NSM>(a, L);
    grid_barrier(a.bar, gen_seen, a.status);
  }
}

// final convergence check of slot X and statistics
template <int NSM>
__global__ void __launch_bounds__(CT) k_finish(SolveArgs a) {
  __shared__ Shared L;
  const int NS = a.NS;
  load_scalars(a, 0, L);
  finish_partials(fetch_partials(2, a, SLOT_X), 2, a, L);
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double tol2 = a.rtol * a.rtol;
  int unconverged = 0;
  if (L.sc[SC_ANY][0] != 0.0)
    for (int s = 0; s < NS; ++s)
      if (L.sc[SC_ACTIVE][s] != 0.0 && !(L.tot[s] <= tol2 * L.sc[SC_BN2][s])) unconverged = 1;
  int it = (int)L.sc[SC_ITERS][0];
  a.status[2] = it;
  atomicMax(&a.status[3], it);
  atomicAdd(&a.status[4], it);
  atomicAdd(&a.status[5], 1);
  if (unconverged) {
    atomicOr(&a.status[0], 2);
    atomicCAS(&a.status[1], -1, step_of(a));
  }
}

// parts: 1 = start-up and the enqueued iterations, 2 = the rescue kernel,
// 4 = the final check (a captured graph holds parts 1 and 4; the cooperative
// rescue launch runs between its replays)
template <int NSM>
hipError_t enqueue(const SolveArgs& a, int iters, int max_more, unsigned blocks, int parts, hipStream_t s) {
  if (parts & 1) {
    {
      ProfScope ps(PK_SOLVE_INIT, s);
      hipLaunchKernelGGL(k_init1<NSM>, dim3(blocks), dim3(CT), 0, s, a);
      hipLaunchKernelGGL(k_init2<NSM>, dim3(blocks), dim3(CT), 0, s, a);
    }
    for (int i = 0; i < iters; ++i) {
      {
        ProfScope ps(PK_SOLVE_V, s);
        hipLaunchKernelGGL(k_phase_v<NSM>, dim3(blocks), dim3(CT), 0, s, a);
      }
      {
        ProfScope ps(PK_SOLVE_T, s);
        hipLaunchKernelGGL(k_phase_t<NSM>, dim3(blocks), dim3(CT), 0, s, a);
      }
      ProfScope ps(PK_SOLVE_X, s);
      hipLaunchKernelGGL(k_phase_x<NSM>, dim3(blocks), dim3(CT), 0, s, a);
    }
  }
  if ((parts & 2) && max_more > 0) {
    SolveArgs b = a;
    void* args[] = {&b, &max_more};
    hipError_t e = hipLaunchCooperativeKernel((const void*)k_rescue<NSM>, dim3(blocks), dim3(CT), args, 0, s);
    if (e != hipSuccess) return e;
  }
  if (parts & 4) hipLaunchKernelGGL(k_finish<NSM>, dim3(blocks), dim3(CT), 0, s, a);
  return hipGetLastError();
}

// largest grid whose blocks can all be resident at once (the rescue kernel needs it)
template <int NSM>
int coresident_blocks() {
  static std::atomic<int> cached{0};   // queried once (host threads may race benignly)
  int c = cached.load();
  if (c == 0) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_rescue<NSM>, CT, 0) != hipSuccess) return 0;
    c = per * sbfwi_device_cus();
    cached.store(c);
  }
  return c;
}

}  // namespace

int sbfwi_coarse_work_alloc(CoarseWork* w, sbfwi_mesh_s* m, int NS) {
  if (NS > MAXS) return sbfwi_fail(SBFWI_EINVAL, "at most %d shots per run", MAXS);
  const int64_t n_nodes = m->n_nodes;
  w->NS = NS;
  w->n = n_nodes;
  int64_t sz = n_nodes * NS;
  SBFWI_CHECK(sbfwi_alloc(&w->r, 9 * sz));
  w->rhat = w->r + sz;
  w->p = w->rhat + sz;
  w->v = w->p + sz;
  w->sv = w->v + sz;
  w->t = w->sv + sz;
  w->phat = w->t + sz;
  w->shat = w->phat + sz;
  w->w = w->shat + sz;
  int64_t want = (n_nodes + ELL_SLICE - 1) / ELL_SLICE;
  int cap = NS <= 1 ? coresident_blocks<1>() : NS <= 2 ? coresident_blocks<2>() : NS <= 4 ? coresident_blocks<4>()
          : NS <= 8 ? coresident_blocks<8>() : coresident_blocks<16>();
  if (cap <= 0) return sbfwi_fail(SBFWI_EHIP, "cannot query the co-resident grid size");
  w->nblocks = (int)(want < cap ? want : cap);
  SBFWI_CHECK(sbfwi_alloc(&w->partial, (int64_t)4 * w->nblocks * NQ * NS));
  SBFWI_CHECK(sbfwi_alloc(&w->scal, (int64_t)3 * SC_N * MAXS));
  SBFWI_CHECK(sbfwi_alloc(&w->bar, 64 + 32 * ((w->nblocks + 15) / 16 + 1)));
  SBFWI_CHECK(sbfwi_zero_sync(w->bar, sizeof(unsigned) * (64 + 32 * ((w->nblocks + 15) / 16 + 1))));
  if (m->dsym) {   // direct solve: forward and backward results by elimination position
    SBFWI_CHECK(sbfwi_alloc(&w->dyb, 2 * sz));
    w->dxp = w->dyb + sz;
    SBFWI_CHECK(sbfwi_alloc(&w->dupd, std::max<int64_t>(1, m->dsym->b_ptr[m->dsym->nS]) * NS));
  }
  return SBFWI_OK;
}

void sbfwi_coarse_work_free(CoarseWork* w) {
  sbfwi_dev_free(w->r);
  sbfwi_dev_free(w->partial);
  sbfwi_dev_free(w->scal);
  sbfwi_dev_free(w->bar);
  sbfwi_dev_free(w->dyb);
  sbfwi_dev_free(w->dupd);
  *w = CoarseWork();
}

int sbfwi_coarse_solve(sbfwi_factors_s* f, CoarseWork* w, int transpose, const double* b, double* x,
                       int64_t step, hipStream_t s) {
  return sbfwi_coarse_solve_parts(f, w, transpose, b, x, step, nullptr, 7, s);
}

int sbfwi_coarse_solve_parts(sbfwi_factors_s* f, CoarseWork* w, int transpose, const double* b, double* x,
                             int64_t step, const int64_t* step_ptr, int parts, hipStream_t s) {
  if (f->dnum) {   // direct factors: the whole solve is part 1 (plain launches, no cooperative kernel)
    if (!(parts & 1)) return SBFWI_OK;
    if (!w->dyb) return sbfwi_fail(SBFWI_EINVAL, "work buffers lack the direct-solve scratch");
    return sbfwi_direct_solve(f, w, transpose, b, x, s);
  }
  sbfwi_mesh_s* m = f->m;
  SolveArgs a;
  a.n = m->n_nodes;
  a.n_slices = (m->n_nodes + ELL_SLICE - 1) / ELL_SLICE;
  a.NS = w->NS;
  a.ell_off = m->d.ell_off;
  a.ell_w = m->d.ell_w;
  a.ell_col = m->d.ell_col;
  a.val = transpose ? f->d.KTell : f->d.Kell;
  a.valT = transpose ? f->d.Kell : f->d.KTell;
  a.dinv = f->d.diag_inv;
  a.b = b;
  a.x = x;
  a.r = w->r; a.rhat = w->rhat; a.p = w->p; a.v = w->v; a.sv = w->sv; a.t = w->t;
  a.phat = w->phat; a.shat = w->shat; a.w = w->w;
  a.partial = w->partial;
  a.scal = w->scal;
  a.bar = w->bar;
  a.rtol = f->rtol;
  a.status = f->d.status;
  a.step = step;
  a.step_ptr = step_ptr;
  const int iters = f->enqueued_iters < f->max_iter ? f->enqueued_iters : f->max_iter;
  const int more = f->max_iter - iters;
  const unsigned blocks = (unsigned)w->nblocks;
  ProfScope ps(PK_SOLVE, s);
  hipError_t e;
  if (a.NS == 1) e = enqueue<1>(a, iters, more, blocks, parts, s);
  else if (a.NS == 2) e = enqueue<2>(a, iters, more, blocks, parts, s);
  else if (a.NS <= 4) e = enqueue<4>(a, iters, more, blocks, parts, s);
  else if (a.NS <= 8) e = enqueue<8>(a, iters, more, blocks, parts, s);
  else e = enqueue<16>(a, iters, more, blocks, parts, s);
  if (e != hipSuccess) return sbfwi_fail(SBFWI_EHIP, "coarse solve launch: %s", hipGetErrorString(e));
  return SBFWI_OK;
}

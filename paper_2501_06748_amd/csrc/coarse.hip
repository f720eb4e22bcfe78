// Coarse nodal solve K_g U = F (or K_g^T lambda = r for the adjoint).
//
// The paper assembles the element dynamic stiffnesses S_e into one global
// system on the boundary nodes and leaves the solver open.  S_e of the radial
// finite-difference scheme is not symmetric, so the solver is BiCGStab with a
// Jacobi preconditioner, warm-started by the caller.  One cooperative,
// persistent launch runs the whole solve: rows are strided over the grid and
// the 4 global reductions of an iteration go through per-block partial sums
// that every block then reduces in the same fixed tree order, so all blocks
// take identical convergence decisions and results are bit-reproducible.
// All right-hand sides (shots) of a run are solved together, each with its
// own scalars; a shot stops updating once it has converged.
#include <hip/hip_cooperative_groups.h>

#include "sbfwi_internal.h"

namespace cg = cooperative_groups;

namespace {

constexpr int CT = 1024;    // threads per block
constexpr int MAXS = 16;    // max right-hand sides per solve
constexpr int NQ = 2;       // max quantities per reduction phase

struct SolveArgs {
  int64_t n;
  int NS;
  const int64_t* row_ptr;
  const int32_t* col;
  const double* val;
  const double* dinv;
  const double* b;
  double* x;
  double *r, *rhat, *p, *v, *sv, *t, *phat, *shat;
  double* partial;   // [4 phases][NQ][nblocks][NS]
  double rtol;
  int max_iter;
  int* status;       // [0] flags, [1] step of failure, [2] last, [3] max, [4] total iterations, [5] solves
  int64_t step;
};

template <int NSM>
__device__ __forceinline__ void spmv_row(const SolveArgs& a, int64_t r, const double* __restrict__ xin,
                                         double (&out)[NSM]) {
#pragma unroll
  for (int s = 0; s < NSM; ++s) out[s] = 0.0;
  for (int64_t q = a.row_ptr[r]; q < a.row_ptr[r + 1]; ++q) {
    double kv = a.val[q];
    const double* xc = xin + (int64_t)a.col[q] * a.NS;
#pragma unroll
    for (int s = 0; s < NSM; ++s)
      if (s < a.NS) out[s] += kv * xc[s];
  }
}

// Block sums of nv values held by every thread, in a fixed order (wavefront
// shuffle tree, then the waves in index order); results land in tot[0..nv).
template <int NV>
__device__ void block_sums(double (&v)[NV], int nv, double* wsum /*[CT/64][NV]*/, double* tot /*[NV]*/) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    if (q >= nv) break;
    double x = v[q];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) wsum[wave * NV + q] = x;
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    double t = 0.0;
    for (int w = 0; w < CT / 64; ++w) t += wsum[w * NV + threadIdx.x];
    tot[threadIdx.x] = t;
  }
  __syncthreads();
}

// Block partials of nq quantities x NS shots into this block's slot of a phase.
template <int NSM>
__device__ void block_partial(double (&loc)[NQ][NSM], int nq, const SolveArgs& a, int phase, double* wsum,
                              double* tot) {
  double v[NQ * NSM];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int s = 0; s < NSM; ++s) v[q * NSM + s] = loc[q][s];
  block_sums<NQ * NSM>(v, nq * NSM, wsum, tot);
  if (threadIdx.x < nq * NSM) {
    int q = threadIdx.x / NSM, s = threadIdx.x % NSM;
    if (s < a.NS) a.partial[(((int64_t)phase * NQ + q) * gridDim.x + blockIdx.x) * a.NS + s] = tot[threadIdx.x];
  }
}

// Every block sums all block partials of a phase in the same fixed order.
template <int NSM>
__device__ void grid_total(int nq, const SolveArgs& a, int phase, double* wsum, double* tots,
                           double (&out)[NQ][NSM]) {
  const int nbk = gridDim.x;
  double v[NQ * NSM];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int s = 0; s < NSM; ++s) {
      double acc = 0.0;
      if (q < nq && s < a.NS)
        for (int b = threadIdx.x; b < nbk; b += CT) acc += a.partial[(((int64_t)phase * NQ + q) * nbk + b) * a.NS + s];
      v[q * NSM + s] = acc;
    }
  block_sums<NQ * NSM>(v, nq * NSM, wsum, tots);
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int s = 0; s < NSM; ++s) out[q][s] = (q < nq && s < a.NS) ? tots[q * NSM + s] : 0.0;
  __syncthreads();
}

template <int NSM>
__global__ void __launch_bounds__(CT) bicgstab_kernel(SolveArgs a) {
  __shared__ double red[(CT / 64) * NQ * NSM];
  __shared__ double tsh[NQ * NSM];
  double tot[NQ][NSM];
  cg::grid_group grid = cg::this_grid();
  const int64_t gsz = (int64_t)gridDim.x * CT;
  const int64_t gtid = (int64_t)blockIdx.x * CT + threadIdx.x;
  const int NS = a.NS;
  double bn2[NSM], rho_old[NSM], alpha[NSM], omega[NSM];
  bool active[NSM];
  double loc[NQ][NSM];
  // r = b - K x ; rhat = r ; p = v = 0 ; partials |b|^2, |r|^2
#pragma unroll
  for (int s = 0; s < NSM; ++s) { loc[0][s] = 0.0; loc[1][s] = 0.0; }
  for (int64_t r = gtid; r < a.n; r += gsz) {
    double kx[NSM];
    spmv_row<NSM>(a, r, a.x, kx);
#pragma unroll
    for (int s = 0; s < NSM; ++s) {
      if (s >= NS) continue;
      int64_t g = r * NS + s;
      double bv = a.b[g], rv = bv - kx[s];
      a.r[g] = rv;
      a.rhat[g] = rv;
      a.p[g] = 0.0;
      a.v[g] = 0.0;
      loc[0][s] += bv * bv;
      loc[1][s] += rv * rv;
    }
  }
  block_partial<NSM>(loc, 2, a, 0, red, tsh);
  grid.sync();
  grid_total<NSM>(2, a, 0, red, tsh, tot);
  bool any = false;
#pragma unroll
  for (int s = 0; s < NSM; ++s) {
    bn2[s] = tot[0][s];
    double rn2 = tot[1][s];
    rho_old[s] = rn2;           // (rhat, r) with rhat = r
    alpha[s] = 1.0;
    omega[s] = 1.0;
    active[s] = (s < NS) && (bn2[s] > 0.0) && (rn2 > a.rtol * a.rtol * bn2[s]) && isfinite(rn2);
    any = any || active[s];
  }
  // a zero right-hand side has the zero solution
  for (int64_t r = gtid; r < a.n; r += gsz) {
#pragma unroll
    for (int s = 0; s < NSM; ++s)
      if (s < NS && bn2[s] == 0.0) a.x[r * NS + s] = 0.0;
  }
  double rho_new[NSM];
#pragma unroll
  for (int s = 0; s < NSM; ++s) rho_new[s] = rho_old[s];
  bool first = true;
  int it = 0;
  for (it = 0; it < a.max_iter && any; ++it) {
    // p = r + beta (p - omega v); phat = D^-1 p
    for (int64_t r = gtid; r < a.n; r += gsz) {
#pragma unroll
      for (int s = 0; s < NSM; ++s) {
        if (s >= NS || !active[s]) continue;
        int64_t g = r * NS + s;
        double beta = first ? 0.0 : (rho_new[s] / rho_old[s]) * (alpha[s] / omega[s]);
        double pv = a.r[g] + beta * (a.p[g] - omega[s] * a.v[g]);
        a.p[g] = pv;
        a.phat[g] = a.dinv[r] * pv;
      }
    }
#pragma unroll
    for (int s = 0; s < NSM; ++s) if (!first) rho_old[s] = rho_new[s];
    first = false;
    grid.sync();
    // v = K phat ; (rhat, v)
#pragma unroll
    for (int s = 0; s < NSM; ++s) loc[0][s] = 0.0;
    for (int64_t r = gtid; r < a.n; r += gsz) {
      double kx[NSM];
      spmv_row<NSM>(a, r, a.phat, kx);
#pragma unroll
      for (int s = 0; s < NSM; ++s) {
        if (s >= NS || !active[s]) continue;
        int64_t g = r * NS + s;
        a.v[g] = kx[s];
        loc[0][s] += a.rhat[g] * kx[s];
      }
    }
    block_partial<NSM>(loc, 1, a, 1, red, tsh);
    grid.sync();
    grid_total<NSM>(1, a, 1, red, tsh, tot);
#pragma unroll
    for (int s = 0; s < NSM; ++s)
      if (s < NS && active[s]) alpha[s] = rho_old[s] / tot[0][s];
    // s = r - alpha v ; shat = D^-1 s ; |s|^2
#pragma unroll
    for (int s = 0; s < NSM; ++s) loc[0][s] = 0.0;
    for (int64_t r = gtid; r < a.n; r += gsz) {
#pragma unroll
      for (int s = 0; s < NSM; ++s) {
        if (s >= NS || !active[s]) continue;
        int64_t g = r * NS + s;
        double sv = a.r[g] - alpha[s] * a.v[g];
        a.sv[g] = sv;
        a.shat[g] = a.dinv[r] * sv;
        loc[0][s] += sv * sv;
      }
    }
    block_partial<NSM>(loc, 1, a, 2, red, tsh);
    grid.sync();
    grid_total<NSM>(1, a, 2, red, tsh, tot);
    bool sdone[NSM];
#pragma unroll
    for (int s = 0; s < NSM; ++s) sdone[s] = (s < NS && active[s]) && (tot[0][s] <= a.rtol * a.rtol * bn2[s]);
    // t = K shat ; (t, s), (t, t)
#pragma unroll
    for (int s = 0; s < NSM; ++s) { loc[0][s] = 0.0; loc[1][s] = 0.0; }
    for (int64_t r = gtid; r < a.n; r += gsz) {
      double kx[NSM];
      spmv_row<NSM>(a, r, a.shat, kx);
#pragma unroll
      for (int s = 0; s < NSM; ++s) {
        if (s >= NS || !active[s]) continue;
        int64_t g = r * NS + s;
        if (sdone[s]) {   // converged on the half step: x += alpha phat
          a.x[g] += alpha[s] * a.phat[g];
          continue;
        }
        a.t[g] = kx[s];
        loc[0][s] += kx[s] * a.sv[g];
        loc[1][s] += kx[s] * kx[s];
      }
    }
    block_partial<NSM>(loc, 2, a, 3, red, tsh);
    grid.sync();
    grid_total<NSM>(2, a, 3, red, tsh, tot);
#pragma unroll
    for (int s = 0; s < NSM; ++s) {
      if (sdone[s]) active[s] = false;
      if (s < NS && active[s]) omega[s] = tot[0][s] / tot[1][s];
    }
    // x += alpha phat + omega shat ; r = s - omega t ; (rhat, r), |r|^2
#pragma unroll
    for (int s = 0; s < NSM; ++s) { loc[0][s] = 0.0; loc[1][s] = 0.0; }
    for (int64_t r = gtid; r < a.n; r += gsz) {
#pragma unroll
      for (int s = 0; s < NSM; ++s) {
        if (s >= NS || !active[s]) continue;
        int64_t g = r * NS + s;
        a.x[g] += alpha[s] * a.phat[g] + omega[s] * a.shat[g];
        double rv = a.sv[g] - omega[s] * a.t[g];
        a.r[g] = rv;
        loc[0][s] += a.rhat[g] * rv;
        loc[1][s] += rv * rv;
      }
    }
    block_partial<NSM>(loc, 2, a, 0, red, tsh);
    grid.sync();
    grid_total<NSM>(2, a, 0, red, tsh, tot);
    any = false;
#pragma unroll
    for (int s = 0; s < NSM; ++s) {
      if (s < NS && active[s]) {
        rho_new[s] = tot[0][s];
        double rn2 = tot[1][s];
        if (!isfinite(rn2) || !isfinite(rho_new[s])) {
          active[s] = false;
          if (blockIdx.x == 0 && threadIdx.x == 0) {
            atomicOr(&a.status[0], 4);
            atomicCAS(&a.status[1], -1, (int)a.step);
          }
        } else if (rn2 <= a.rtol * a.rtol * bn2[s]) {
          active[s] = false;
        } else if (rho_new[s] == 0.0) {  // breakdown
          active[s] = false;
          if (blockIdx.x == 0 && threadIdx.x == 0) {
            atomicOr(&a.status[0], 2);
            atomicCAS(&a.status[1], -1, (int)a.step);
          }
        }
      }
      any = any || active[s];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.status[2] = it;
    atomicMax(&a.status[3], it);
    atomicAdd(&a.status[4], it);
    atomicAdd(&a.status[5], 1);
    if (any) {
      atomicOr(&a.status[0], 2);
      atomicCAS(&a.status[1], -1, (int)a.step);
    }
  }
}

int g_coop_blocks[5] = {0, 0, 0, 0, 0};

template <int NSM>
int coop_grid(int idx, int64_t n, int want_blocks) {
  if (g_coop_blocks[idx] == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, bicgstab_kernel<NSM>, CT, 0) != hipSuccess) return 0;
    g_coop_blocks[idx] = per * cus;
  }
  // the cooperative grid barrier costs about 0.13 us per block on MI355X, so a
  // small grid of large blocks is faster than filling the chip
  int64_t want = (n + CT - 1) / CT;
  if (want > want_blocks) want = want_blocks;
  int64_t cap = g_coop_blocks[idx] < 256 ? g_coop_blocks[idx] : 256;
  if (want < 1) want = 1;
  return (int)(want < cap ? want : cap);
}

}  // namespace

int sbfwi_coarse_work_alloc(CoarseWork* w, int64_t n_nodes, int NS) {
  if (NS > MAXS) return sbfwi_fail(SBFWI_EINVAL, "at most %d shots per run", MAXS);
  w->NS = NS;
  w->n = n_nodes;
  int64_t sz = n_nodes * NS;
  SBFWI_CHECK(sbfwi_alloc(&w->r, 8 * sz));
  w->rhat = w->r + sz;
  w->p = w->rhat + sz;
  w->v = w->p + sz;
  w->sv = w->v + sz;
  w->t = w->sv + sz;
  w->phat = w->t + sz;
  w->shat = w->phat + sz;
  SBFWI_CHECK(sbfwi_alloc(&w->partial, (int64_t)4 * NQ * 256 * NS));
  return SBFWI_OK;
}

void sbfwi_coarse_work_free(CoarseWork* w) {
  sbfwi_dev_free(w->r);
  sbfwi_dev_free(w->partial);
  *w = CoarseWork();
}

int sbfwi_coarse_solve(sbfwi_factors_s* f, CoarseWork* w, int transpose, const double* b, double* x,
                       int64_t step, hipStream_t s) {
  sbfwi_mesh_s* m = f->m;
  SolveArgs a;
  a.n = m->n_nodes;
  a.NS = w->NS;
  a.row_ptr = m->d.row_ptr;
  a.col = m->d.col;
  a.val = transpose ? f->d.KTval : f->d.Kval;
  a.dinv = f->d.diag_inv;
  a.b = b;
  a.x = x;
  a.r = w->r; a.rhat = w->rhat; a.p = w->p; a.v = w->v; a.sv = w->sv; a.t = w->t;
  a.phat = w->phat; a.shat = w->shat;
  a.partial = w->partial;
  a.rtol = f->rtol;
  a.max_iter = f->max_iter;
  a.status = f->d.status;
  a.step = step;
  void* args[] = {&a};
  int nsm = a.NS <= 1 ? 1 : a.NS <= 2 ? 2 : a.NS <= 4 ? 4 : a.NS <= 8 ? 8 : 16;
  const void* fn;
  int blocks;
  switch (nsm) {
    case 1: fn = (const void*)bicgstab_kernel<1>; blocks = coop_grid<1>(0, a.n, f->solver_blocks); break;
    case 2: fn = (const void*)bicgstab_kernel<2>; blocks = coop_grid<2>(1, a.n, f->solver_blocks); break;
    case 4: fn = (const void*)bicgstab_kernel<4>; blocks = coop_grid<4>(2, a.n, f->solver_blocks); break;
    case 8: fn = (const void*)bicgstab_kernel<8>; blocks = coop_grid<8>(3, a.n, f->solver_blocks); break;
    default: fn = (const void*)bicgstab_kernel<16>; blocks = coop_grid<16>(4, a.n, f->solver_blocks); break;
  }
  if (blocks <= 0) return sbfwi_fail(SBFWI_EHIP, "cannot size the cooperative coarse-solve grid");
  ProfScope ps(PK_SOLVE, s);
  SBFWI_HIP(hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(CT), args, 0, s));
  return SBFWI_OK;
}

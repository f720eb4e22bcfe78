// Per-step kernels of the condensed scheme (Section "Radial discretization").
//
// One wavefront per (element, group of S shots).  Items (i, s) -- boundary
// node i, shot s -- are spread over the 64 lanes.  Each radial level streams
// one dense block phi~_j^-1 (nb x nb FP64) from HBM into LDS, double
// buffered: the next level's block is loaded into registers while the current
// level is computed, so the HBM stream never waits on the level recursion.
//
// Forward sweep (condense), with y the swept residual source and
// q_j = phi~_j^-1 y_j:
//   y_0 = P_0 w_0,   y_j = P_j w_j - theta_j q_{j-1}   (j = 1 .. n),
//   f_hat = -theta_{n+1} q_{n-1} - G y_n,
// which equals the paper's p~_j = p_j - rho_j p~_{j-1}, p~_{n+1} = -rho_{n+1} p~_{n-1},
// f_hat = p~_{n+1} - G p~_n because rho_j = theta_j phi~_{j-1}^-1.
// Backward sweep (recover): u_n from the coarse solve, then
//   u_j = q_j - phi~_j^-1 (psi~_j u_{j+1})   (j = n-1 .. 0),
// the paper's u_j = phi~_j^-1 (p~_j - psi~_j u_{j+1}); then the Newmark update of
// velocity and acceleration at every level (eq. Newmark).
#include "sbfwi_internal.h"

namespace {

__device__ __forceinline__ int md(int i, int nb) { return i < 0 ? i + nb : (i >= nb ? i - nb : i); }

struct StepArgs {
  int NS;                 // shots in the run (stride of the shot index)
  double *u, *v, *a;      // interior state
  double *U, *V, *A;      // nodal state
  double *q, *yn, *fhat, *Unew;
  double *xs, *fs;        // optional stores (unknowns with ghosts, level field)
  int field_kind;         // fs: 0 = a^k, 1 = v^k
  double* vs;             // optional second level-field store (v^k) when fs holds a^k
};

template <int NBT, int S>
struct StepLds {
  double F[2][NBT * NBT];
  double w[NBT * S];
  double y[NBT * S];
  double x[NBT * S];
  double t[NBT * S];
  double u1[NBT * S];
};

constexpr int WT = 64;

template <int NBT>
__device__ __forceinline__ void prefetch(double (&reg)[(NBT * NBT + WT - 1) / WT], const double* src, int nbnb) {
#pragma unroll
  for (int r = 0; r < (NBT * NBT + WT - 1) / WT; ++r) {
    int q = threadIdx.x + r * WT;
    reg[r] = q < nbnb ? src[q] : 0.0;
  }
}

template <int NBT>
__device__ __forceinline__ void commit(const double (&reg)[(NBT * NBT + WT - 1) / WT], double* dst, int nb) {
#pragma unroll
  for (int r = 0; r < (NBT * NBT + WT - 1) / WT; ++r) {
    int q = threadIdx.x + r * WT;
    if (q < nb * nb) dst[(q / nb) * NBT + (q % nb)] = reg[r];
  }
}

// y(i, s) = band_row_i . vec(i-1, i, i+1; s)
__device__ __forceinline__ double band_mv(const double* band, const double* vec, int nb, int i, int s, int S) {
  return band[i] * vec[md(i - 1, nb) * S + s] + band[nb + i] * vec[i * S + s] +
         band[2 * nb + i] * vec[md(i + 1, nb) * S + s];
}

template <int NBT>
__device__ __forceinline__ double dense_mv(const double* F, const double* vec, int nb, int i, int s, int S) {
  double acc = 0.0;
  for (int c = 0; c < nb; ++c) acc += F[i * NBT + c] * vec[c * S + s];
  return acc;
}

template <int NBT, int S>
__global__ void __launch_bounds__(WT) condense_kernel(const int32_t* __restrict__ elems, MeshDev m,
                                                      FactorsDev f, StepArgs a) {
  __shared__ StepLds<NBT, S> L;
  const int e = elems[blockIdx.x];
  const int s0 = blockIdx.y * S;
  const int ns = min(S, a.NS - s0);
  const int nb = m.nb[e], n = m.nr[e] - 1, nbnb = nb * nb;
  const int64_t io = m.int_off[e], lo = m.loop_off[e], po = m.par_off[e];
  const double* Fe = f.finv + m.finv_off[e];
  const int items = nb * S;
  double reg[(NBT * NBT + WT - 1) / WT];
  prefetch<NBT>(reg, Fe, nbnb);
  commit<NBT>(reg, L.F[0], nb);
  int cur = 0;
  for (int j = 0; j <= n; ++j) {
    // w_j = a0 u + a1 v + a2 a (interior level, or the nodal state on the boundary level)
    for (int it = threadIdx.x; it < items; it += WT) {
      int i = it / S, s = it % S;
      double w = 0.0;
      if (s < ns) {
        if (j < n) {
          int64_t g = (io + (int64_t)j * nb + i) * a.NS + s0 + s;
          w = f.a0 * a.u[g] + f.a1 * a.v[g] + f.a2 * a.a[g];
        } else {
          int64_t g = m.loop_nodes[lo + i] * a.NS + s0 + s;
          w = f.a0 * a.U[g] + f.a1 * a.V[g] + f.a2 * a.A[g];
        }
      }
      L.w[it] = w;
    }
    if (j + 1 < n) prefetch<NBT>(reg, Fe + (int64_t)(j + 1) * nbnb, nbnb);
    __syncthreads();
    const double* pm = f.pm_band + 3 * (po + (int64_t)j * nb);
    const double* th = f.th_band + 3 * (po + (int64_t)j * nb);
    for (int it = threadIdx.x; it < items; it += WT) {
      int i = it / S, s = it % S;
      double y = band_mv(pm, L.w, nb, i, s, S);
      if (j > 0) y -= band_mv(th, L.x, nb, i, s, S);   // L.x holds q_{j-1}
      L.y[it] = y;
    }
    __syncthreads();
    if (j < n) {
      for (int it = threadIdx.x; it < items; it += WT) {
        int i = it / S, s = it % S;
        double qv = dense_mv<NBT>(L.F[cur], L.y, nb, i, s, S);
        L.t[it] = qv;
        if (s < ns) a.q[(io + (int64_t)j * nb + i) * a.NS + s0 + s] = qv;
      }
      if (j + 1 < n) commit<NBT>(reg, L.F[cur ^ 1], nb);
      __syncthreads();
      for (int it = threadIdx.x; it < items; it += WT) L.x[it] = L.t[it];  // q_j
      __syncthreads();
      cur ^= 1;
    }
  }
  // y_n -> global; f_hat = -theta_{n+1} q_{n-1} - G y_n
  const double* Ge = f.G + m.dense_off[e];
  prefetch<NBT>(reg, Ge, nbnb);
  commit<NBT>(reg, L.F[cur], nb);
  __syncthreads();
  const double* thn1 = f.th_np1 + 3 * lo;
  for (int it = threadIdx.x; it < items; it += WT) {
    int i = it / S, s = it % S;
    double fh = -band_mv(thn1, L.x, nb, i, s, S) - dense_mv<NBT>(L.F[cur], L.y, nb, i, s, S);
    if (s < ns) {
      a.yn[(lo + i) * a.NS + s0 + s] = L.y[it];
      a.fhat[(lo + i) * a.NS + s0 + s] = fh;
    }
  }
}

template <int NBT, int S>
__global__ void __launch_bounds__(WT) recover_kernel(const int32_t* __restrict__ elems, MeshDev m,
                                                     FactorsDev f, StepArgs a) {
  __shared__ StepLds<NBT, S> L;
  const int e = elems[blockIdx.x];
  const int s0 = blockIdx.y * S;
  const int ns = min(S, a.NS - s0);
  const int nb = m.nb[e], n = m.nr[e] - 1, nbnb = nb * nb;
  const int64_t io = m.int_off[e], lo = m.loop_off[e], po = m.par_off[e], xo = m.x_off[e];
  const double* Fe = f.finv + m.finv_off[e];
  const int items = nb * S;
  double reg[(NBT * NBT + WT - 1) / WT];
  prefetch<NBT>(reg, Fe + (int64_t)(n - 1) * nbnb, nbnb);
  commit<NBT>(reg, L.F[0], nb);
  for (int it = threadIdx.x; it < items; it += WT) {
    int i = it / S, s = it % S;
    double un = 0.0;
    if (s < ns) un = a.Unew[m.loop_nodes[lo + i] * a.NS + s0 + s];
    L.x[it] = un;
    L.w[it] = un;  // keep u_n for the ghost
    if (a.xs && s < ns) {
      a.xs[(xo + (int64_t)(n + 1) * nb + i) * a.NS + s0 + s] = un;
      double fv = a.field_kind == 0 ? a.A[m.loop_nodes[lo + i] * a.NS + s0 + s]
                                    : a.V[m.loop_nodes[lo + i] * a.NS + s0 + s];
      a.fs[(po + (int64_t)n * nb + i) * a.NS + s0 + s] = fv;
      if (a.vs) a.vs[(po + (int64_t)n * nb + i) * a.NS + s0 + s] = a.V[m.loop_nodes[lo + i] * a.NS + s0 + s];
    }
  }
  int cur = 0;
  __syncthreads();
  for (int j = n - 1; j >= 0; --j) {
    if (j > 0) prefetch<NBT>(reg, Fe + (int64_t)(j - 1) * nbnb, nbnb);
    // t = psi~_j u_{j+1}
    if (j > 0) {
      const double* ps = f.ps_band + 3 * (po + (int64_t)j * nb);
      for (int it = threadIdx.x; it < items; it += WT) L.t[it] = band_mv(ps, L.x, nb, it / S, it % S, S);
    } else {
      const double* P0 = f.psit0 + m.dense_off[e];
      for (int it = threadIdx.x; it < items; it += WT) {
        int i = it / S, s = it % S;
        double acc = 0.0;
        for (int c = 0; c < nb; ++c) acc += P0[i * nb + c] * L.x[c * S + s];
        L.t[it] = acc;
      }
    }
    __syncthreads();
    for (int it = threadIdx.x; it < items; it += WT) {
      int i = it / S, s = it % S;
      double uj = 0.0;
      if (s < ns) {
        int64_t g = (io + (int64_t)j * nb + i) * a.NS + s0 + s;
        uj = a.q[g] - dense_mv<NBT>(L.F[cur], L.t, nb, i, s, S);
        double uo = a.u[g], vo = a.v[g], ao = a.a[g];
        double w = f.a0 * uo + f.a1 * vo + f.a2 * ao;
        double vn = f.c1 * (uj - uo) + f.c2 * vo + f.c3 * ao;
        double an = f.a0 * uj - w;
        a.u[g] = uj;
        a.v[g] = vn;
        a.a[g] = an;
        if (a.xs) {
          a.xs[(xo + (int64_t)(j + 1) * nb + i) * a.NS + s0 + s] = uj;
          a.fs[(po + (int64_t)j * nb + i) * a.NS + s0 + s] = a.field_kind == 0 ? an : vn;
          if (a.vs) a.vs[(po + (int64_t)j * nb + i) * a.NS + s0 + s] = vn;
        }
      }
      L.y[it] = uj;
    }
    if (j > 0) commit<NBT>(reg, L.F[cur ^ 1], nb);
    __syncthreads();
    for (int it = threadIdx.x; it < items; it += WT) {
      if (j == 1) L.u1[it] = L.y[it];
      L.x[it] = L.y[it];
    }
    __syncthreads();
    cur ^= 1;
  }
  if (!a.xs) return;
  // ghosts: u_{-1} = theta_{-1}^-1 (-(phi_{-1} u_0 + psi_{-1} u_1)),
  //         u_{n+1} = psi_n^-1 (y_n - phi~_n u_n)
  const int64_t dofs = m.dense_off[e];
  const double* phm1 = f.phim1 + 3 * lo;
  const double* psm1 = f.psim1 + 3 * lo;
  for (int it = threadIdx.x; it < items; it += WT) {
    int i = it / S, s = it % S;
    L.t[it] = -(band_mv(phm1, L.x, nb, i, s, S) + band_mv(psm1, L.u1, nb, i, s, S));
    double acc = 0.0;
    const double* Pn = f.phit_n + dofs;
    for (int c = 0; c < nb; ++c) acc += Pn[i * nb + c] * L.w[c * S + s];
    L.y[it] = (s < ns ? a.yn[(lo + i) * a.NS + s0 + s] : 0.0) - acc;
  }
  __syncthreads();
  const double* Tm = f.thm1_inv + dofs;
  const double* Qn = f.psin_inv + dofs;
  for (int it = threadIdx.x; it < items; it += WT) {
    int i = it / S, s = it % S;
    double lo_g = 0.0, hi_g = 0.0;
    for (int c = 0; c < nb; ++c) {
      lo_g += Tm[i * nb + c] * L.t[c * S + s];
      hi_g += Qn[i * nb + c] * L.y[c * S + s];
    }
    if (s < ns) {
      a.xs[(xo + i) * a.NS + s0 + s] = lo_g;
      a.xs[(xo + (int64_t)(n + 2) * nb + i) * a.NS + s0 + s] = hi_g;
    }
  }
}

// F = sum of element sources gathered over node -> slot + point sources;
// Unew = initial guess of the coarse solve: the predictor u + dt v + dt^2/2 a
// plus the correction the previous step needed on top of its own predictor.
__global__ void rhs_kernel(MeshDev m, int NS, const double* __restrict__ fhat, double* __restrict__ F,
                           const double* __restrict__ U, const double* __restrict__ V,
                           const double* __restrict__ A, double* __restrict__ Unew,
                           const double* __restrict__ corr, double dt, SourceTable src, int64_t k) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= m.n_nodes * NS) return;
  int64_t node = g / NS;
  int s = (int)(g % NS);
  double acc = 0.0;
  for (int64_t t = m.node_ptr[node]; t < m.node_ptr[node + 1]; ++t) acc += fhat[m.node_slot[t] * NS + s];
  if (src.amp) {
    int64_t idx = src.reversed ? (src.amp_steps - k) : (k - 1);
    for (int c = 0; c < src.n_src; ++c) {
      int64_t nd = src.node[(src.node_stride ? (int64_t)s * src.n_src : 0) + c];
      if (nd == node) acc += src.amp[((int64_t)s * src.n_src + c) * src.amp_steps + idx];
    }
  }
  F[g] = acc;
  Unew[g] = U[g] + dt * V[g] + 0.5 * dt * dt * A[g] + corr[g];
}

// Nodal Newmark update, predictor correction and receiver sampling.
__global__ void nodal_kernel(int64_t n_nodes, int NS, FactorsDev f, const double* __restrict__ Unew,
                             double* __restrict__ U, double* __restrict__ V, double* __restrict__ A,
                             double* __restrict__ corr,
                             int n_rec, const int64_t* __restrict__ rec_node, double* __restrict__ traces,
                             int64_t n_steps, int64_t k) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t nn = n_nodes * NS;
  if (g < nn) {
    double uo = U[g], vo = V[g], ao = A[g], un = Unew[g];
    double w = f.a0 * uo + f.a1 * vo + f.a2 * ao;
    corr[g] = un - (uo + f.dt * vo + 0.5 * f.dt * f.dt * ao);
    V[g] = f.c1 * (un - uo) + f.c2 * vo + f.c3 * ao;
    A[g] = f.a0 * un - w;
    U[g] = un;
  } else if (traces && g < nn + (int64_t)n_rec * NS) {
    int64_t t = g - nn;
    int s = (int)(t / n_rec), r = (int)(t % n_rec);
    traces[((int64_t)s * n_rec + r) * n_steps + k - 1] = Unew[rec_node[r] * NS + s];
  }
}

template <int NBT, int S>
void launch_cr(bool condense, sbfwi_mesh_s* m, int cl, const FactorsDev& f, const StepArgs& a,
               hipStream_t st) {
  int64_t cnt = (int64_t)m->h_class_elems[cl].size();
  if (cnt == 0) return;
  dim3 grid((unsigned)cnt, (unsigned)((a.NS + S - 1) / S));
  if (condense)
    hipLaunchKernelGGL((condense_kernel<NBT, S>), grid, dim3(WT), 0, st, m->class_elems[cl], m->d, f, a);
  else
    hipLaunchKernelGGL((recover_kernel<NBT, S>), grid, dim3(WT), 0, st, m->class_elems[cl], m->d, f, a);
}

template <int S>
void launch_all(bool condense, sbfwi_mesh_s* m, const FactorsDev& f, const StepArgs& a, hipStream_t st) {
  launch_cr<8, S>(condense, m, 0, f, a, st);
  launch_cr<16, S>(condense, m, 1, f, a, st);
  launch_cr<24, S>(condense, m, 2, f, a, st);
}

void launch_sweep(bool condense, sbfwi_mesh_s* m, const FactorsDev& f, const StepArgs& a, hipStream_t st) {
  ProfScope ps(condense ? PK_CONDENSE : PK_RECOVER, st);
  if (a.NS >= 4)
    launch_all<4>(condense, m, f, a, st);
  else if (a.NS == 3 || a.NS == 2)
    launch_all<2>(condense, m, f, a, st);
  else
    launch_all<1>(condense, m, f, a, st);
}

}  // namespace

// interior u, v, a; nodal U, V, A and the predictor correction of the coarse solve
int64_t sbfwi_state_size(sbfwi_mesh_s* m, int NS) { return (3 * m->n_int + 4 * m->n_nodes) * (int64_t)NS; }

int sbfwi_step_work_alloc(StepWork* w, sbfwi_mesh_s* m, int NS) {
  w->NS = NS;
  int64_t ni = m->n_int * NS, nn = m->n_nodes * NS, nl = m->n_loop * NS;
  SBFWI_CHECK(sbfwi_alloc(&w->u, 3 * ni + 4 * nn));  // u, v, a, U, V, A, corr contiguous
  w->v = w->u + ni;
  w->a = w->v + ni;
  w->U = w->a + ni;
  w->V = w->U + nn;
  w->A = w->V + nn;
  w->corr = w->A + nn;
  SBFWI_CHECK(sbfwi_alloc(&w->q, ni));
  SBFWI_CHECK(sbfwi_alloc(&w->yn, nl));
  SBFWI_CHECK(sbfwi_alloc(&w->fhat, nl));
  SBFWI_CHECK(sbfwi_alloc(&w->F, nn));
  SBFWI_CHECK(sbfwi_alloc(&w->Unew, nn));
  SBFWI_CHECK(sbfwi_coarse_work_alloc(&w->cw, m->n_nodes, NS));
  return SBFWI_OK;
}

void sbfwi_step_work_free(StepWork* w) {
  sbfwi_dev_free(w->u);
  sbfwi_dev_free(w->q);
  sbfwi_dev_free(w->yn);
  sbfwi_dev_free(w->fhat);
  sbfwi_dev_free(w->F);
  sbfwi_dev_free(w->Unew);
  sbfwi_coarse_work_free(&w->cw);
  *w = StepWork();
}

int sbfwi_step_zero(sbfwi_mesh_s* m, StepWork* w, hipStream_t s) {
  SBFWI_HIP(hipMemsetAsync(w->u, 0, sizeof(double) * sbfwi_state_size(m, w->NS), s));
  return SBFWI_OK;
}

int sbfwi_state_copy(sbfwi_mesh_s* m, StepWork* w, double* dst, int to_store, hipStream_t s) {
  size_t bytes = sizeof(double) * sbfwi_state_size(m, w->NS);
  if (to_store)
    SBFWI_HIP(hipMemcpyAsync(dst, w->u, bytes, hipMemcpyDeviceToDevice, s));
  else
    SBFWI_HIP(hipMemcpyAsync(w->u, dst, bytes, hipMemcpyDeviceToDevice, s));
  return SBFWI_OK;
}

int sbfwi_forward_step(sbfwi_factors_s* f, StepWork* w, int64_t k, const SourceTable& src, int n_rec,
                       const int64_t* rec_node, double* traces, int64_t n_steps, double* xs, double* fs,
                       int field_kind, hipStream_t st, double* vs) {
  sbfwi_mesh_s* m = f->m;
  StepArgs a;
  a.NS = w->NS;
  a.u = w->u; a.v = w->v; a.a = w->a;
  a.U = w->U; a.V = w->V; a.A = w->A;
  a.q = w->q; a.yn = w->yn; a.fhat = w->fhat; a.Unew = w->Unew;
  a.xs = xs; a.fs = fs; a.field_kind = field_kind; a.vs = vs;
  launch_sweep(true, m, f->d, a, st);
  int64_t nn = m->n_nodes * w->NS;
  {
  ProfScope ps(PK_RHS, st);
  hipLaunchKernelGGL(rhs_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, m->d, w->NS, w->fhat,
                     w->F, w->U, w->V, w->A, w->Unew, w->corr, f->dt, src, k);
  }
  SBFWI_HIP(hipGetLastError());
  SBFWI_CHECK(sbfwi_coarse_solve(f, &w->cw, 0, w->F, w->Unew, k, st));
  int64_t tot = nn + (int64_t)n_rec * w->NS;
  {
  ProfScope ps(PK_NODAL, st);
  hipLaunchKernelGGL(nodal_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, m->n_nodes, w->NS,
                     f->d, w->Unew, w->U, w->V, w->A, w->corr, n_rec, rec_node, traces, n_steps, k);
  }
  launch_sweep(false, m, f->d, a, st);
  SBFWI_HIP(hipGetLastError());
  return SBFWI_OK;
}

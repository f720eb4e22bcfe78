// Time loop of the low-frequency expansion path (scheme 2).
//
// With radially constant density every element contributes a stiffness K_e
// and a mass M_e on its boundary nodes only (Section "Low-frequency
// expansion": S(omega) ~ K - omega^2 M).  The factor kernels form K_e as the
// static condensation of linear radial elements and M_e as their radial mass
// seen through the static modes, and assemble K_g + a0 M_g (factored once by
// the coarse solver) and M_g.  A Newmark step (eq. Newmark) is then nodal
// only: F = M_g w + f^k with w = a0 U + a1 V + a2 A, the coarse solve
// (K_g + a0 M_g) U' = F, and the update of V, A.  One thread per (node, shot)
// in every kernel; values are node-major with the shots innermost, as in the
// condensed path.
//
// The path's gradient is the paper's truncated kernel (implementation notes
// of Section "Numerical examples"): the time integral of the product of the
// forward and back-propagated velocities at the nodal points, the
// back-propagated field being this same time loop driven by the time-reversed
// residuals at the receivers.  The forward run keeps every step's nodal
// velocity for it.
#include "sbfwi_internal.h"

namespace {

// F = M_g (a0 U + a1 V + a2 A) + point forces of step k: one source per shot
// (n_rec = 0: wav[s][k - 1] at src[s]), or the receivers as sources with the
// time-reversed amplitudes wav[s][r][n_steps - k] (n_rec > 0, src = receivers).
__global__ void lfe_rhs_kernel(MeshDev m, int NS, FactorsDev f, const double* __restrict__ U,
                               const double* __restrict__ V, const double* __restrict__ A,
                               const int64_t* __restrict__ src, int n_rec, const double* __restrict__ wav,
                               int64_t n_steps, int64_t k, double* __restrict__ F) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= m.n_nodes * NS) return;
  const int64_t node = g / NS;
  const int s = (int)(g % NS);
  double acc = 0.0;
  for (int64_t t = m.row_ptr[node]; t < m.row_ptr[node + 1]; ++t) {
    const int64_t c = (int64_t)m.col[t] * NS + s;
    acc += f.Mval[t] * (f.a0 * U[c] + f.a1 * V[c] + f.a2 * A[c]);
  }
  if (n_rec == 0) {
    if (src[s] == node) acc += wav[(int64_t)s * n_steps + k - 1];
  } else {
    for (int r = 0; r < n_rec; ++r)
      if (src[r] == node) acc += wav[((int64_t)s * n_rec + r) * n_steps + (n_steps - k)];
  }
  F[g] = acc;
}

// Newmark update of V, A and U, and the receiver samples of step k.
__global__ void lfe_nodal_kernel(int64_t n_nodes, int NS, FactorsDev f, const double* __restrict__ Unew,
                                 double* __restrict__ U, double* __restrict__ V, double* __restrict__ A,
                                 int n_rec, const int64_t* __restrict__ rec, double* __restrict__ traces,
                                 int64_t n_steps, int64_t k, double* __restrict__ vstore,
                                 const double* __restrict__ vfwd, double* __restrict__ corr) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = n_nodes * NS;
  if (g < nn) {
    const double uo = U[g], vo = V[g], ao = A[g], un = Unew[g];
    const double w = f.a0 * uo + f.a1 * vo + f.a2 * ao;
    const double vn = f.c1 * (un - uo) + f.c2 * vo + f.c3 * ao;
    V[g] = vn;
    A[g] = f.a0 * un - w;
    U[g] = un;
    if (vstore) vstore[(k - 1) * nn + g] = vn;
    if (corr) corr[g] += vn * vfwd[g];   // back-propagation: zero-lag product with the forward velocity
  } else if (traces && g < nn + (int64_t)n_rec * NS) {
    const int64_t t = g - nn;
    const int s = (int)(t / n_rec), r = (int)(t % n_rec);
    traces[((int64_t)s * n_rec + r) * n_steps + k - 1] = Unew[rec[r] * NS + s];
  }
}

// grad[(s) + par_off[e] + (N_r - 1) n_b + k] += scale * corr at the node of loop slot k:
// every element's boundary-level density at a node takes that node's kernel.
__global__ void lfe_scatter_kernel(MeshDev m, int NS, const double* __restrict__ corr, double scale,
                                   double* __restrict__ grad, int64_t shot_stride) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (e >= m.n_elem) return;
  const int nb = m.nb[e], nr = m.nr[e];
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    const int64_t node = m.loop_nodes[m.loop_off[e] + k];
    const int64_t p = m.par_off[e] + (int64_t)(nr - 1) * nb + k;
    if (shot_stride == 0) {
      double t = 0.0;
      for (int s = 0; s < NS; ++s) t += corr[node * NS + s];
      grad[p] += scale * t;
    } else {
      for (int s = 0; s < NS; ++s) grad[s * shot_stride + p] += scale * corr[node * NS + s];
    }
  }
}

__global__ void lfe_zero_kernel(double* __restrict__ p, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0.0;
}

struct LfeWork {
  hipStream_t s = nullptr;
  double *U = nullptr, *V = nullptr, *A = nullptr, *F = nullptr, *Unew = nullptr;
  CoarseWork cw;
  ~LfeWork() {
    (void)hipStreamSynchronize(s);
    sbfwi_dev_free(U);
    sbfwi_dev_free(V);
    sbfwi_dev_free(A);
    sbfwi_dev_free(F);
    sbfwi_dev_free(Unew);
    sbfwi_coarse_work_free(&cw);
  }
};

}  // namespace

// One run of the time loop: sources as described at lfe_rhs_kernel; vstore
// (optional) keeps every step's velocity; vfwd/corr (optional) accumulate the
// zero-lag product with the kept forward velocities, step k pairing with
// forward step n_steps + 1 - k.
static int lfe_run(sbfwi_factors_s* f, int NS, int64_t n_steps, const int64_t* src, int n_src_rec,
                   const double* amp, int n_rec, const int64_t* rec_node, double* traces, double* vstore,
                   const double* vfwd, double* corr, hipStream_t s) {
  sbfwi_mesh_s* m = f->m;
  const int64_t nn = m->n_nodes * NS;
  LfeWork w;
  w.s = s;
  SBFWI_CHECK(sbfwi_alloc(&w.U, nn));
  SBFWI_CHECK(sbfwi_alloc(&w.V, nn));
  SBFWI_CHECK(sbfwi_alloc(&w.A, nn));
  SBFWI_CHECK(sbfwi_alloc(&w.F, nn));
  SBFWI_CHECK(sbfwi_alloc(&w.Unew, nn));
  SBFWI_CHECK(sbfwi_coarse_work_alloc(&w.cw, m, NS));
  const unsigned b = (unsigned)((nn + 255) / 256);
  for (double* p : {w.U, w.V, w.A, w.Unew}) hipLaunchKernelGGL(lfe_zero_kernel, dim3(b), dim3(256), 0, s, p, nn);
  int flags0[2] = {0, -1};
  SBFWI_HIP(hipMemcpyAsync(f->d.status, flags0, 2 * sizeof(int), hipMemcpyHostToDevice, s));
  const unsigned bn = (unsigned)((nn + (int64_t)(traces ? n_rec : 0) * NS + 255) / 256);
  for (int64_t k = 1; k <= n_steps; ++k) {
    hipLaunchKernelGGL(lfe_rhs_kernel, dim3(b), dim3(256), 0, s, m->d, NS, f->d, w.U, w.V, w.A, src, n_src_rec,
                       amp, n_steps, k, w.F);
    SBFWI_CHECK(sbfwi_coarse_solve(f, &w.cw, 0, w.F, w.Unew, k, s));
    hipLaunchKernelGGL(lfe_nodal_kernel, dim3(bn), dim3(256), 0, s, m->n_nodes, NS, f->d, w.Unew, w.U, w.V, w.A,
                       n_rec, rec_node, traces, n_steps, k, vstore,
                       vfwd ? vfwd + (n_steps - k) * nn : nullptr, corr);
  }
  SBFWI_HIP(hipGetLastError());
  int flags[2];
  SBFWI_HIP(hipMemcpyAsync(flags, f->d.status, sizeof(flags), hipMemcpyDeviceToHost, s));
  SBFWI_HIP(hipStreamSynchronize(s));
  if (flags[0] & 4) return sbfwi_fail(SBFWI_ENONFINITE, "non-finite coarse residual at step %d", flags[1]);
  if (flags[0] & 2) return sbfwi_fail(SBFWI_ENOCONV, "coarse solve did not converge at step %d", flags[1]);
  return SBFWI_OK;
}

int sbfwi_lfe_forward(sbfwi_factors_s* f, int n_shots, int64_t n_steps, const int64_t* src_node,
                      const double* wavelet, int n_rec, const int64_t* rec_node, double* traces, double* vstore,
                      hipStream_t s) {
  return lfe_run(f, n_shots, n_steps, src_node, 0, wavelet, n_rec, rec_node, traces, vstore, nullptr, nullptr, s);
}

int sbfwi_lfe_adjoint(sbfwi_factors_s* f, sbfwi_ckpt_s* ck, const double* adj_src, int per_shot, double* grad,
                      hipStream_t s) {
  sbfwi_mesh_s* m = f->m;
  const int NS = ck->n_shots;
  if (!ck->vstore) return sbfwi_fail(SBFWI_EINVAL, "the forward run kept no velocities");
  double* corr = nullptr;
  SBFWI_CHECK(sbfwi_alloc(&corr, m->n_nodes * NS));
  const int64_t nn = m->n_nodes * NS;
  hipLaunchKernelGGL(lfe_zero_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, corr, nn);
  int rc = lfe_run(f, NS, ck->n_steps, ck->rec_node, ck->n_rec, adj_src, 0, nullptr, nullptr, nullptr, ck->vstore,
                   corr, s);
  if (rc == SBFWI_OK) {
    const int64_t stride = per_shot ? m->n_params : 0;
    hipLaunchKernelGGL(lfe_scatter_kernel, dim3((unsigned)((m->n_elem + 7) / 8)), dim3(32, 8), 0, s, m->d, NS,
                       corr, -1.0, grad, stride);   // adj_src = dt (u - d): the rectangle rule's dt is in corr
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = sbfwi_fail(SBFWI_EHIP, "gradient scatter: %s", hipGetErrorString(e));
  }
  (void)hipStreamSynchronize(s);
  sbfwi_dev_free(corr);
  return rc;
}

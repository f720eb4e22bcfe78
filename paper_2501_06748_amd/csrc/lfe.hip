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
#include "sbfwi_internal.h"

namespace {

// F = M_g (a0 U + a1 V + a2 A) + point forces of step k.
__global__ void lfe_rhs_kernel(MeshDev m, int NS, FactorsDev f, const double* __restrict__ U,
                               const double* __restrict__ V, const double* __restrict__ A,
                               const int64_t* __restrict__ src, const double* __restrict__ wav, int64_t n_steps,
                               int64_t k, double* __restrict__ F) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= m.n_nodes * NS) return;
  const int64_t node = g / NS;
  const int s = (int)(g % NS);
  double acc = 0.0;
  for (int64_t t = m.row_ptr[node]; t < m.row_ptr[node + 1]; ++t) {
    const int64_t c = (int64_t)m.col[t] * NS + s;
    acc += f.Mval[t] * (f.a0 * U[c] + f.a1 * V[c] + f.a2 * A[c]);
  }
  if (src[s] == node) acc += wav[(int64_t)s * n_steps + k - 1];
  F[g] = acc;
}

// Newmark update of V, A and U, and the receiver samples of step k.
__global__ void lfe_nodal_kernel(int64_t n_nodes, int NS, FactorsDev f, const double* __restrict__ Unew,
                                 double* __restrict__ U, double* __restrict__ V, double* __restrict__ A,
                                 int n_rec, const int64_t* __restrict__ rec, double* __restrict__ traces,
                                 int64_t n_steps, int64_t k) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = n_nodes * NS;
  if (g < nn) {
    const double uo = U[g], vo = V[g], ao = A[g], un = Unew[g];
    const double w = f.a0 * uo + f.a1 * vo + f.a2 * ao;
    V[g] = f.c1 * (un - uo) + f.c2 * vo + f.c3 * ao;
    A[g] = f.a0 * un - w;
    U[g] = un;
  } else if (g < nn + (int64_t)n_rec * NS) {
    const int64_t t = g - nn;
    const int s = (int)(t / n_rec), r = (int)(t % n_rec);
    traces[((int64_t)s * n_rec + r) * n_steps + k - 1] = Unew[rec[r] * NS + s];
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

int sbfwi_lfe_forward(sbfwi_factors_s* f, int n_shots, int64_t n_steps, const int64_t* src_node,
                      const double* wavelet, int n_rec, const int64_t* rec_node, double* traces, hipStream_t s) {
  sbfwi_mesh_s* m = f->m;
  const int NS = n_shots;
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
  const unsigned bn = (unsigned)((nn + (int64_t)n_rec * NS + 255) / 256);
  for (int64_t k = 1; k <= n_steps; ++k) {
    hipLaunchKernelGGL(lfe_rhs_kernel, dim3(b), dim3(256), 0, s, m->d, NS, f->d, w.U, w.V, w.A, src_node, wavelet,
                       n_steps, k, w.F);
    SBFWI_CHECK(sbfwi_coarse_solve(f, &w.cw, 0, w.F, w.Unew, k, s));
    hipLaunchKernelGGL(lfe_nodal_kernel, dim3(bn), dim3(256), 0, s, m->n_nodes, NS, f->d, w.Unew, w.U, w.V, w.A,
                       n_rec, rec_node, traces, n_steps, k);
  }
  SBFWI_HIP(hipGetLastError());
  int flags[2];
  SBFWI_HIP(hipMemcpyAsync(flags, f->d.status, sizeof(flags), hipMemcpyDeviceToHost, s));
  SBFWI_HIP(hipStreamSynchronize(s));
  if (flags[0] & 4) return sbfwi_fail(SBFWI_ENONFINITE, "forward: non-finite coarse residual at step %d", flags[1]);
  if (flags[0] & 2) return sbfwi_fail(SBFWI_ENOCONV, "forward: coarse solve did not converge at step %d", flags[1]);
  return SBFWI_OK;
}

// Backward pass: exact discrete adjoint and the paper's truncated kernel.
//
// Step k of the forward scheme solves A X^k = P w^{k-1} + F^k for the
// uncondensed unknowns X (levels -1 .. n+1 of every element, level n shared
// at the nodes; eq. system) and updates velocity and acceleration (eq.
// Newmark).  Its exact reverse, given the adjoint seeds (u-bar, v-bar, a-bar)
// of the state after step k, is
//   u~ = u-bar + c1 v-bar + a0 a-bar (+ dt (u - d) at the receivers),
//   lambda = A^-T u~,
//   w-bar = P^T lambda - a-bar,
//   seeds of step k-1: u-bar = -c1 v-bar + a0 w-bar, v-bar = c2 v-bar + a1 w-bar,
//   a-bar = c3 v-bar + a2 w-bar,
// and the gradient gains -lambda^T (dA_stiff/drho) X^k + xi^2 lambda^T (dM0/drho) a^k
// (the a0 M0 part of A and P combine into the acceleration a^k = a0 u^k - w^{k-1}).
// u-bar enters the next step only through u~, so the interior levels keep u~
// in its place: the transposed condense reads one seed instead of three, and
// the joint transposed sweep, which hands u~ over in LDS, writes only v-bar and
// a-bar.
//
// A^-T reuses the forward factors transposed.  With the paper's block
// elimination A = L U (pivots theta_{-1}, phi~_0 .. phi~_{n-1}, psi_n, S), the
// transposed solve is U^T z = u~ swept upwards (z_j = phi~_j^-T (u~_j - psi~_{j-1}^T
// z_{j-1})), the coarse system K_g^T lambda_B = u~_B - sum_e psi_{n-1}^T z_{n-1},
// then L^T lambda = z swept downwards: lambda_n = -G^T lambda_{n+1},
// lambda_j = z_j - phi~_j^-T theta_{j+1}^T lambda_{j+1} (plus theta_{n+1}^T lambda_{n+1}
// at j = n-1), lambda_{-1} = -theta_{-1}^-T theta_0^T lambda_0.
//
// The gradient is the zero-lag correlation of the adjoint rows with the
// forward unknowns, contracted with the derivatives of the coefficient
// matrices with respect to the nodal densities of each level (eq. Es is
// linear in the densities); every thread owns one fine-grid parameter and
// sums over shots, so the accumulation is deterministic.
#include <atomic>

#include "fd_bands.h"
#include "sbfwi_internal.h"

namespace {

__device__ __forceinline__ int md(int i, int nb) { return i < 0 ? i + nb : (i >= nb ? i - nb : i); }

constexpr int WT = 64;

struct AdjArgs {
  int NS;
  double *ut, *vb, *ab;     // interior seeds, u-bar kept as u~ = u-bar + c1 v-bar + a0 a-bar
  double *UB, *VB, *AB;     // nodal seeds
  double *z, *gB, *pl, *lamB, *lam;
};

template <int NBT, int S>
struct AdjLds {
  double F[2][NBT * NBT];
  double x[NBT * S];
  double y[NBT * S];
  double t[NBT * S];
  double l1[NBT * S];
};

// loads are unconditional (lanes past the block reread word 0), so that the
// waits for them do not depend on branches
template <int NBT>
__device__ __forceinline__ void prefetch(double (&reg)[(NBT * NBT + WT - 1) / WT], const double* src, int nbnb) {
#pragma unroll
  for (int r = 0; r < (NBT * NBT + WT - 1) / WT; ++r) {
    int q = threadIdx.x + r * WT;
    const double v = src[q < nbnb ? q : 0];
    reg[r] = q < nbnb ? v : 0.0;
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

// (B^T x)_i for a band B: B[i-1][i] x_{i-1} + B[i][i] x_i + B[i+1][i] x_{i+1}
__device__ __forceinline__ double bandT_mv(const double* band, const double* vec, int nb, int i, int s, int S) {
  int im = md(i - 1, nb), ip = md(i + 1, nb);
  return band[2 * nb + im] * vec[im * S + s] + band[nb + i] * vec[i * S + s] + band[ip] * vec[ip * S + s];
}

__device__ __forceinline__ double band_mv(const double* band, const double* vec, int nb, int i, int s, int S) {
  return band[i] * vec[md(i - 1, nb) * S + s] + band[nb + i] * vec[i * S + s] +
         band[2 * nb + i] * vec[md(i + 1, nb) * S + s];
}

template <int NBT>
__device__ __forceinline__ double denseT_mv(const double* F, const double* vec, int nb, int i, int s, int S) {
  double acc = 0.0;
  for (int c = 0; c < nb; ++c) acc += F[c * NBT + i] * vec[c * S + s];
  return acc;
}

// Target of the stores of lanes without an item, so that every lane stores
// unconditionally and the waits for the prefetched level count exactly.
__device__ double g_adj_sink[WT];

// u~ = u-bar + c1 v-bar + a0 a-bar from a level's seeds, with explicit
// multiply-adds so that every sweep that forms it rounds it alike.
__device__ __forceinline__ double adj_utilde(const FactorsDev& f, double ub, double vb, double ab) {
  return fma(f.a0, ab, fma(f.c1, vb, ub));
}

// U^T sweep: z_j, and the coupling psi~_{n-1}^T z_{n-1} to the coarse rows.
// The next level's F block, seeds and psi~ band entries are loaded at the top
// of each level and consumed at its end; lanes without an item load word 0 of
// their arrays and store to g_adj_sink.
// JOINT: u~ of every level comes from ukeep (LDS, level-major, written by the
// transposed recover sweep of the later step in the same block) instead of the
// seeds in HBM.
// FLY (central differences, n_b <= 21): psi_{j-1} formed from the density rows
// (fd_bands.h) instead of loaded.
template <int NBT, int S, bool JOINT = false, bool FLY = false>
__device__ __forceinline__ void adj_condense_body(int e, int s0, const MeshDev& m, const FactorsDev& f,
                                                  const AdjArgs& a, AdjLds<NBT, S>& L,
                                                  const double* ukeep = nullptr) {
  constexpr int IPT = (NBT * S + WT - 1) / WT;
  const int ns = min(S, a.NS - s0);
  const int nb = m.nb[e], n = m.nr[e] - 1, nbnb = nb * nb;
  const int64_t io = m.int_off[e], lo = m.loop_off[e], po = m.par_off[e];
  const double* Fe = f.finv + m.finv_off[e];
  const int items = nb * S;
  int ii[IPT], si[IPT];
  bool own[IPT], ok[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int it = threadIdx.x + u * WT;
    own[u] = it < items;
    ii[u] = own[u] ? it / S : 0;
    si[u] = it % S;
    ok[u] = own[u] && si[u] < ns;
  }
  double reg[(NBT * NBT + WT - 1) / WT];
  double cu[IPT], cb[3][IPT];
  static_assert(!FLY || 3 * NBT <= WT, "rows on the fly need 3 n_b <= 64");
  // FLY: the call for level j forms row j and hands over row j - 1 (prev)
  FdSweepRows fr;
  double prev = 0.0;
  if constexpr (FLY) fr.init_up(f.bkap + lo * 3 * kFdKappa, f.rho + po, m.xi0, n, nb);
  // u~ of level j and the entries of psi~_{j-1}^T's row i (psi_0's for j = 0: unused)
  auto load_level = [&](int j, double (&uu)[IPT], double (&bd)[3][IPT]) {
    double psv = 0.0;
    if constexpr (FLY) {
      psv = prev;
      prev = fr.next_up().ps;
    }
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int i = ii[u];
      const int64_t g = ok[u] ? (io + (int64_t)j * nb + i) * a.NS + s0 + si[u] : 0;
      uu[u] = JOINT ? 0.0 : a.ut[g];   // with JOINT u~ comes from ukeep: no seed loads
      if constexpr (FLY) {
        bd[0][u] = __shfl(psv, 2 * nb + md(i - 1, nb), WT);
        bd[1][u] = __shfl(psv, nb + i, WT);
        bd[2][u] = __shfl(psv, md(i + 1, nb), WT);
      } else {
        const double* bp = f.ps_band + 3 * (po + (int64_t)(j > 0 ? j - 1 : 0) * nb);
        bd[0][u] = bp[2 * nb + md(i - 1, nb)];
        bd[1][u] = bp[nb + i];
        bd[2][u] = bp[md(i + 1, nb)];
      }
    }
  };
  prefetch<NBT>(reg, Fe, nbnb);
  commit<NBT>(reg, L.F[0], nb);
  load_level(0, cu, cb);
  int cur = 0;
  __syncthreads();
  __builtin_amdgcn_s_waitcnt(0);   // nothing in flight at the loop entry
  for (int j = 0; j < n; ++j) {
    const int jn = j + 1 < n ? j + 1 : n - 1;   // the last level reloads its own data (unused)
    prefetch<NBT>(reg, Fe + (int64_t)jn * nbnb, nbnb);
    double nu[IPT], nbd[3][IPT];
    load_level(jn, nu, nbd);
    // y = u~_j - psi~_{j-1}^T z_{j-1}
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int it = threadIdx.x + u * WT, i = ii[u], s = si[u];
      double y = JOINT ? ukeep[j * items + it] : (ok[u] ? cu[u] : 0.0);
      if (j == 1) {
        const double* P0 = f.psit0 + m.dense_off[e];
        double acc = 0.0;
        for (int c = 0; c < nb; ++c) acc += P0[c * nb + i] * L.x[c * S + s];
        y -= acc;
      } else if (j > 1) {
        y -= cb[0][u] * L.x[md(i - 1, nb) * S + s] + cb[1][u] * L.x[i * S + s] + cb[2][u] * L.x[md(i + 1, nb) * S + s];
      }
      if (own[u]) L.y[it] = y;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int it = threadIdx.x + u * WT, i = ii[u], s = si[u];
      const double zv = denseT_mv<NBT>(L.F[cur], L.y, nb, i, s, S);
      if (own[u]) L.t[it] = zv;
      const int64_t g = (io + (int64_t)j * nb + i) * a.NS + s0 + s;
      *(ok[u] ? a.z + g : g_adj_sink + threadIdx.x) = zv;
    }
    commit<NBT>(reg, L.F[cur ^ 1], nb);
    __syncthreads();
    for (int it = threadIdx.x; it < items; it += WT) L.x[it] = L.t[it];
    __syncthreads();
    cur ^= 1;
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      cu[u] = nu[u];
#pragma unroll
      for (int k = 0; k < 3; ++k) cb[k][u] = nbd[k][u];
    }
  }
  // coupling to the coarse rows: psi_{n-1}^T z_{n-1} (n >= 2, so psi~_{n-1} = psi_{n-1})
  const double* psn1 = f.ps_band + 3 * (po + (int64_t)(n - 1) * nb);
  for (int it = threadIdx.x; it < items; it += WT) {
    int i = it / S, s = it % S;
    if (s < ns) a.gB[(lo + i) * a.NS + s0 + s] = bandT_mv(psn1, L.x, nb, i, s, S);
  }
}

// Level loop of the L^T sweep (j = n-1 .. 0) with the adjoint Newmark chain;
// the next level's F block, z, seeds and the theta / P band entries are loaded
// at the top of each level and consumed at its end.
// KEEP: ukeep (LDS) receives u~ of the new seeds of every level, ukeep[j *
// items + it], for the transposed condense of the earlier step, in place of
// the u~ seeds in HBM.
// FLY: theta_{j+1} and P_j formed from the density rows instead of loaded.
template <int NBT, int S, bool LAM, bool KEEP, bool FLY>
__device__ __forceinline__ void adj_recover_levels(int e, int s0, const MeshDev& m, const FactorsDev& f,
                                                   const AdjArgs& a, AdjLds<NBT, S>& L,
                                                   double (&reg)[(NBT * NBT + WT - 1) / WT], double* ukeep) {
  constexpr int IPT = (NBT * S + WT - 1) / WT;
  const int ns = min(S, a.NS - s0);
  const int nb = m.nb[e], n = m.nr[e] - 1, nbnb = nb * nb;
  const int64_t io = m.int_off[e], lo = m.loop_off[e], po = m.par_off[e], xo = m.x_off[e];
  const double* Fe = f.finv + m.finv_off[e];
  const int items = nb * S;
  int ii[IPT], si[IPT];
  bool own[IPT], ok[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int it = threadIdx.x + u * WT;
    own[u] = it < items;
    ii[u] = own[u] ? it / S : 0;
    si[u] = it % S;
    ok[u] = own[u] && si[u] < ns;
  }
  double cz[IPT], cv[IPT], ca[IPT], ct[3][IPT], cp[3][IPT];
  static_assert(!FLY || 3 * NBT <= WT, "rows on the fly need 3 n_b <= 64");
  // FLY: rows from n down; the call for level j forms row j (P_j) and hands over
  // theta of row j + 1 (thn) formed by the call before
  FdSweepRows fr;
  double thn = 0.0;
  if constexpr (FLY) {
    fr.init_down(f.bkap + lo * 3 * kFdKappa, f.rho + po, m.xi0, n, nb);
    thn = fr.next_down().th;
  }
  // level j: z, v-bar and a-bar seeds, row i of theta_{j+1}^T and of P_j^T
  auto load_level = [&](int j, double (&zz)[IPT], double (&vv)[IPT], double (&aa)[IPT], double (&tb)[3][IPT],
                        double (&pb)[3][IPT]) {
    double thv = 0.0, pmv = 0.0;
    if constexpr (FLY) {
      const FdRow o = fr.next_down();
      thv = thn;
      pmv = o.pm;
      thn = o.th;
    }
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int i = ii[u], im = md(i - 1, nb), ip = md(i + 1, nb);
      const int64_t g = ok[u] ? (io + (int64_t)j * nb + i) * a.NS + s0 + si[u] : 0;
      zz[u] = a.z[g];
      vv[u] = a.vb[g];
      aa[u] = a.ab[g];
      if constexpr (FLY) {
        tb[0][u] = __shfl(thv, 2 * nb + im, WT);
        tb[1][u] = __shfl(thv, nb + i, WT);
        tb[2][u] = __shfl(thv, ip, WT);
        pb[0][u] = __shfl(pmv, 2 * nb + im, WT);
        pb[1][u] = __shfl(pmv, nb + i, WT);
        pb[2][u] = __shfl(pmv, ip, WT);
      } else {
        const double* tp = f.th_band + 3 * (po + (int64_t)(j + 1) * nb);
        const double* pp = f.pm_band + 3 * (po + (int64_t)j * nb);
        tb[0][u] = tp[2 * nb + im];
        tb[1][u] = tp[nb + i];
        tb[2][u] = tp[ip];
        pb[0][u] = pp[2 * nb + im];
        pb[1][u] = pp[nb + i];
        pb[2][u] = pp[ip];
      }
    }
  };
  load_level(n - 1, cz, cv, ca, ct, cp);
  int cur = 1;
  __syncthreads();
  __builtin_amdgcn_s_waitcnt(0);   // nothing in flight at the loop entry
  for (int j = n - 1; j >= 0; --j) {
    const int jn = j > 0 ? j - 1 : 0;   // the last level reloads level 0 (unused)
    prefetch<NBT>(reg, Fe + (int64_t)jn * nbnb, nbnb);
    double nz[IPT], nv[IPT], na[IPT], nt[3][IPT], np[3][IPT];
    load_level(jn, nz, nv, na, nt, np);
    // t = theta_{j+1}^T lambda_{j+1} (+ theta_{n+1}^T lambda_{n+1} when j = n-1)
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int it = threadIdx.x + u * WT, i = ii[u], s = si[u];
      double tv = ct[0][u] * L.x[md(i - 1, nb) * S + s] + ct[1][u] * L.x[i * S + s] + ct[2][u] * L.x[md(i + 1, nb) * S + s];
      if (j == n - 1) tv += bandT_mv(f.th_np1 + 3 * lo, L.l1, nb, i, s, S);
      if (own[u]) L.t[it] = tv;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int it = threadIdx.x + u * WT, i = ii[u], s = si[u];
      const double lv = ok[u] ? cz[u] - denseT_mv<NBT>(L.F[cur], L.t, nb, i, s, S) : 0.0;
      if (own[u]) L.y[it] = lv;
    }
    commit<NBT>(reg, L.F[cur ^ 1], nb);   // the last level commits an unused block
    __syncthreads();
    // adjoint Newmark chain at level j: w-bar = P_j^T lambda_j - a-bar
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int it = threadIdx.x + u * WT, i = ii[u], s = si[u];
      const int64_t g = (io + (int64_t)j * nb + i) * a.NS + s0 + s;
      const double vb = cv[u];
      const double wb = (cp[0][u] * L.y[md(i - 1, nb) * S + s] + cp[1][u] * L.y[i * S + s] +
                         cp[2][u] * L.y[md(i + 1, nb) * S + s]) - ca[u];
      double* sink = g_adj_sink + threadIdx.x;
      const double nub = -f.c1 * vb + f.a0 * wb, nvb = f.c2 * vb + f.a1 * wb, nab = f.c3 * vb + f.a2 * wb;
      const double ut = adj_utilde(f, nub, nvb, nab);
      if (KEEP) {   // u~ to the transposed condense in the same block
        if (own[u]) ukeep[j * items + it] = ok[u] ? ut : 0.0;
      } else {
        *(ok[u] ? a.ut + g : sink) = ut;
      }
      *(ok[u] ? a.vb + g : sink) = nvb;
      *(ok[u] ? a.ab + g : sink) = nab;
      if (LAM) *(ok[u] ? a.lam + (xo + (int64_t)(j + 1) * nb + i) * a.NS + s0 + s : sink) = own[u] ? L.y[it] : 0.0;
    }
    __syncthreads();
    for (int it = threadIdx.x; it < items; it += WT) L.x[it] = L.y[it];
    __syncthreads();
    cur ^= 1;
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      cz[u] = nz[u];
      cv[u] = nv[u];
      ca[u] = na[u];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        ct[k][u] = nt[k][u];
        cp[k][u] = np[k][u];
      }
    }
  }
}

// L^T sweep, adjoint Newmark chain at the interior levels, and P_n^T lambda_n.
// KEEP: u~ of the new seeds goes to ukeep (LDS) instead of the seeds in HBM.
template <int NBT, int S, bool KEEP = false, bool FLY = false>
__device__ __forceinline__ void adj_recover_body(int e, int s0, const MeshDev& m, const FactorsDev& f,
                                                 const AdjArgs& a, AdjLds<NBT, S>& L, double* ukeep = nullptr) {
  const int ns = min(S, a.NS - s0);
  const int nb = m.nb[e], n = m.nr[e] - 1, nbnb = nb * nb;
  const int64_t io = m.int_off[e], lo = m.loop_off[e], po = m.par_off[e], xo = m.x_off[e];
  const int64_t dofs = m.dense_off[e];
  const double* Fe = f.finv + m.finv_off[e];
  const int items = nb * S;
  double reg[(NBT * NBT + WT - 1) / WT];
  prefetch<NBT>(reg, f.G + dofs, nbnb);
  commit<NBT>(reg, L.F[0], nb);
  for (int it = threadIdx.x; it < items; it += WT) {
    int i = it / S, s = it % S;
    L.l1[it] = s < ns ? a.lamB[m.loop_nodes[lo + i] * a.NS + s0 + s] : 0.0;   // lambda_{n+1}
  }
  prefetch<NBT>(reg, Fe + (int64_t)(n - 1) * nbnb, nbnb);
  __syncthreads();
  // lambda_n = -G^T lambda_{n+1}
  for (int it = threadIdx.x; it < items; it += WT) {
    int i = it / S, s = it % S;
    L.x[it] = -denseT_mv<NBT>(L.F[0], L.l1, nb, i, s, S);
  }
  __syncthreads();
  commit<NBT>(reg, L.F[1], nb);
  const double* pmn = f.pm_band + 3 * (po + (int64_t)n * nb);
  for (int it = threadIdx.x; it < items; it += WT) {
    int i = it / S, s = it % S;
    if (s < ns) {
      a.pl[(lo + i) * a.NS + s0 + s] = bandT_mv(pmn, L.x, nb, i, s, S);
      if (a.lam) {
        a.lam[(xo + (int64_t)(n + 2) * nb + i) * a.NS + s0 + s] = L.l1[it];
        a.lam[(xo + (int64_t)(n + 1) * nb + i) * a.NS + s0 + s] = L.x[it];
      }
    }
  }
  __syncthreads();
  if (a.lam) adj_recover_levels<NBT, S, true, KEEP, FLY>(e, s0, m, f, a, L, reg, ukeep);
  else adj_recover_levels<NBT, S, false, KEEP, FLY>(e, s0, m, f, a, L, reg, ukeep);
  if (!a.lam) return;
  // lambda_{-1} = -theta_{-1}^-T theta_0^T lambda_0
  const double* th0 = f.th_band + 3 * po;
  for (int it = threadIdx.x; it < items; it += WT) L.t[it] = bandT_mv(th0, L.x, nb, it / S, it % S, S);
  __syncthreads();
  const double* Tm = f.thm1_inv + dofs;
  for (int it = threadIdx.x; it < items; it += WT) {
    int i = it / S, s = it % S;
    double acc = 0.0;
    for (int c = 0; c < nb; ++c) acc += Tm[c * nb + i] * L.t[c * S + s];
    if (s < ns) a.lam[(xo + i) * a.NS + s0 + s] = -acc;
  }
}


// One block per (element of an n_b class, group of S shots).
template <int NBT, int S, bool FLY>
__global__ void __launch_bounds__(WT) adj_condense_kernel(const int32_t* __restrict__ elems, int64_t n_el,
                                                          MeshDev m, FactorsDev f, AdjArgs a) {
  __shared__ AdjLds<NBT, S> L;
  int64_t ei;
  int g;
  if (!sweep_item(n_el, (a.NS + S - 1) / S, ei, g)) return;
  adj_condense_body<NBT, S, false, FLY>(elems[ei], g * S, m, f, a, L);
}

template <int NBT, int S, bool FLY>
__global__ void __launch_bounds__(WT) adj_recover_kernel(const int32_t* __restrict__ elems, int64_t n_el,
                                                         MeshDev m, FactorsDev f, AdjArgs a) {
  __shared__ AdjLds<NBT, S> L;
  int64_t ei;
  int g;
  if (!sweep_item(n_el, (a.NS + S - 1) / S, ei, g)) return;
  adj_recover_body<NBT, S, false, FLY>(elems[ei], g * S, m, f, a, L);
}

// Joint transposed sweep of one (element, group of S shots): the transposed
// recover of adjoint step k (down the levels), which keeps u~ of every level's
// new seeds in LDS, then the transposed condense of step k - 1 (up the levels)
// from them; the same expressions as the separate sweeps, so the same bits,
// with u~ handed over in LDS instead of written and read back, and one launch
// fewer.
template <int NBT, int S, bool FLY>
__global__ void __launch_bounds__(WT) adj_joint_kernel(const int32_t* __restrict__ elems, int64_t n_el, MeshDev m,
                                                       FactorsDev f, AdjArgs a) {
  __shared__ AdjLds<NBT, S> L;
  extern __shared__ double ukeep[];   // [interior levels][n_b * S] of the element
  int64_t ei;
  int g;
  if (!sweep_item(n_el, (a.NS + S - 1) / S, ei, g)) return;
  const int e = elems[ei];
  const int s0 = g * S;
  adj_recover_body<NBT, S, true, FLY>(e, s0, m, f, a, L, ukeep);
  __syncthreads();
  adj_condense_body<NBT, S, true, FLY>(e, s0, m, f, a, L, ukeep);
}

// One persistent launch over all n_b classes (work items in order of
// decreasing cost; LDS sized for the largest class).
template <int S, bool CONDENSE>
__global__ void __launch_bounds__(WT) adj_sweep_fused_kernel(const int32_t* __restrict__ order, int64_t n_work,
                                                             int groups, MeshDev m, FactorsDev f, AdjArgs a) {
  __shared__ AdjLds<24, S> L;
  for (int64_t w = blockIdx.x; w < n_work; w += gridDim.x) {
    const int e = order[w / groups];
    const int s0 = (int)(w % groups) * S;
    const int nb = m.nb[e];
    if (nb <= 8) {
      auto& Ls = *reinterpret_cast<AdjLds<8, S>*>(&L);
      if (CONDENSE) adj_condense_body<8, S>(e, s0, m, f, a, Ls); else adj_recover_body<8, S>(e, s0, m, f, a, Ls);
    } else if (nb <= 16) {
      auto& Ls = *reinterpret_cast<AdjLds<16, S>*>(&L);
      if (CONDENSE) adj_condense_body<16, S>(e, s0, m, f, a, Ls); else adj_recover_body<16, S>(e, s0, m, f, a, Ls);
    } else {
      if (CONDENSE) adj_condense_body<24, S>(e, s0, m, f, a, L); else adj_recover_body<24, S>(e, s0, m, f, a, L);
    }
    __syncthreads();
  }
}

// rhs_B = u~_B - sum_e psi_{n-1}^T z_{n-1} + adjoint source at the receivers,
// for item g = (node, shot) from the nodal adjoint state (ub, vb, ab) of the item.
__device__ __forceinline__ double adj_rhs_at(int64_t g, int NS, const MeshDev& m, const FactorsDev& f,
                                             const AdjArgs& a, double ub, double vb, double ab, int n_rec,
                                             const int64_t* __restrict__ rec_node, const double* __restrict__ adj,
                                             int64_t n_steps, int64_t k) {
  const int64_t node = g / NS;
  const int s = (int)(g % NS);
  double acc = ub + f.c1 * vb + f.a0 * ab;
  acc = node_gather<true>(acc, m.node_slot, m.node_ptr[node], m.node_ptr[node + 1], a.gB, NS, s);
  if (adj)
    for (int r = 0; r < n_rec; ++r)
      if (rec_node[r] == node) acc += adj[((int64_t)s * n_rec + r) * n_steps + k - 1];
  return acc;
}

// Nodal adjoint Newmark chain of item g: the new (ub, vb, ab), stored.
__device__ __forceinline__ void adj_nodal_at(int64_t g, int NS, const MeshDev& m, const FactorsDev& f,
                                             const AdjArgs& a, double& ub, double& vb, double& ab) {
  const int64_t node = g / NS;
  const int s = (int)(g % NS);
  double wb = -a.AB[g];
  wb = node_gather<false>(wb, m.node_slot, m.node_ptr[node], m.node_ptr[node + 1], a.pl, NS, s);
  const double v = a.VB[g];
  ub = -f.c1 * v + f.a0 * wb;
  vb = f.c2 * v + f.a1 * wb;
  ab = f.c3 * v + f.a2 * wb;
  a.UB[g] = ub;
  a.VB[g] = vb;
  a.AB[g] = ab;
}

__global__ void adj_rhs_kernel(MeshDev m, int NS, FactorsDev f, AdjArgs a, double* __restrict__ rhs,
                               int n_rec, const int64_t* __restrict__ rec_node, const double* __restrict__ adj,
                               int64_t n_steps, int64_t k) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= m.n_nodes * NS) return;
  rhs[g] = adj_rhs_at(g, NS, m, f, a, a.UB[g], a.VB[g], a.AB[g], n_rec, rec_node, adj, n_steps, k);
}

__global__ void adj_nodal_kernel(MeshDev m, int NS, FactorsDev f, AdjArgs a) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= m.n_nodes * NS) return;
  double ub, vb, ab;
  adj_nodal_at(g, NS, m, f, a, ub, vb, ab);
}

// The nodal chain of adjoint step k + 1 and the right-hand side of step k in
// one pass over the items (nothing between them reads or writes the nodal
// adjoint state once the joint transposed sweep has condensed step k).
__global__ void adj_nodal_rhs_kernel(MeshDev m, int NS, FactorsDev f, AdjArgs a, double* __restrict__ rhs,
                                     int n_rec, const int64_t* __restrict__ rec_node,
                                     const double* __restrict__ adj, int64_t n_steps, int64_t k) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= m.n_nodes * NS) return;
  double ub, vb, ab;
  adj_nodal_at(g, NS, m, f, a, ub, vb, ab);
  rhs[g] = adj_rhs_at(g, NS, m, f, a, ub, vb, ab, n_rec, rec_node, adj, n_steps, k);
}

// Lanes of one wavefront exchanging values through LDS: the LDS operations of
// a wave complete in issue order, so only the compiler's code motion has to be
// fenced (the block of these kernels is exactly one wavefront).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Adds the gradient of levels l0c .. lev (collected in Gb by item) to grad.
// Every entry receives one addition per launch (launches are ordered on the
// stream), so the hardware's floating-point add at the memory side gives the
// same result as a read-modify-write, without the lane waiting for the read.
template <int NBT, int S, int GCH>
__device__ __forceinline__ void flush_chunk(const double (&Gb)[GCH][NBT * S], int l0c, int lev, int nb, int ns,
                                            int it, int s0, int64_t po, int64_t shot_stride,
                                            double* __restrict__ grad) {
  const int nl = lev - l0c + 1;
  if (shot_stride == 0) {
    for (int q = it; q < nl * nb; q += WT) {
      const int l = q / nb, k = q % nb;
      double t = 0.0;
      for (int u = 0; u < ns; ++u) t += Gb[l][k * S + u];
      unsafeAtomicAdd(grad + po + (int64_t)(l0c + l) * nb + k, t);
    }
  } else {
    for (int q = it; q < nl * nb * ns; q += WT) {
      const int l = q / (nb * ns), r = q % (nb * ns), k = r / ns, u = r % ns;
      unsafeAtomicAdd(grad + (int64_t)(s0 + u) * shot_stride + po + (int64_t)(l0c + l) * nb + k, Gb[l][k * S + u]);
    }
  }
}

// Exact gradient for one step: one wavefront per (element, group of S shots),
// one item (boundary node i, shot s) per lane.  At level m the band entries of
// the sensitivities of E0, E1, E2 and M0 are short sums of products of
// quantities of the two nodes involved:
//   e0(i, j) = sum_a lam_i[a] Q_j[a]        e1(i, j) = sum_a R_i[a] lam_j[a] - lam_i[1] T_j
//   e2(i, j) = -lam_i[1] X_j(m)             m0(i, j) = lam_i[1] acc_j(m)
// with lam[a] the adjoint rows m-1, m, m+1 and Q, R, T the forward unknowns'
// radial differences weighted by the FD stencil of every row that touches
// level m (one-sided at the ends, plus the flux rows at xi0 and at the
// boundary).  Each lane forms the 12 quantities of its node from register
// windows of X (levels m-2 .. m+2), lam (rows m-1 .. m+1) and the
// accelerations (level m), takes those of node i+1 from that node's lane by
// cross-lane permutes, evaluates the four band entries of the segment
// (i, i+1) it owns and contracts them with that segment's density derivatives
// alpha (registers): the end-0 part is node i's, the end-1 part is passed to
// node i+1's lane the same way.  The next level's X, lam and accelerations are
// loaded while the current level is computed; the results of GCH levels
// collect in LDS and are added to the gradient together.
template <int NBT, int S>
__device__ __forceinline__ void grad_exact_group(int e, const MeshDev& m, const FactorsDev& f, int NS,
                                                 const double* __restrict__ X, const double* __restrict__ lam,
                                                 const double* __restrict__ acc_a, double* __restrict__ grad,
                                                 int s0, int64_t shot_stride) {
  static_assert(NBT * S <= WT, "one (node, shot) item per lane");
  constexpr int GCH = 16;
  __shared__ double Gb[GCH][NBT * S]; // gradient per level of the chunk and item
  const int ns = min(S, NS - s0);
  const int nb = m.nb[e], n = m.nr[e] - 1;
  const int64_t po = m.par_off[e], lo = m.loop_off[e], xo = m.x_off[e];
  const double h = (1.0 - m.xi0) / n, xi0 = m.xi0;
  // 1/h and 1/(2h) once per element: the per-level coefficients below then
  // take multiplications only (an FP64 division is about ten instructions)
  const double ih = 1.0 / h, i2h = 0.5 * ih;
  const int it = threadIdx.x;
  const bool own = it < nb * S;           // the lane holds an item (node i, shot s)
  const int i = own ? it / S : 0, s = it % S;
  const bool act = own && s < ns;         // ... of a shot of the run
  const int itp = md(i + 1, nb) * S + s;  // item of node i + 1, end 1 of segment (i, i + 1)
  const int itm = md(i - 1, nb) * S + s;  // item of node i - 1, whose segment ends at node i
  const bool summed = shot_stride == 0;
  double al[32];   // alpha of segment (i, i + 1): [tau * 8 + end * 4 + k], then M0 at 24 + end * 4 + k
#pragma unroll
  for (int q = 0; q < 32; ++q) al[q] = own ? f.gbasis[32 * (lo + i) + q] : 0.0;
  // loads are unconditional (a lane without a value reads word 0 and drops it), so
  // that the waits for the prefetched level do not depend on branches
  auto ldx = [&](int l) -> double {
    const bool ok = act && l <= n + 1;
    const double v = X[ok ? (xo + (int64_t)(l + 1) * nb + i) * NS + s0 + s : 0];
    return ok ? v : 0.0;
  };
  auto ldl = [&](int r) -> double {
    const bool ok = act && r <= n + 1;
    const double v = lam[ok ? (xo + (int64_t)(r + 1) * nb + i) * NS + s0 + s : 0];
    return ok ? v : 0.0;
  };
  auto lda = [&](int l) -> double {
    const bool ok = act && l <= n;
    const double v = acc_a[ok ? (po + (int64_t)l * nb + i) * NS + s0 + s : 0];
    return ok ? v : 0.0;
  };
  // FD weight of level mm in the radial derivative at row r (one-sided at the ends)
  auto dw = [&](int r, int mm) -> double {
    if (r == 0) return mm == 0 ? -ih : (mm == 1 ? ih : 0.0);
    if (r == n) return mm == n - 1 ? -ih : (mm == n ? ih : 0.0);
    return mm == r - 1 ? -i2h : (mm == r + 1 ? i2h : 0.0);
  };
  // windows at level 0 (X(-2) does not exist: its weights are zero)
  double x0 = 0.0, x1 = ldx(-1), x2 = ldx(0), x3 = ldx(1), x4 = ldx(2);
  double l0 = ldl(-1), l1 = ldl(0), l2 = ldl(1);
  double aw = lda(0);
  for (int lev = 0; lev <= n; ++lev) {
    const double px = ldx(lev + 3), pl = ldl(lev + 2), pa = lda(lev + 1);
    const double xm = xi0 + h * lev, hm = xm * i2h;
    // weights of rows lev - 1, lev, lev + 1: c for the E0 terms, b for the E1 terms
    double cw[3], bw[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int r = lev - 1 + a;
      const double w = (r >= 0 && r <= n) ? dw(r, lev) : 0.0, xr = xi0 + h * r;
      cw[a] = w * xr * xr * i2h;
      bw[a] = w * xr;
    }
    const double f0 = lev == 0 ? xi0 * i2h : 0.0, g0 = lev == 0 ? 1.0 : 0.0;
    const double fn = lev == n ? (xi0 + h * n) * i2h : 0.0, gn = lev == n ? 1.0 : 0.0;
    // this node's quantities
    const double dm = x2 - x0, d0 = x3 - x1, dp = x4 - x2, T = hm * d0;
    const double Lp[3] = {l0, l1, l2};
    const double Qp[3] = {cw[0] * dm + f0 * d0, xm * xm * (ih * ih) * (x1 - 2.0 * x2 + x3) + T + cw[1] * d0,
                          cw[2] * dp + fn * d0};
    const double Rp[3] = {bw[0] * x1 + g0 * x2, T + bw[1] * x2, bw[2] * x3 + gn * x2};
    // node i + 1's quantities from its lane (every lane takes part in the exchange)
    double Lq[3], Qq[3], Rq[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Lq[a] = __shfl(Lp[a], itp, WT);
      Qq[a] = __shfl(Qp[a], itp, WT);
      Rq[a] = __shfl(Rp[a], itp, WT);
    }
    const double Tq = __shfl(T, itp, WT), Xq = __shfl(x2, itp, WT), Aq = __shfl(aw, itp, WT);
    {
      // band entries (p, p), (p, q), (q, p), (q, q) of the segment, p = i, q = i + 1
      const double E0[4] = {Lp[0] * Qp[0] + Lp[1] * Qp[1] + Lp[2] * Qp[2],
                            Lp[0] * Qq[0] + Lp[1] * Qq[1] + Lp[2] * Qq[2],
                            Lq[0] * Qp[0] + Lq[1] * Qp[1] + Lq[2] * Qp[2],
                            Lq[0] * Qq[0] + Lq[1] * Qq[1] + Lq[2] * Qq[2]};
      const double E1[4] = {Rp[0] * Lp[0] + Rp[1] * Lp[1] + Rp[2] * Lp[2] - Lp[1] * T,
                            Rp[0] * Lq[0] + Rp[1] * Lq[1] + Rp[2] * Lq[2] - Lp[1] * Tq,
                            Rq[0] * Lp[0] + Rq[1] * Lp[1] + Rq[2] * Lp[2] - Lq[1] * T,
                            Rq[0] * Lq[0] + Rq[1] * Lq[1] + Rq[2] * Lq[2] - Lq[1] * Tq};
      const double E2[4] = {-Lp[1] * x2, -Lp[1] * Xq, -Lq[1] * x2, -Lq[1] * Xq};
      const double M0[4] = {Lp[1] * aw, Lp[1] * Aq, Lq[1] * aw, Lq[1] * Aq};
      double s0e = 0.0, s1e = 0.0, s0m = 0.0, s1m = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        s0e += al[k] * E0[k] + al[8 + k] * E1[k] + al[16 + k] * E2[k];
        s1e += al[4 + k] * E0[k] + al[12 + k] * E1[k] + al[20 + k] * E2[k];
        s0m += al[24 + k] * M0[k];
        s1m += al[28 + k] * M0[k];
      }
      const double end0 = xm * xm * s0m - s0e, end1 = xm * xm * s1m - s1e;
      // the end-1 part of segment (i - 1, i) comes from that segment's lane
      const double c1 = __shfl(end1, itm, WT);
      if (own) Gb[lev % GCH][it] = end0 + c1;
    }
    if (lev % GCH == GCH - 1 || lev == n) {       // add the chunk's levels to the gradient
      wave_lds_sync();
      flush_chunk<NBT, S, GCH>(Gb, lev - lev % GCH, lev, nb, ns, it, s0, po, shot_stride, grad);
      wave_lds_sync();
    }
    x0 = x1; x1 = x2; x2 = x3; x3 = x4; x4 = px;
    l0 = l1; l1 = l2; l2 = pl;
    aw = pa;
  }
}

// Exact gradient of the radial Galerkin scheme for one step, in the lane
// organisation of grad_exact_group.  The level matrices E_m enter the
// Galerkin blocks of the two intervals around level m (as the interpolation
// end 1 of interval m - 1 and end 0 of interval m), so the band entries of
// the sensitivities at level m are
//   e0(i, j) = sum_a L_a[i] Q_a[j]      e1(i, j) = sum_a (L_a[i] Zb_a[j] + Za_a[i] L_a[j])
//   e2(i, j) = sum_a L_a[i] Y_a[j]      m0(i, j) = sum_a L_a[i] A_a[j]
// over the Galerkin rows r = m - 1 + a (a = 0, 1, 2): L_a is the adjoint of
// row r with the sign that makes the gradient -lambda^T dR/drho (rows of the
// interior levels are stored negated; the boundary row is row n + 1 of the
// layout), Q, Za, Zb, Y the unknowns of levels m - 1 .. m + 1 weighted by the
// quadrature weights of E0, E1^T, E1 and E2 in block (r, l), and A the
// accelerations weighted by the lumped-mass weights.  (For the boundary row
// the mass term uses the boundary level's acceleration with the boundary
// row's adjoint, which equals the identity row's adjoint of the unused level
// n + 1.)
template <int NBT, int S>
__device__ __forceinline__ void grad_rg_group(int e, const MeshDev& m, const FactorsDev& f, int NS,
                                              const double* __restrict__ X, const double* __restrict__ lam,
                                              const double* __restrict__ acc_a, double* __restrict__ grad, int s0,
                                              int64_t shot_stride, const double* W) {
  static_assert(NBT * S <= WT, "one (node, shot) item per lane");
  constexpr int GCH = 16;
  __shared__ double Gb[GCH][NBT * S]; // gradient per level of the chunk and item
  const int ns = min(S, NS - s0);
  const int nb = m.nb[e], n = m.nr[e] - 1;
  const int64_t po = m.par_off[e], lo = m.loop_off[e], xo = m.x_off[e];
  const int it = threadIdx.x;
  const bool own = it < nb * S;
  const int i = own ? it / S : 0, s = it % S;
  const bool act = own && s < ns;
  const int itp = md(i + 1, nb) * S + s;  // item of node i + 1
  const int itm = md(i - 1, nb) * S + s;  // item of node i - 1
  const bool summed = shot_stride == 0;
  double al[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) al[q] = own ? f.gbasis[32 * (lo + i) + q] : 0.0;
  auto ldx = [&](int l) -> double {   // unknowns of level l (0 .. n)
    const bool ok = act && l >= 0 && l <= n;
    const double v = X[ok ? (xo + (int64_t)(l + 1) * nb + i) * NS + s0 + s : 0];
    return ok ? v : 0.0;
  };
  auto ldl = [&](int r) -> double {   // adjoint of Galerkin row r (0 .. n) as stored
    const bool ok = act && r >= 0 && r <= n;
    const int fr = r < n ? r : n + 1;
    const double v = lam[ok ? (xo + (int64_t)(fr + 1) * nb + i) * NS + s0 + s : 0];
    return ok ? v : 0.0;
  };
  // the boundary row's adjoint is stored with the opposite sign; the sign is
  // applied where the value is used, so that no load waits inside a branch
  auto sgn = [&](int r, double v) { return r == n ? -v : v; };
  auto lda = [&](int l) -> double {
    const bool ok = act && l >= 0 && l <= n;
    const double v = acc_a[ok ? (po + (int64_t)l * nb + i) * NS + s0 + s : 0];
    return ok ? v : 0.0;
  };
  double xa = 0.0, xb = ldx(0), xc = ldx(1);       // levels m - 1, m, m + 1
  double la = 0.0, lb = ldl(0), lc = ldl(1);       // rows m - 1, m, m + 1
  double aa = 0.0, ab = lda(0), ac = lda(1);
  for (int lev = 0; lev <= n; ++lev) {
    const double px = ldx(lev + 2), pl = ldl(lev + 2), pa = lda(lev + 2);
    // weights of interval lev - 1 (level lev at its end 1) and interval lev (end 0)
    const double* wl = W + (int64_t)(lev >= 1 ? lev - 1 : 0) * kRgW;
    const double* wr = W + (int64_t)(lev < n ? lev : n - 1) * kRgW;
    const bool hl = lev >= 1, hr = lev < n;
    // both tables exist for every level (an element has at least one interval):
    // unconditional loads, then a select, so that no branch orders the waits
    auto wL = [&](int o) {
      const double v = wl[o];
      return hl ? v : 0.0;
    };
    auto wR = [&](int o) {
      const double v = wr[o];
      return hr ? v : 0.0;
    };
    double Qk[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int b = 8 * k;
      Qk[k][0] = wL(b + 0 + 0 + 1) * xa + wL(b + 0 + 2 + 1) * xb;
      Qk[k][1] = wL(b + 4 + 0 + 1) * xa + wL(b + 4 + 2 + 1) * xb + wR(b + 0 + 0 + 0) * xb + wR(b + 0 + 2 + 0) * xc;
      Qk[k][2] = wR(b + 4 + 0 + 0) * xb + wR(b + 4 + 2 + 0) * xc;
    }
    const double Ap[3] = {wL(32 + 0 + 1) * aa, (wL(32 + 2 + 1) + wR(32 + 0 + 0)) * ab, wR(32 + 2 + 0) * ac};
    const double Lp[3] = {sgn(lev - 1, la), sgn(lev, lb), sgn(lev + 1, lc)};
    // node i + 1's quantities from its lane (every lane takes part in the exchange)
    double Lq[3], Qq[3], Zaq[3], Zbq[3], Yq[3], Aq[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Lq[a] = __shfl(Lp[a], itp, WT);
      Qq[a] = __shfl(Qk[0][a], itp, WT);
      Zaq[a] = __shfl(Qk[1][a], itp, WT);
      Zbq[a] = __shfl(Qk[2][a], itp, WT);
      Yq[a] = __shfl(Qk[3][a], itp, WT);
      Aq[a] = __shfl(Ap[a], itp, WT);
    }
    {
      double E0[4] = {0, 0, 0, 0}, E1[4] = {0, 0, 0, 0}, E2[4] = {0, 0, 0, 0}, M0[4] = {0, 0, 0, 0};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        E0[0] += Lp[a] * Qk[0][a]; E0[1] += Lp[a] * Qq[a]; E0[2] += Lq[a] * Qk[0][a]; E0[3] += Lq[a] * Qq[a];
        E1[0] += Lp[a] * Qk[2][a] + Qk[1][a] * Lp[a];
        E1[1] += Lp[a] * Zbq[a] + Qk[1][a] * Lq[a];
        E1[2] += Lq[a] * Qk[2][a] + Zaq[a] * Lp[a];
        E1[3] += Lq[a] * Zbq[a] + Zaq[a] * Lq[a];
        E2[0] += Lp[a] * Qk[3][a]; E2[1] += Lp[a] * Yq[a]; E2[2] += Lq[a] * Qk[3][a]; E2[3] += Lq[a] * Yq[a];
        M0[0] += Lp[a] * Ap[a]; M0[1] += Lp[a] * Aq[a]; M0[2] += Lq[a] * Ap[a]; M0[3] += Lq[a] * Aq[a];
      }
      double s0e = 0.0, s1e = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        s0e += al[k] * E0[k] + al[8 + k] * E1[k] + al[16 + k] * E2[k] + al[24 + k] * M0[k];
        s1e += al[4 + k] * E0[k] + al[12 + k] * E1[k] + al[20 + k] * E2[k] + al[28 + k] * M0[k];
      }
      // the end-1 part of segment (i - 1, i) comes from that segment's lane
      const double c1 = __shfl(s1e, itm, WT);
      if (own) Gb[lev % GCH][it] = s0e + c1;
    }
    if (lev % GCH == GCH - 1 || lev == n) {
      wave_lds_sync();
      flush_chunk<NBT, S, GCH>(Gb, lev - lev % GCH, lev, nb, ns, it, s0, po, shot_stride, grad);
      wave_lds_sync();
    }
    xa = xb; xb = xc; xc = px;
    la = lb; lb = lc; lc = pl;
    aa = ab; ab = ac; ac = pa;
  }
}

// Paper kernel: g -= w * sum_s v~ v at every fine-grid point.  The back-propagated
// run is driven by adj_src = dt (u - d), dt times the paper's residual source, so
// the rectangle rule's dt of the kernel's time integral is already in v~ (w = 1).
__global__ void grad_paper_kernel(int NS, double w, int64_t n_params, const double* __restrict__ vb,
                                  const double* __restrict__ vf, double* __restrict__ grad, int per_shot) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_params) return;
  double g = 0.0;
  for (int s = 0; s < NS; ++s) {
    const double vl = vb[p * NS + s];
    if (per_shot)
      grad[s * n_params + p] -= w * (vl * vf[p * NS + s]);
    else
      g += vl * vf[p * NS + s];
  }
  if (!per_shot) grad[p] -= w * g;
}

__global__ void misfit_kernel(const double* __restrict__ tr, const double* __restrict__ ob, int64_t count,
                              double dt, double* __restrict__ res, double* __restrict__ misfit) {
  __shared__ double ws[16];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += blockDim.x) {
    double r = tr[i] - ob[i];
    if (res) res[i] = dt * r;
    acc += r * r;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += ws[w];
    misfit[0] = 0.5 * dt * t;
  }
}

template <int NBT, int S>
void launch_adj(bool condense, sbfwi_mesh_s* m, int cl, const FactorsDev& f, const AdjArgs& a, hipStream_t st) {
  int64_t cnt = (int64_t)m->h_class_elems[cl].size();
  if (cnt == 0) return;
  dim3 grid((unsigned)sweep_blocks(cnt, (a.NS + S - 1) / S));
  if constexpr (3 * NBT <= WT) {
    if (sbfwi_fly_rows(f)) {
      if (condense)
        hipLaunchKernelGGL((adj_condense_kernel<NBT, S, true>), grid, dim3(WT), 0, st, m->class_elems[cl], cnt, m->d,
                           f, a);
      else
        hipLaunchKernelGGL((adj_recover_kernel<NBT, S, true>), grid, dim3(WT), 0, st, m->class_elems[cl], cnt, m->d,
                           f, a);
      return;
    }
  }
  if (condense)
    hipLaunchKernelGGL((adj_condense_kernel<NBT, S, false>), grid, dim3(WT), 0, st, m->class_elems[cl], cnt, m->d, f,
                       a);
  else
    hipLaunchKernelGGL((adj_recover_kernel<NBT, S, false>), grid, dim3(WT), 0, st, m->class_elems[cl], cnt, m->d, f,
                       a);
}

template <int NBT>
void launch_adj_s(bool condense, sbfwi_mesh_s* m, int cl, int S, const FactorsDev& f, const AdjArgs& a,
                  hipStream_t st) {
  switch (S) {
    case 1: launch_adj<NBT, 1>(condense, m, cl, f, a, st); break;
    case 2: launch_adj<NBT, 2>(condense, m, cl, f, a, st); break;
    case 4: launch_adj<NBT, 4>(condense, m, cl, f, a, st); break;
    case 8: launch_adj<NBT, 8>(condense, m, cl, f, a, st); break;
    default: launch_adj<NBT, 16>(condense, m, cl, f, a, st); break;
  }
}

void launch_adj_cls(bool condense, sbfwi_mesh_s* m, int cl, int S, const FactorsDev& f, const AdjArgs& a,
                    hipStream_t st) {
  if (cl == 0) launch_adj_s<8>(condense, m, cl, S, f, a, st);
  else if (cl == 1) launch_adj_s<16>(condense, m, cl, S, f, a, st);
  else launch_adj_s<24>(condense, m, cl, S, f, a, st);
}

template <int S>
void launch_adj_fused_s(bool condense, sbfwi_mesh_s* m, const FactorsDev& f, const AdjArgs& a, hipStream_t st) {
  const int groups = (a.NS + S - 1) / S;
  const int64_t n_work = m->n_elem * groups;
  auto kern = condense ? adj_sweep_fused_kernel<S, true> : adj_sweep_fused_kernel<S, false>;
  static std::atomic<int> per_cu[2] = {0, 0};   // occupancy, queried once per kernel
  int pc = per_cu[condense ? 0 : 1].load();
  if (pc == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, kern, WT, 0) != hipSuccess || pc <= 0) pc = 1;
    per_cu[condense ? 0 : 1].store(pc);
  }
  const int64_t cap = (int64_t)(pc > 0 ? pc : 1) * sbfwi_device_cus();
  const unsigned blocks = (unsigned)(n_work < cap ? n_work : cap);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(WT), 0, st, m->d.elem_by_cost, n_work, groups, m->d, f, a);
}

void launch_adj_fused(bool condense, int S, sbfwi_mesh_s* m, const FactorsDev& f, const AdjArgs& a,
                      hipStream_t st) {
  switch (S) {
    case 1: launch_adj_fused_s<1>(condense, m, f, a, st); break;
    case 2: launch_adj_fused_s<2>(condense, m, f, a, st); break;
    case 4: launch_adj_fused_s<4>(condense, m, f, a, st); break;
    case 8: launch_adj_fused_s<8>(condense, m, f, a, st); break;
    default: launch_adj_fused_s<16>(condense, m, f, a, st); break;
  }
}

// Transposed condense or recover over every element with the plan's shape choices.
void launch_adj_plan(bool condense, sbfwi_mesh_s* m, const FactorsDev& f, const SweepPlan& plan,
                     const AdjArgs& a, hipStream_t st) {
  const int kind = condense ? SW_ADJ_CONDENSE : SW_ADJ_RECOVER;
  if (plan.fusedS[kind] > 0) {
    launch_adj_fused(condense, plan.fusedS[kind], m, f, a, st);
    return;
  }
  const int def = sbfwi_default_shots_per_block(a.NS);
  for (int cl = 0; cl < 3; ++cl)
    launch_adj_cls(condense, m, cl, plan.S[kind][cl] > 0 ? plan.S[kind][cl] : def, f, a, st);
}

void launch_adj_sweep(bool condense, sbfwi_factors_s* fac, const AdjArgs& a, hipStream_t st) {
  ProfScope ps(condense ? PK_ADJ_CONDENSE : PK_ADJ_RECOVER, st);
  launch_adj_plan(condense, fac->m, fac->d, fac->plan, a, st);
}

// LDS bound of a joint transposed-sweep block; larger classes run the two sweeps in turn.
constexpr size_t kAdjJointLdsMax = 48 * 1024;

template <int NBT, int S>
bool launch_adj_joint_cls(sbfwi_mesh_s* m, int cl, const FactorsDev& f, const AdjArgs& a, hipStream_t st) {
  const int64_t cnt = (int64_t)m->h_class_elems[cl].size();
  if (cnt == 0) return true;
  const size_t dyn = (size_t)m->class_nmax[cl] * NBT * S * sizeof(double);
  if (sizeof(AdjLds<NBT, S>) + dyn > kAdjJointLdsMax) return false;
  dim3 grid((unsigned)sweep_blocks(cnt, (a.NS + S - 1) / S));
  if constexpr (3 * NBT <= WT) {
    if (sbfwi_fly_rows(f)) {
      hipLaunchKernelGGL((adj_joint_kernel<NBT, S, true>), grid, dim3(WT), dyn, st, m->class_elems[cl], cnt, m->d, f,
                         a);
      return true;
    }
  }
  hipLaunchKernelGGL((adj_joint_kernel<NBT, S, false>), grid, dim3(WT), dyn, st, m->class_elems[cl], cnt, m->d, f,
                     a);
  return true;
}

template <int NBT>
bool launch_adj_joint_s(sbfwi_mesh_s* m, int cl, int S, const FactorsDev& f, const AdjArgs& a, hipStream_t st) {
  switch (S) {
    case 1: return launch_adj_joint_cls<NBT, 1>(m, cl, f, a, st);
    case 2: return launch_adj_joint_cls<NBT, 2>(m, cl, f, a, st);
    case 4: return launch_adj_joint_cls<NBT, 4>(m, cl, f, a, st);
    case 8: return launch_adj_joint_cls<NBT, 8>(m, cl, f, a, st);
    default: return launch_adj_joint_cls<NBT, 16>(m, cl, f, a, st);
  }
}

// Transposed recover of step k and transposed condense of step k - 1: one joint
// launch per n_b class with the recover's shots per block, or the two sweeps in
// turn where the LDS would not fit or the plan runs a persistent launch.
void launch_adj_joint(sbfwi_factors_s* fac, const AdjArgs& a, hipStream_t st) {
  sbfwi_mesh_s* m = fac->m;
  const SweepPlan& plan = fac->plan;
  if (plan.fusedS[SW_ADJ_RECOVER] > 0 || plan.fusedS[SW_ADJ_CONDENSE] > 0) {
    launch_adj_sweep(false, fac, a, st);
    launch_adj_sweep(true, fac, a, st);
    return;
  }
  ProfScope ps(PK_ADJ_JOINT, st);
  const int def = sbfwi_default_shots_per_block(a.NS);
  for (int cl = 0; cl < 3; ++cl) {
    const int S = plan.S[SW_ADJ_RECOVER][cl] > 0 ? plan.S[SW_ADJ_RECOVER][cl] : def;
    const bool ok = cl == 0 ? launch_adj_joint_s<8>(m, cl, S, fac->d, a, st)
                            : cl == 1 ? launch_adj_joint_s<16>(m, cl, S, fac->d, a, st)
                                      : launch_adj_joint_s<24>(m, cl, S, fac->d, a, st);
    if (ok) continue;
    const int Sc = plan.S[SW_ADJ_CONDENSE][cl] > 0 ? plan.S[SW_ADJ_CONDENSE][cl] : def;
    launch_adj_cls(false, m, cl, S, fac->d, a, st);
    launch_adj_cls(true, m, cl, Sc, fac->d, a, st);
  }
}

// One block per element of a class: the shot groups of the element in turn, so
// each gradient entry has one writer and receives its additions in a fixed
// order (each group's memory-side adds complete before the next group's), and
// the groups' reads of the element's rows share the caches.
template <int NBT, int S, bool RG>
__global__ void __launch_bounds__(WT) grad_exact_kernel(const int32_t* __restrict__ elems, MeshDev m,
                                                        FactorsDev f, int NS, const double* __restrict__ X,
                                                        const double* __restrict__ lam,
                                                        const double* __restrict__ acc_a, double* __restrict__ grad,
                                                        int64_t shot_stride) {
  const int e = elems[blockIdx.x];
  extern __shared__ double rg_w[];   // Galerkin: the weights of the element's n intervals, [n][kRgW]
  if constexpr (RG) {
    const int n = m.nr[e] - 1;
    const double* W = f.rgw + f.rgw_off[n + 1];
    for (int q = threadIdx.x; q < n * kRgW; q += WT) rg_w[q] = W[q];
    __syncthreads();
  }
  for (int s0 = 0; s0 < NS; s0 += S) {
    if (s0 > 0) {
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
    if constexpr (RG)
      grad_rg_group<NBT, S>(e, m, f, NS, X, lam, acc_a, grad, s0, shot_stride, rg_w);
    else
      grad_exact_group<NBT, S>(e, m, f, NS, X, lam, acc_a, grad, s0, shot_stride);
  }
}

template <int NBT, int S>
void launch_grad_cls(sbfwi_mesh_s* m, int cl, const FactorsDev& f, int NS, const double* X, const double* lam,
                     const double* acc, double* grad, int64_t stride, hipStream_t st) {
  int64_t cnt = (int64_t)m->h_class_elems[cl].size();
  if (cnt == 0) return;
  if (f.scheme == SBFWI_SCHEME_RADIAL_GALERKIN)
    hipLaunchKernelGGL((grad_exact_kernel<NBT, S, true>), dim3((unsigned)cnt), dim3(WT),
                       (size_t)m->class_nmax[cl] * kRgW * sizeof(double), st, m->class_elems[cl], m->d, f, NS, X,
                       lam, acc, grad, stride);
  else
    hipLaunchKernelGGL((grad_exact_kernel<NBT, S, false>), dim3((unsigned)cnt), dim3(WT), 0, st, m->class_elems[cl],
                       m->d, f, NS, X, lam, acc, grad, stride);
}

template <int S>
void launch_grad_all(sbfwi_mesh_s* m, const FactorsDev& f, int NS, const double* X, const double* lam,
                     const double* acc, double* grad, int64_t stride, hipStream_t st) {
  // at most one item per lane: 8 shots per group for n_b <= 8, 4 for <= 16, 2 for <= 24
  launch_grad_cls<8, S>(m, 0, f, NS, X, lam, acc, grad, stride, st);
  launch_grad_cls<16, (S < 4 ? S : 4)>(m, 1, f, NS, X, lam, acc, grad, stride, st);
  launch_grad_cls<24, (S < 2 ? S : 2)>(m, 2, f, NS, X, lam, acc, grad, stride, st);
}

// stride 0: gradient summed over shots; stride n_params: one gradient per shot
void launch_grad(sbfwi_mesh_s* m, const FactorsDev& f, int NS, const double* X, const double* lam,
                 const double* acc, double* grad, int64_t stride, hipStream_t st) {
  ProfScope ps(PK_GRAD_EXACT, st);
  if (NS <= 1) launch_grad_all<1>(m, f, NS, X, lam, acc, grad, stride, st);
  else if (NS <= 2) launch_grad_all<2>(m, f, NS, X, lam, acc, grad, stride, st);
  else if (NS <= 4) launch_grad_all<4>(m, f, NS, X, lam, acc, grad, stride, st);
  else launch_grad_all<8>(m, f, NS, X, lam, acc, grad, stride, st);
}

struct AdjWork {
  double *seeds = nullptr, *z = nullptr, *gB = nullptr, *pl = nullptr, *rhs = nullptr, *lamB = nullptr,
         *lam = nullptr;
  double* bvf = nullptr;   // paper kernel: velocity of the back-propagated field at every level
  int32_t* par_elem = nullptr;
  CoarseWork cw;
};

void adj_free(AdjWork* w) {
  sbfwi_dev_free(w->seeds);
  sbfwi_dev_free(w->z);
  sbfwi_dev_free(w->gB);
  sbfwi_dev_free(w->pl);
  sbfwi_dev_free(w->rhs);
  sbfwi_dev_free(w->lamB);
  sbfwi_dev_free(w->lam);
  sbfwi_dev_free(w->bvf);
  sbfwi_dev_free(w->par_elem);
  sbfwi_coarse_work_free(&w->cw);
}

}  // namespace

int sbfwi_misfit_residual(const double* traces, const double* observed, int64_t count, double dt,
                          double* residual, double* misfit, hipStream_t s) {
  hipLaunchKernelGGL(misfit_kernel, dim3(1), dim3(1024), 0, s, traces, observed, count, dt, residual, misfit);
  SBFWI_HIP(hipGetLastError());
  return SBFWI_OK;
}

extern "C" int sbfwi_misfit(const double* observed, const double* traces, int64_t count, double dt,
                            double* residual, double* misfit, hipStream_t s) {
  if (!misfit || (count > 0 && (!observed || !traces))) return sbfwi_fail(SBFWI_EINVAL, "NULL argument");
  if (count < 0 || !(dt > 0)) return sbfwi_fail(SBFWI_EINVAL, "count must be >= 0 and dt positive");
  return sbfwi_misfit_residual(traces, observed, count, dt, residual, misfit, s);
}

// The backward pass.  Checkpoint segments are recomputed (forward steps that
// store the unknowns with ghosts and the level field of every step) and then
// stepped back by the adjoint.  With a recompute stream sr, the recompute of
// segment s - 1 runs on sr into the other of two segment stores while the
// adjoint steps of segment s run on st (events ev[0..1]: segment in store b
// recomputed; ev[2..3]: the adjoint and its gradient contractions are done
// with store b).  With a gradient stream sg (exact mode), the contraction of
// step k runs on sg while the adjoint computes step k - 1; the adjoint rows
// alternate between two buffers lam[0..1] (events ev[5..6]: rows of buffer q
// written; ev[7..8]: the contraction is done reading them).
static int adjoint_run(sbfwi_factors_s* f, sbfwi_ckpt_s* ck, const double* adj_src, int mode, double* grad,
                       hipStream_t st, AdjWork& w, StepWork& fw, StepWork& bw, double* const xseg[2],
                       double* const fseg[2], hipStream_t sr, hipStream_t sg, const hipEvent_t* ev) {
  sbfwi_mesh_s* m = f->m;
  const int NS = ck->n_shots;
  const int64_t N = ck->n_steps, C = ck->interval;
  const int64_t nn = m->n_nodes * NS;
  // element of every fine-grid parameter
  {
    std::vector<int32_t> pe(m->n_params);
    for (int64_t e = 0; e < m->n_elem; ++e)
      for (int64_t p = m->h_par_off[e]; p < m->h_par_off[e + 1]; ++p) pe[p] = (int32_t)e;
    SBFWI_CHECK(sbfwi_upload(&w.par_elem, pe));
  }
  const int per_shot = (mode & SBFWI_GRAD_PER_SHOT) ? 1 : 0;
  mode &= ~SBFWI_GRAD_PER_SHOT;
  SBFWI_HIP(hipMemsetAsync(grad, 0, sizeof(double) * m->n_params * (per_shot ? NS : 1), st));
  SourceTable fsrc;
  fsrc.n_src = 1;
  fsrc.node = ck->src_node;
  fsrc.node_stride = 1;
  fsrc.amp = ck->wavelet;
  fsrc.amp_steps = N;
  AdjArgs a;
  a.NS = NS;
  if (mode == SBFWI_GRAD_EXACT) {
    int64_t ni = m->n_int * NS;
    SBFWI_CHECK(sbfwi_alloc(&w.seeds, 3 * ni + 3 * nn));
    SBFWI_HIP(hipMemsetAsync(w.seeds, 0, sizeof(double) * (3 * ni + 3 * nn), st));
    a.ut = w.seeds; a.vb = a.ut + ni; a.ab = a.vb + ni;
    a.UB = a.ab + ni; a.VB = a.UB + nn; a.AB = a.VB + nn;
    SBFWI_CHECK(sbfwi_alloc(&w.z, ni));
    SBFWI_CHECK(sbfwi_alloc(&w.gB, m->n_loop * NS));
    SBFWI_CHECK(sbfwi_alloc(&w.pl, m->n_loop * NS));
    SBFWI_CHECK(sbfwi_alloc(&w.rhs, nn));
    SBFWI_CHECK(sbfwi_alloc(&w.lamB, nn));
    SBFWI_CHECK(sbfwi_alloc(&w.lam, (sg ? 2 : 1) * m->n_x * NS));
    SBFWI_HIP(hipMemsetAsync(w.lamB, 0, sizeof(double) * nn, st));
    SBFWI_CHECK(sbfwi_coarse_work_alloc(&w.cw, m, NS));
    a.z = w.z; a.gB = w.gB; a.pl = w.pl; a.lamB = w.lamB; a.lam = w.lam;
  } else {
    SBFWI_CHECK(sbfwi_step_work_alloc(&bw, m, NS));
    SBFWI_CHECK(sbfwi_step_zero(m, &bw, st));
    SBFWI_CHECK(sbfwi_alloc(&w.bvf, m->n_params * NS));
  }
  SourceTable bsrc;  // paper kernel: receivers as sources, time-reversed
  bsrc.n_src = ck->n_rec;
  bsrc.node = ck->rec_node;
  bsrc.node_stride = 0;
  bsrc.amp = adj_src;
  bsrc.amp_steps = N;
  bsrc.reversed = 1;
  const int kind = mode == SBFWI_GRAD_EXACT ? 0 : 1;
  const int64_t nseg = (N + C - 1) / C;
  const unsigned gp = (unsigned)((m->n_params + 255) / 256);
  const unsigned gn = (unsigned)((nn + 255) / 256);
  // recompute of segment seg into store b: its start (state copy) and its step k
  auto recompute_begin = [&](int64_t seg, hipStream_t s) -> int {
    return sbfwi_state_copy(m, &fw, ck->states + seg * sbfwi_state_size(m, NS), 0, s);
  };
  auto recompute_step = [&](int64_t seg, int b, int64_t k, hipStream_t s) -> int {
    const int64_t k0 = seg * C;
    double* xs = xseg[b] + (k - k0 - 1) * m->n_x * NS;
    double* fs = fseg[b] + (k - k0 - 1) * m->n_params * NS;
    const double* us = ck->ustore ? ck->ustore + (k - 1) * m->n_nodes * NS : nullptr;
    return sbfwi_forward_step(f, &fw, k, fsrc, 0, nullptr, nullptr, N, xs, fs, kind, s, nullptr, us,
                              k < std::min(k0 + C, N));
  };
  auto recompute = [&](int64_t seg, int b, hipStream_t s) -> int {
    const int64_t k0 = seg * C, k1 = std::min(k0 + C, N);
    SBFWI_CHECK(recompute_begin(seg, s));
    for (int64_t k = k0 + 1; k <= k1; ++k) SBFWI_CHECK(recompute_step(seg, b, k, s));
    return SBFWI_OK;
  };
  const bool ov = sr != nullptr && !ck->full_store;
  const bool gs = sg != nullptr && mode == SBFWI_GRAD_EXACT;
  // segments tseg0 .. nseg - 1 come from the tail store of the forward run (exact mode):
  // no recompute
  const int64_t tseg0 = (ck->tail_x && kind == 0) ? ck->tail_k0 / C : nseg;
  bool adj_condensed = false;   // the transposed condense of the next adjoint step is done
  bool nodal_due = false;       // the last step's nodal chain is still to run
  int64_t n_grad = 0;   // contractions launched on sg
  if (ov || gs) {   // the side streams start after everything enqueued on st so far
    SBFWI_HIP(hipEventRecord(ev[4], st));
    if (ov) SBFWI_HIP(hipStreamWaitEvent(sr, ev[4], 0));
    if (gs) SBFWI_HIP(hipStreamWaitEvent(sg, ev[4], 0));
  }
  if (ov && nseg - 1 < tseg0) {
    SBFWI_CHECK(recompute(nseg - 1, (int)((nseg - 1) % 2), sr));
    SBFWI_HIP(hipEventRecord(ev[(nseg - 1) % 2], sr));
  }
  for (int64_t seg = nseg - 1; seg >= 0; --seg) {
    const int64_t k0 = seg * C, k1 = std::min(k0 + C, N);
    const int b = ov ? (int)(seg % 2) : 0;
    const bool tail = seg >= tseg0;
    // recompute of segment seg - 1 (into the other store), paced by this segment's
    // adjoint steps: its step j waits until the adjoint's step j has been reached,
    // so that every adjoint step (and its latency-bound coarse solve) runs beside
    // one recompute step instead of the recompute running ahead and the adjoint
    // then running alone
    const int nb = (int)((seg + 1) % 2);
    int64_t kr = 0, kr1 = 0;   // next and last step of the paced recompute
    if (ov) {
      if (seg >= 1 && seg - 1 < tseg0) {   // once the adjoint of seg + 1 is done with that store
        if (seg + 1 <= nseg - 1) SBFWI_HIP(hipStreamWaitEvent(sr, ev[2 + nb], 0));
        SBFWI_CHECK(recompute_begin(seg - 1, sr));
        kr = (seg - 1) * C + 1;
        kr1 = seg * C;
      }
      if (!tail) SBFWI_HIP(hipStreamWaitEvent(st, ev[b], 0));
    } else if (!ck->full_store && !tail) {
      SBFWI_CHECK(recompute(seg, 0, st));
    }
    for (int64_t k = k1; k > k0; --k) {
      if (kr && kr <= kr1) {
        SBFWI_HIP(hipEventRecord(ev[9], st));
        SBFWI_HIP(hipStreamWaitEvent(sr, ev[9], 0));
        SBFWI_CHECK(recompute_step(seg - 1, nb, kr, sr));
        ++kr;
      }
      const double* X = ck->full_store ? ck->xstore + (k - 1) * m->n_x * NS
                        : tail        ? ck->tail_x + (k - ck->tail_k0 - 1) * m->n_x * NS
                                      : xseg[b] + (k - k0 - 1) * m->n_x * NS;
      const double* Fs = ck->full_store ? (kind == 0 ? ck->fstore : ck->vstore) + (k - 1) * m->n_params * NS
                         : tail         ? ck->tail_f + (k - ck->tail_k0 - 1) * m->n_params * NS
                                        : fseg[b] + (k - k0 - 1) * m->n_params * NS;
      if (mode == SBFWI_GRAD_EXACT) {
        const int q = (int)(k % 2);
        if (gs) {   // rows buffer q: the contraction of step k + 2 must be done reading it
          if (n_grad >= 2) SBFWI_HIP(hipStreamWaitEvent(st, ev[7 + q], 0));
          a.lam = w.lam + (int64_t)q * m->n_x * NS;
        }
        if (!adj_condensed) launch_adj_sweep(true, f, a, st);
        {
          ProfScope ps(PK_ADJ_RHS, st);
          if (nodal_due)   // step k + 1's nodal chain, deferred to here
            hipLaunchKernelGGL(adj_nodal_rhs_kernel, dim3(gn), dim3(256), 0, st, m->d, NS, f->d, a, w.rhs,
                               ck->n_rec, ck->rec_node, adj_src, N, k);
          else
            hipLaunchKernelGGL(adj_rhs_kernel, dim3(gn), dim3(256), 0, st, m->d, NS, f->d, a, w.rhs, ck->n_rec,
                               ck->rec_node, adj_src, N, k);
          nodal_due = false;
        }
        SBFWI_HIP(hipGetLastError());
        SBFWI_CHECK(sbfwi_coarse_solve(f, &w.cw, 1, w.rhs, w.lamB, k, st));
        // the transposed recover of step k, joined with the transposed condense of step k - 1
        if (k > 1 && f->joint_sweeps) {
          launch_adj_joint(f, a, st);
          adj_condensed = true;
        } else {
          launch_adj_sweep(false, f, a, st);
          adj_condensed = false;
        }
        // the nodal chain of step k: joined with the right-hand side of step k - 1 when
        // that step's transposed condense is already done (the joint sweep)
        if (adj_condensed) {
          nodal_due = true;
        } else {
          ProfScope ps(PK_ADJ_NODAL, st);
          hipLaunchKernelGGL(adj_nodal_kernel, dim3(gn), dim3(256), 0, st, m->d, NS, f->d, a);
        }
        if (gs) {
          SBFWI_HIP(hipEventRecord(ev[5 + q], st));
          SBFWI_HIP(hipStreamWaitEvent(sg, ev[5 + q], 0));
          launch_grad(m, f->d, NS, X, (const double*)a.lam, Fs, grad, per_shot ? m->n_params : 0, sg);
          SBFWI_HIP(hipEventRecord(ev[7 + q], sg));
          ++n_grad;
        } else {
          launch_grad(m, f->d, NS, X, (const double*)w.lam, Fs, grad, per_shot ? m->n_params : 0, st);
        }
        SBFWI_HIP(hipGetLastError());
      } else {
        const int64_t kp = N + 1 - k;  // back-propagation step paired with forward step k
        // its velocity at every level into w.bvf (a level field)
        SBFWI_CHECK(sbfwi_forward_step(f, &bw, kp, bsrc, 0, nullptr, nullptr, N, nullptr, w.bvf, 1, st, nullptr,
                                       nullptr, kp < N));
        ProfScope ps(PK_GRAD_PAPER, st);
        hipLaunchKernelGGL(grad_paper_kernel, dim3(gp), dim3(256), 0, st, NS, 1.0, m->n_params,
                           (const double*)w.bvf, Fs, grad, per_shot);
        SBFWI_HIP(hipGetLastError());
      }
    }
    if (kr) {   // the rest of the paced recompute (a last segment shorter than the others)
      for (; kr <= kr1; ++kr) SBFWI_CHECK(recompute_step(seg - 1, nb, kr, sr));
      SBFWI_HIP(hipEventRecord(ev[nb], sr));
    }
    // the segment's contractions read its store too: st waits for the last one
    if (gs && n_grad > 0) SBFWI_HIP(hipStreamWaitEvent(st, ev[7 + (int)((k0 + 1) % 2)], 0));
    if (ov) SBFWI_HIP(hipEventRecord(ev[2 + b], st));
  }
  if (nodal_due) {   // (step 1 never defers its chain; kept for safety)
    ProfScope ps(PK_ADJ_NODAL, st);
    hipLaunchKernelGGL(adj_nodal_kernel, dim3(gn), dim3(256), 0, st, m->d, NS, f->d, a);
    SBFWI_HIP(hipGetLastError());
  }
  return SBFWI_OK;
}

int sbfwi_adjoint_impl(sbfwi_factors_s* f, sbfwi_ckpt_s* ck, const double* adj_src, int mode, double* grad,
                       hipStream_t st) {
  sbfwi_mesh_s* m = f->m;
  const int NS = ck->n_shots;
  AdjWork w;
  StepWork fw, bw;
  double* xseg[2] = {nullptr, nullptr};
  double* fseg[2] = {nullptr, nullptr};
  hipStream_t sr = nullptr, sg = nullptr;   // recompute and contraction streams
  hipEvent_t ev[10] = {};
  int rc = SBFWI_OK;
  if (!ck->full_store) {
    rc = sbfwi_step_work_alloc(&fw, m, NS);
    if (rc == SBFWI_OK) rc = sbfwi_alloc(&xseg[0], ck->interval * m->n_x * NS);
    if (rc == SBFWI_OK) rc = sbfwi_alloc(&fseg[0], ck->interval * m->n_params * NS);
    // overlap of recompute and adjoint (direct coarse solver only: no cooperative launches);
    // skipped if the second segment store does not fit
    if (rc == SBFWI_OK && f->overlap_adjoint && f->dnum && ck->interval < ck->n_steps) {
      if (sbfwi_alloc(&xseg[1], ck->interval * m->n_x * NS) == SBFWI_OK &&
          sbfwi_alloc(&fseg[1], ck->interval * m->n_params * NS) == SBFWI_OK) {
        bool ok = hipStreamCreateWithFlags(&sr, hipStreamNonBlocking) == hipSuccess &&
                  hipStreamCreateWithFlags(&sg, hipStreamNonBlocking) == hipSuccess;
        for (int q = 0; q < 10 && ok; ++q) ok = hipEventCreateWithFlags(&ev[q], hipEventDisableTiming) == hipSuccess;
        if (!ok) rc = sbfwi_fail(SBFWI_EHIP, "adjoint: cannot create the side streams");
      } else {
        (void)hipGetLastError();   // the second store did not fit: one segment after the other
      }
    }
  }
  if (rc == SBFWI_OK) {
    int flags0[4] = {0, -1, 0, 0};
    hipError_t he = hipMemcpyAsync(f->d.status, flags0, 2 * sizeof(int), hipMemcpyHostToDevice, st);
    if (he != hipSuccess) rc = sbfwi_fail(SBFWI_EHIP, "status reset: %s", hipGetErrorString(he));
  }
  if (rc == SBFWI_OK) rc = adjoint_run(f, ck, adj_src, mode, grad, st, w, fw, bw, xseg, fseg, sr, sg, ev);
  int flags[4] = {0, -1, 0, 0};
  if (rc == SBFWI_OK) {
    hipError_t he = hipMemcpyAsync(flags, f->d.status, sizeof(flags), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) rc = sbfwi_fail(SBFWI_EHIP, "adjoint: %s", hipGetErrorString(he));
  } else {
    (void)hipStreamSynchronize(st);
  }
  if (sr) (void)hipStreamSynchronize(sr);
  if (sg) (void)hipStreamSynchronize(sg);
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  if (sr) (void)hipStreamDestroy(sr);
  if (sg) (void)hipStreamDestroy(sg);
  adj_free(&w);
  if (!ck->full_store) sbfwi_step_work_free(&fw);
  if (bw.r) sbfwi_step_work_free(&bw);
  for (int b = 0; b < 2; ++b) {
    sbfwi_dev_free(xseg[b]);
    sbfwi_dev_free(fseg[b]);
  }
  if (rc != SBFWI_OK) return rc;
  if (flags[0] & 8) return sbfwi_fail(SBFWI_EHIP, "adjoint: coarse-solve grid barrier timed out");
  if (flags[0] & 4) return sbfwi_fail(SBFWI_ENONFINITE, "non-finite coarse residual at step %d", flags[1]);
  if (flags[0] & 2) return sbfwi_fail(SBFWI_ENOCONV, "coarse solve did not converge at step %d", flags[1]);
  return SBFWI_OK;
}

namespace {

template <typename Fn>
int time_launch(Fn&& fn, int reps, hipStream_t st, hipEvent_t e0, hipEvent_t e1, float* ms) {
  fn();
  SBFWI_HIP(hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r) fn();
  SBFWI_HIP(hipEventRecord(e1, st));
  SBFWI_HIP(hipEventSynchronize(e1));
  SBFWI_HIP(hipGetLastError());
  float t = 0.f;
  SBFWI_HIP(hipEventElapsedTime(&t, e0, e1));
  *ms = t / reps;
  return SBFWI_OK;
}

int tune_adj(sbfwi_factors_s* f, const AdjArgs& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1, double* out) {
  sbfwi_mesh_s* m = f->m;
  const int cands[5] = {1, 2, 4, 8, 16};
  int smax = 1;
  while (smax < a.NS) smax *= 2;
  for (int kind = SW_ADJ_CONDENSE; kind <= SW_ADJ_RECOVER; ++kind) {
    const bool cond = kind == SW_ADJ_CONDENSE;
    double sum_best = 0.0;
    for (int cl = 0; cl < 3; ++cl) {
      f->plan.S[kind][cl] = 0;
      if (m->h_class_elems[cl].empty()) continue;
      float best = 1e30f;
      int bs = 0;
      for (int S : cands) {
        if (S > smax) break;
        float t = 0.f;
        SBFWI_CHECK(time_launch([&] { launch_adj_cls(cond, m, cl, S, f->d, a, st); }, 3, st, e0, e1, &t));
        if (t < best) { best = t; bs = S; }
      }
      f->plan.S[kind][cl] = bs;
      sum_best += best;
    }
    float bestf = 1e30f;
    int bfs = 0;
    for (int S : cands) {
      if (S > smax) break;
      float t = 0.f;
      SBFWI_CHECK(time_launch([&] { launch_adj_fused(cond, S, m, f->d, a, st); }, 3, st, e0, e1, &t));
      if (t < bestf) { bestf = t; bfs = S; }
    }
    f->plan.fusedS[kind] = bestf < 0.97 * sum_best ? bfs : 0;
    if (out) {
      double* o = out + 6 * kind;
      for (int cl = 0; cl < 3; ++cl) o[cl] = f->plan.S[kind][cl];
      o[3] = f->plan.fusedS[kind];
      o[4] = sum_best;
      o[5] = bestf;
    }
  }
  return SBFWI_OK;
}

}  // namespace

int sbfwi_tune_adj_sweeps(sbfwi_factors_s* f, int NS, hipStream_t st, double* out) {
  sbfwi_mesh_s* m = f->m;
  AdjWork w;
  AdjArgs a;
  a.NS = NS;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int64_t ni = m->n_int * NS, nn = m->n_nodes * NS;
  int rc = sbfwi_alloc(&w.seeds, 3 * ni + 3 * nn);
  if (rc == SBFWI_OK) rc = sbfwi_alloc(&w.z, ni);
  if (rc == SBFWI_OK) rc = sbfwi_alloc(&w.gB, m->n_loop * NS);
  if (rc == SBFWI_OK) rc = sbfwi_alloc(&w.pl, m->n_loop * NS);
  if (rc == SBFWI_OK) rc = sbfwi_alloc(&w.lamB, nn);
  if (rc == SBFWI_OK) rc = sbfwi_alloc(&w.lam, m->n_x * NS);
  if (rc == SBFWI_OK) {
    a.ut = w.seeds; a.vb = a.ut + ni; a.ab = a.vb + ni;
    a.UB = a.ab + ni; a.VB = a.UB + nn; a.AB = a.VB + nn;
    a.z = w.z; a.gB = w.gB; a.pl = w.pl; a.lamB = w.lamB; a.lam = w.lam;
    // zero inputs: the timings do not depend on the values
    bool ok = hipMemsetAsync(w.seeds, 0, sizeof(double) * (3 * ni + 3 * nn), st) == hipSuccess;
    ok = ok && hipMemsetAsync(w.z, 0, sizeof(double) * ni, st) == hipSuccess;
    ok = ok && hipMemsetAsync(w.gB, 0, sizeof(double) * m->n_loop * NS, st) == hipSuccess;
    ok = ok && hipMemsetAsync(w.pl, 0, sizeof(double) * m->n_loop * NS, st) == hipSuccess;
    ok = ok && hipMemsetAsync(w.lamB, 0, sizeof(double) * nn, st) == hipSuccess;
    ok = ok && hipMemsetAsync(w.lam, 0, sizeof(double) * m->n_x * NS, st) == hipSuccess;
    if (!ok) rc = sbfwi_fail(SBFWI_EHIP, "memset failed");
  }
  if (rc == SBFWI_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = sbfwi_fail(SBFWI_EHIP, "event creation failed");
  if (rc == SBFWI_OK) rc = tune_adj(f, a, st, e0, e1, out);
  (void)hipStreamSynchronize(st);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  adj_free(&w);
  return rc;
}

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
//
// Interior state.  A step uses the old interior u, v, a only through two linear
// combinations: w = a0 u + a1 v + a2 a (the condense's source, and a^{k+1} =
// a0 u^{k+1} - w) and r = c1 u - c2 v - c3 a (v^{k+1} = c1 u^{k+1} - r).  The
// new pair follows from u^{k+1}, v^{k+1}, a^{k+1} by the same two combinations,
// so every interior level keeps (r, w) only: two words per node and shot
// instead of three, read and written once per step (the condense reads w
// alone).  u, v and a of a level are formed where a store needs them.  The
// boundary level keeps the nodal u, v, a, and the nodal update also writes the
// boundary level's w for the next condense.
#include <atomic>
#include <functional>

#include "sbfwi_internal.h"

// Multiply-adds fuse within an expression only: every launch shape (items per
// lane, shots per block) then rounds each (element, shot) the same way.
#pragma clang fp contract(on)

namespace {

__device__ __forceinline__ int md(int i, int nb) { return i < 0 ? i + nb : (i >= nb ? i - nb : i); }

struct StepArgs {
  int NS;                 // shots in the run (stride of the shot index)
  double *r, *w;          // interior state (r, w) of every level
  double *U, *V, *A;      // nodal state
  double* W;              // nodal w = a0 U + a1 V + a2 A
  double *q, *yn, *fhat, *Unew;
  double *xs, *fs;        // optional stores (unknowns with ghosts, level field)
  int field_kind;         // fs: 0 = a^k, 1 = v^k
  double* vs;             // optional second level-field store (v^k) when fs holds a^k
};

// Row stride of the dense blocks in LDS: one word of padding per row, so
// that the lanes of a wave, which read one row each in dense_mv, fall on
// different banks (an unpadded stride of NBT words puts every row on the same
// banks).
__host__ __device__ constexpr int fstride(int nbt) { return nbt + 1; }

template <int NBT, int S>
struct StepLds {
  double F[2][NBT * fstride(NBT)];
  double w[NBT * S];
  double y[NBT * S];
  double x[NBT * S];
  double t[NBT * S];
  double u1[NBT * S];
};

constexpr int WT = 64;

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
    if (q < nb * nb) dst[(q / nb) * fstride(NBT) + (q % nb)] = reg[r];
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
  for (int c = 0; c < nb; ++c) acc += F[i * fstride(NBT) + c] * vec[c * S + s];
  return acc;
}

// Target of the stores of lanes without an item, so that every lane stores
// unconditionally and the waits for the prefetched level count exactly.
__device__ double g_sink[WT];

// Newmark combination w = a0 u + a1 v + a2 a (eq. ODE_Newmark), written with
// explicit multiply-adds so that every sweep that forms it rounds it alike.
__device__ __forceinline__ double newmark_w(const FactorsDev& f, double u, double v, double a) {
  return fma(f.a2, a, fma(f.a1, v, f.a0 * u));
}

// r = c1 u - c2 v - c3 a, so that v^{k+1} = c1 u^{k+1} - r^k (eq. Newmark).
__device__ __forceinline__ double newmark_r(const FactorsDev& f, double u, double v, double a) {
  return fma(-f.c3, a, fma(-f.c2, v, f.c1 * u));
}

// JOINT: the interior levels' w comes from wkeep (LDS, level-major, written by
// the recover sweep of the previous step in the same block) instead of the
// state in HBM; the boundary level always takes the nodal state.
template <int NBT, int S, bool JOINT = false>
__device__ __forceinline__ void condense_body(int e, int s0, const MeshDev& m, const FactorsDev& f,
                                              const StepArgs& a, StepLds<NBT, S>& L,
                                              const double* wkeep = nullptr) {
  // Levels j = 0 .. n-1 stream: the next level's F block, w (on the boundary
  // level the nodal W) and bands P, theta are loaded at the top of
  // each level and consumed at its end; lanes without an item load word 0 of
  // their arrays and store to g_sink.
  constexpr int IPT = (NBT * S + WT - 1) / WT;
  const int ns = min(S, a.NS - s0);
  const int nb = m.nb[e], n = m.nr[e] - 1, nbnb = nb * nb;
  const int64_t io = m.int_off[e], lo = m.loop_off[e], po = m.par_off[e];
  const double* Fe = f.finv + m.finv_off[e];
  const int items = nb * S;
  int ii[IPT], si[IPT];
  bool own[IPT], ok[IPT];
  int64_t lnode[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int it = threadIdx.x + u * WT;
    own[u] = it < items;
    ii[u] = own[u] ? it / S : 0;
    si[u] = it % S;
    ok[u] = own[u] && si[u] < ns;
    lnode[u] = m.loop_nodes[lo + ii[u]];
  }
  double reg[(NBT * NBT + WT - 1) / WT];
  // n_b <= 21: a level's three band rows of P (and of theta) fit the 64 lanes,
  // one load each, and every item takes its entries by cross-lane shuffles
  constexpr bool kBandShfl = 3 * NBT <= WT;
  double cw[IPT], cp[3][IPT], ct[3][IPT];
  auto load_level = [&](int j, double (&ww)[IPT], double (&pb)[3][IPT], double (&tb)[3][IPT]) {
    const bool nodal = j == n;
    const double* sw = nodal ? a.W : a.w;
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int64_t row = nodal ? lnode[u] : io + (int64_t)j * nb + ii[u];
      const int64_t g = ok[u] ? row * a.NS + s0 + si[u] : 0;
      if (JOINT && !nodal)   // interior w from wkeep: no state loads
        ww[u] = 0.0;
      else
        ww[u] = sw[g];
      if constexpr (!kBandShfl) {
        const double* pp = f.pm_band + 3 * (po + (int64_t)j * nb) + ii[u];   // node 0 for lanes without an item
        const double* tp = f.th_band + 3 * (po + (int64_t)j * nb) + ii[u];
        pb[0][u] = pp[0];
        pb[1][u] = pp[nb];
        pb[2][u] = pp[2 * nb];
        tb[0][u] = tp[0];
        tb[1][u] = tp[nb];
        tb[2][u] = tp[2 * nb];
      }
    }
    if constexpr (kBandShfl) {   // word l of the level's three band rows in lane l (lanes past them: word 0)
      const int l = (int)threadIdx.x < 3 * nb ? (int)threadIdx.x : 0;
      pb[0][0] = f.pm_band[3 * (po + (int64_t)j * nb) + l];
      tb[0][0] = f.th_band[3 * (po + (int64_t)j * nb) + l];
    }
  };
  // y_j = P_j w_j - theta_j q_{j-1} into L.y (L.x holds q_{j-1})
  auto level_rhs = [&](int j) {
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int it = threadIdx.x + u * WT;
      if (own[u])
        L.w[it] = JOINT && j < n ? wkeep[j * items + it] : (ok[u] ? cw[u] : 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int it = threadIdx.x + u * WT, i = ii[u], s = si[u];
      const int im = md(i - 1, nb) * S + s, ic = i * S + s, ip = md(i + 1, nb) * S + s;
      double p0, p1, p2, t0, t1, t2;
      if constexpr (kBandShfl) {   // band row entries of node i from the lanes that loaded them
        p0 = __shfl(cp[0][0], i, WT);
        p1 = __shfl(cp[0][0], nb + i, WT);
        p2 = __shfl(cp[0][0], 2 * nb + i, WT);
        t0 = __shfl(ct[0][0], i, WT);
        t1 = __shfl(ct[0][0], nb + i, WT);
        t2 = __shfl(ct[0][0], 2 * nb + i, WT);
      } else {
        p0 = cp[0][u]; p1 = cp[1][u]; p2 = cp[2][u];
        t0 = ct[0][u]; t1 = ct[1][u]; t2 = ct[2][u];
      }
      double y = p0 * L.w[im] + p1 * L.w[ic] + p2 * L.w[ip];
      if (j > 0) y -= t0 * L.x[im] + t1 * L.x[ic] + t2 * L.x[ip];
      if (own[u]) L.y[it] = y;
    }
    __syncthreads();
  };
  prefetch<NBT>(reg, Fe, nbnb);
  commit<NBT>(reg, L.F[0], nb);
  load_level(0, cw, cp, ct);
  int cur = 0;
  __syncthreads();
  __builtin_amdgcn_s_waitcnt(0);   // nothing in flight at the loop entry
  for (int j = 0; j < n; ++j) {
    const int jf = j + 1 < n ? j + 1 : n - 1;   // the last interior level reloads its own block (unused)
    prefetch<NBT>(reg, Fe + (int64_t)jf * nbnb, nbnb);
    double nw[IPT], np[3][IPT], nt[3][IPT];
    load_level(j + 1, nw, np, nt);
    level_rhs(j);
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int it = threadIdx.x + u * WT, i = ii[u], s = si[u];
      const double qv = dense_mv<NBT>(L.F[cur], L.y, nb, i, s, S);
      if (own[u]) L.t[it] = qv;
      const int64_t g = (io + (int64_t)j * nb + i) * a.NS + s0 + s;
      *(ok[u] ? a.q + g : g_sink + threadIdx.x) = qv;
    }
    commit<NBT>(reg, L.F[cur ^ 1], nb);
    __syncthreads();
    for (int it = threadIdx.x; it < items; it += WT) L.x[it] = L.t[it];  // q_j
    __syncthreads();
    cur ^= 1;
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      cw[u] = nw[u];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        cp[k][u] = np[k][u];
        ct[k][u] = nt[k][u];
      }
    }
  }
  level_rhs(n);   // boundary level: y_n
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

// Level loop of the recovery sweep (j = n-1 .. 0).  The next level's F block,
// state (q, r, w) and psi~ band are loaded at the top of each level and
// consumed at its end, so the sweep streams without waiting on the level
// recursion; the loads of lanes without an item read word 0 and the stores
// of such lanes go to g_sink.
// wkeep (LDS, may be NULL): receives the new w of every interior level,
// wkeep[j * items + it], for the condense of the next step in the same block.
template <int NBT, int S, bool STORE>
__device__ __forceinline__ void recover_levels(int e, int s0, const MeshDev& m, const FactorsDev& f,
                                               const StepArgs& a, StepLds<NBT, S>& L, double* wkeep) {
  constexpr int IPT = (NBT * S + WT - 1) / WT;
  const int ns = min(S, a.NS - s0);
  const int nb = m.nb[e], n = m.nr[e] - 1, nbnb = nb * nb;
  const int64_t io = m.int_off[e], po = m.par_off[e], xo = m.x_off[e];
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
  double cq[IPT], cr[IPT], cw[IPT], cb[3][IPT];
  auto load_level = [&](int j, double (&q)[IPT], double (&rr)[IPT], double (&ww)[IPT], double (&bd)[3][IPT]) {
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int64_t g = ok[u] ? (io + (int64_t)j * nb + ii[u]) * a.NS + s0 + si[u] : 0;
      q[u] = a.q[g];
      rr[u] = a.r[g];
      ww[u] = a.w[g];
      const double* bp = f.ps_band + 3 * (po + (int64_t)j * nb) + ii[u];   // node 0 for lanes without an item
      bd[0][u] = bp[0];
      bd[1][u] = bp[nb];
      bd[2][u] = bp[2 * nb];
    }
  };
  load_level(n - 1, cq, cr, cw, cb);
  int cur = 0;
  __syncthreads();
  // nothing in flight at the loop entry: the compiler then counts the waits
  // inside the loop from the loop's own loads and stores alone
  __builtin_amdgcn_s_waitcnt(0);
  for (int j = n - 1; j >= 0; --j) {
    const int jn = j > 0 ? j - 1 : 0;   // the last level reloads level 0 (unused)
    prefetch<NBT>(reg, Fe + (int64_t)jn * nbnb, nbnb);
    double nq[IPT], nr[IPT], nw[IPT], nbd[3][IPT];
    load_level(jn, nq, nr, nw, nbd);
    // t = psi~_j u_{j+1}
    if (j > 0) {
#pragma unroll
      for (int u = 0; u < IPT; ++u) {
        const int it = threadIdx.x + u * WT, i = ii[u], s = si[u];
        if (own[u])
          L.t[it] = cb[0][u] * L.x[md(i - 1, nb) * S + s] + cb[1][u] * L.x[i * S + s] +
                    cb[2][u] * L.x[md(i + 1, nb) * S + s];
      }
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
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int it = threadIdx.x + u * WT, i = ii[u], s = si[u];
      const int64_t g = (io + (int64_t)j * nb + i) * a.NS + s0 + s;
      const double uj = ok[u] ? cq[u] - dense_mv<NBT>(L.F[cur], L.t, nb, i, s, S) : 0.0;
      const double vn = f.c1 * uj - cr[u];
      const double an = f.a0 * uj - cw[u];
      const double wn = newmark_w(f, uj, vn, an);
      if (wkeep && own[u]) wkeep[j * items + it] = ok[u] ? wn : 0.0;
      double* sink = g_sink + threadIdx.x;
      *(ok[u] ? a.r + g : sink) = newmark_r(f, uj, vn, an);
      *(ok[u] ? a.w + g : sink) = wn;
      if (STORE) {
        const int64_t gp = (po + (int64_t)j * nb + i) * a.NS + s0 + s;
        *(ok[u] && a.xs ? a.xs + (xo + (int64_t)(j + 1) * nb + i) * a.NS + s0 + s : sink) = uj;
        *(ok[u] ? a.fs + gp : sink) = a.field_kind == 0 ? an : vn;
        *(ok[u] && a.vs ? a.vs + gp : sink) = vn;
      }
      if (own[u]) L.y[it] = uj;
    }
    commit<NBT>(reg, L.F[cur ^ 1], nb);   // the last level commits an unused block
    __syncthreads();
    for (int it = threadIdx.x; it < items; it += WT) {
      if (j == 1) L.u1[it] = L.y[it];
      L.x[it] = L.y[it];
    }
    __syncthreads();
    cur ^= 1;
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      cq[u] = nq[u];
      cr[u] = nr[u];
      cw[u] = nw[u];
      cb[0][u] = nbd[0][u];
      cb[1][u] = nbd[1][u];
      cb[2][u] = nbd[2][u];
    }
  }
}

// STORE: the checkpoint recompute's launches, which also store the unknowns
// with ghosts and the level field for the adjoint (a.xs, a.fs, a.vs; a.xs may
// be NULL when only the level field is wanted).
template <int NBT, int S, bool STORE>
__device__ __forceinline__ void recover_body(int e, int s0, const MeshDev& m, const FactorsDev& f,
                                             const StepArgs& a, StepLds<NBT, S>& L,
                                             double* wkeep = nullptr) {
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
    if (STORE && s < ns) {
      if (a.xs) a.xs[(xo + (int64_t)(n + 1) * nb + i) * a.NS + s0 + s] = un;
      double fv = a.field_kind == 0 ? a.A[m.loop_nodes[lo + i] * a.NS + s0 + s]
                                    : a.V[m.loop_nodes[lo + i] * a.NS + s0 + s];
      a.fs[(po + (int64_t)n * nb + i) * a.NS + s0 + s] = fv;
      if (a.vs) a.vs[(po + (int64_t)n * nb + i) * a.NS + s0 + s] = a.V[m.loop_nodes[lo + i] * a.NS + s0 + s];
    }
  }
  __syncthreads();
  recover_levels<NBT, S, STORE>(e, s0, m, f, a, L, wkeep);
  if (!STORE || !a.xs) return;
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

// Device step counter of graph replays.
__global__ void set_step_kernel(int64_t* kdev, int64_t k) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *kdev = k;
}

__global__ void advance_step_kernel(int64_t* kdev) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *kdev = *kdev + 1;
}

// One block per (element of an n_b class, group of S shots), blocks ordered by
// sweep_item.
template <int NBT, int S>
__global__ void __launch_bounds__(WT) condense_kernel(const int32_t* __restrict__ elems, int64_t n_el, MeshDev m,
                                                      FactorsDev f, StepArgs a) {
  __shared__ StepLds<NBT, S> L;
  int64_t ei;
  int g;
  if (!sweep_item(n_el, (a.NS + S - 1) / S, ei, g)) return;
  condense_body<NBT, S>(elems[ei], g * S, m, f, a, L);
}

template <int NBT, int S, bool STORE>
__global__ void __launch_bounds__(WT) recover_kernel(const int32_t* __restrict__ elems, int64_t n_el, MeshDev m,
                                                     FactorsDev f, StepArgs a) {
  __shared__ StepLds<NBT, S> L;
  int64_t ei;
  int g;
  if (!sweep_item(n_el, (a.NS + S - 1) / S, ei, g)) return;
  recover_body<NBT, S, STORE>(elems[ei], g * S, m, f, a, L);
}

// Joint sweep of one (element, group of S shots): the recover sweep of step k
// (down the levels), which keeps every level's new w in LDS, then the condense
// sweep of step k + 1 (up the levels) from that w and the nodal state already
// updated by step k.  Every value is computed by the same expressions as in the
// two separate sweeps, so the results are bit-identical; the interior state is
// read and written once per step (the condense takes its w from LDS), and one
// launch is saved.
template <int NBT, int S, bool STORE>
__global__ void __launch_bounds__(WT) joint_kernel(const int32_t* __restrict__ elems, int64_t n_el, MeshDev m,
                                                   FactorsDev f, StepArgs a) {
  __shared__ StepLds<NBT, S> L;
  extern __shared__ double wkeep[];   // [interior levels][n_b * S] of the element
  int64_t ei;
  int g;
  if (!sweep_item(n_el, (a.NS + S - 1) / S, ei, g)) return;
  const int e = elems[ei];
  const int s0 = g * S;
  recover_body<NBT, S, STORE>(e, s0, m, f, a, L, wkeep);
  __syncthreads();
  condense_body<NBT, S, true>(e, s0, m, f, a, L, wkeep);
}

// One persistent launch over all n_b classes: the blocks walk the work items
// (element, group of S shots) in order of decreasing cost (N_r n_b^2), item
// w = blockIdx.x + i gridDim.x; each item runs the body of its element's class
// in a shared LDS buffer sized for the largest class.
template <int S, bool CONDENSE, bool STORE>
__global__ void __launch_bounds__(WT) sweep_fused_kernel(const int32_t* __restrict__ order, int64_t n_work,
                                                         int groups, MeshDev m, FactorsDev f, StepArgs a) {
  __shared__ StepLds<24, S> L;
  for (int64_t w = blockIdx.x; w < n_work; w += gridDim.x) {
    const int e = order[w / groups];
    const int s0 = (int)(w % groups) * S;
    const int nb = m.nb[e];
    if (nb <= 8) {
      auto& Ls = *reinterpret_cast<StepLds<8, S>*>(&L);
      if (CONDENSE) condense_body<8, S>(e, s0, m, f, a, Ls); else recover_body<8, S, STORE>(e, s0, m, f, a, Ls);
    } else if (nb <= 16) {
      auto& Ls = *reinterpret_cast<StepLds<16, S>*>(&L);
      if (CONDENSE) condense_body<16, S>(e, s0, m, f, a, Ls); else recover_body<16, S, STORE>(e, s0, m, f, a, Ls);
    } else {
      if (CONDENSE) condense_body<24, S>(e, s0, m, f, a, L); else recover_body<24, S, STORE>(e, s0, m, f, a, L);
    }
    __syncthreads();
  }
}

// F = sum of element sources gathered over node -> slot + point sources;
// Unew = initial guess of the coarse solve: the predictor u + dt v + dt^2/2 a
// plus the correction the previous step needed on top of its own predictor.
__global__ void rhs_kernel(MeshDev m, int NS, const double* __restrict__ fhat, double* __restrict__ F,
                           const double* __restrict__ U, const double* __restrict__ V,
                           const double* __restrict__ A, double* __restrict__ Unew,
                           const double* __restrict__ corr, double dt, SourceTable src, int64_t k,
                           const int64_t* __restrict__ kdev) {
  if (kdev) k = *kdev;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= m.n_nodes * NS) return;
  int64_t node = g / NS;
  int s = (int)(g % NS);
  double acc = 0.0;
  acc = node_gather<false>(acc, m.node_slot, m.node_ptr[node], m.node_ptr[node + 1], fhat, NS, s);
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

// Nodal Newmark update (W: the nodal w of the old state in, of the new one
// out), predictor correction and receiver sampling.  With env
// (growth envelope of the run, [n_steps][NS]) every new nodal displacement is
// checked against the bound of its step and shot: a non-finite value sets status
// bit 32, a finite one beyond the bound bit 16, and the first such step is kept
// in status[1].
__global__ void nodal_kernel(int64_t n_nodes, int NS, FactorsDev f, const double* __restrict__ Unew,
                             double* __restrict__ U, double* __restrict__ V, double* __restrict__ A,
                             double* __restrict__ W, double* __restrict__ corr,
                             int n_rec, const int64_t* __restrict__ rec_node, double* __restrict__ traces,
                             int64_t n_steps, int64_t k, const int64_t* __restrict__ kdev,
                             double* __restrict__ ustore, const double* __restrict__ env,
                             int* __restrict__ status) {
  if (kdev) k = *kdev;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t nn = n_nodes * NS;
  if (g < nn) {
    double uo = U[g], vo = V[g], ao = A[g], un = Unew[g];
    if (env && !(fabs(un) <= env[(k - 1) * NS + g % NS])) {
      atomicOr(&status[0], isfinite(un) ? 16 : 32);
      atomicCAS(&status[1], -1, (int)k);
    }
    if (ustore) ustore[(k - 1) * nn + g] = un;
    corr[g] = un - (uo + f.dt * vo + 0.5 * f.dt * f.dt * ao);
    const double vn = f.c1 * (un - uo) + f.c2 * vo + f.c3 * ao;
    const double an = f.a0 * un - W[g];
    V[g] = vn;
    A[g] = an;
    U[g] = un;
    W[g] = newmark_w(f, un, vn, an);
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
  dim3 grid((unsigned)sweep_blocks(cnt, (a.NS + S - 1) / S));
  if (condense)
    hipLaunchKernelGGL((condense_kernel<NBT, S>), grid, dim3(WT), 0, st, m->class_elems[cl], cnt, m->d, f, a);
  else if (a.xs || a.fs)
    hipLaunchKernelGGL((recover_kernel<NBT, S, true>), grid, dim3(WT), 0, st, m->class_elems[cl], cnt, m->d, f, a);
  else
    hipLaunchKernelGGL((recover_kernel<NBT, S, false>), grid, dim3(WT), 0, st, m->class_elems[cl], cnt, m->d, f,
                       a);
}

template <int NBT>
void launch_cr_s(bool condense, sbfwi_mesh_s* m, int cl, int S, const FactorsDev& f, const StepArgs& a,
                 hipStream_t st) {
  switch (S) {
    case 1: launch_cr<NBT, 1>(condense, m, cl, f, a, st); break;
    case 2: launch_cr<NBT, 2>(condense, m, cl, f, a, st); break;
    case 4: launch_cr<NBT, 4>(condense, m, cl, f, a, st); break;
    case 8: launch_cr<NBT, 8>(condense, m, cl, f, a, st); break;
    default: launch_cr<NBT, 16>(condense, m, cl, f, a, st); break;
  }
}

template <int S>
void launch_fused(bool condense, sbfwi_mesh_s* m, const FactorsDev& f, const StepArgs& a, hipStream_t st) {
  const int groups = (a.NS + S - 1) / S;
  const int64_t n_work = m->n_elem * groups;
  const int which = condense ? 0 : (a.xs || a.fs ? 2 : 1);
  auto kern = which == 0 ? sweep_fused_kernel<S, true, false>
                         : which == 1 ? sweep_fused_kernel<S, false, false> : sweep_fused_kernel<S, false, true>;
  static std::atomic<int> per_cu[3] = {0, 0, 0};   // occupancy, queried once per kernel
  int pc = per_cu[which].load();
  if (pc == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, kern, WT, 0) != hipSuccess || pc <= 0) pc = 1;
    per_cu[which].store(pc);
  }
  const int64_t cap = (int64_t)(pc > 0 ? pc : 1) * sbfwi_device_cus();
  const unsigned blocks = (unsigned)(n_work < cap ? n_work : cap);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(WT), 0, st, m->d.elem_by_cost, n_work, groups, m->d, f, a);
}

// Condense or recover over every element, with the shots-per-block choice of
// the plan for each n_b class (or its single persistent launch).
void launch_step_sweep(bool condense, sbfwi_mesh_s* m, const FactorsDev& f, const SweepPlan& plan,
                             const StepArgs& a, hipStream_t st) {
  const int kind = condense ? SW_CONDENSE : SW_RECOVER;
  const int fs = plan.fusedS[kind];
  if (fs > 0) {
    switch (fs) {
      case 1: launch_fused<1>(condense, m, f, a, st); break;
      case 2: launch_fused<2>(condense, m, f, a, st); break;
      case 4: launch_fused<4>(condense, m, f, a, st); break;
      case 8: launch_fused<8>(condense, m, f, a, st); break;
      default: launch_fused<16>(condense, m, f, a, st); break;
    }
    return;
  }
  const int def = sbfwi_default_shots_per_block(a.NS);
  launch_cr_s<8>(condense, m, 0, plan.S[kind][0] > 0 ? plan.S[kind][0] : def, f, a, st);
  launch_cr_s<16>(condense, m, 1, plan.S[kind][1] > 0 ? plan.S[kind][1] : def, f, a, st);
  launch_cr_s<24>(condense, m, 2, plan.S[kind][2] > 0 ? plan.S[kind][2] : def, f, a, st);
}

void launch_sweep(bool condense, sbfwi_factors_s* fac, const StepArgs& a, hipStream_t st) {
  ProfScope ps(condense ? PK_CONDENSE : (a.xs || a.fs ? PK_RECOVER_STORE : PK_RECOVER), st);
  launch_step_sweep(condense, fac->m, fac->d, fac->plan, a, st);
}

// LDS of a joint-sweep block (the static sweep buffers and the kept w of the
// class's deepest element) is held within this bound; larger classes run the
// two sweeps one after the other.
constexpr size_t kJointLdsMax = 48 * 1024;

template <int NBT, int S>
bool launch_joint_cls(sbfwi_mesh_s* m, int cl, const FactorsDev& f, const StepArgs& a, hipStream_t st) {
  const int64_t cnt = (int64_t)m->h_class_elems[cl].size();
  if (cnt == 0) return true;
  const size_t dyn = (size_t)m->class_nmax[cl] * NBT * S * sizeof(double);
  if (sizeof(StepLds<NBT, S>) + dyn > kJointLdsMax) return false;
  dim3 grid((unsigned)sweep_blocks(cnt, (a.NS + S - 1) / S));
  if (a.xs || a.fs)
    hipLaunchKernelGGL((joint_kernel<NBT, S, true>), grid, dim3(WT), dyn, st, m->class_elems[cl], cnt, m->d, f, a);
  else
    hipLaunchKernelGGL((joint_kernel<NBT, S, false>), grid, dim3(WT), dyn, st, m->class_elems[cl], cnt, m->d, f,
                       a);
  return true;
}

template <int NBT>
bool launch_joint_s(sbfwi_mesh_s* m, int cl, int S, const FactorsDev& f, const StepArgs& a, hipStream_t st) {
  switch (S) {
    case 1: return launch_joint_cls<NBT, 1>(m, cl, f, a, st);
    case 2: return launch_joint_cls<NBT, 2>(m, cl, f, a, st);
    case 4: return launch_joint_cls<NBT, 4>(m, cl, f, a, st);
    case 8: return launch_joint_cls<NBT, 8>(m, cl, f, a, st);
    default: return launch_joint_cls<NBT, 16>(m, cl, f, a, st);
  }
}

// Recover of step k and condense of step k + 1: one joint launch per n_b class
// with the recover sweep's shots per block, or, where its LDS would not fit or
// the plan runs a sweep as one persistent launch, the two sweeps in turn.
void launch_joint(sbfwi_factors_s* fac, const StepArgs& a, hipStream_t st) {
  sbfwi_mesh_s* m = fac->m;
  const SweepPlan& plan = fac->plan;
  if (plan.fusedS[SW_RECOVER] > 0 || plan.fusedS[SW_CONDENSE] > 0) {
    launch_sweep(false, fac, a, st);
    launch_sweep(true, fac, a, st);
    return;
  }
  ProfScope ps(a.xs || a.fs ? PK_JOINT_STORE : PK_JOINT, st);
  const int def = sbfwi_default_shots_per_block(a.NS);
  for (int cl = 0; cl < 3; ++cl) {
    const int S = plan.S[SW_RECOVER][cl] > 0 ? plan.S[SW_RECOVER][cl] : def;
    const bool ok = cl == 0 ? launch_joint_s<8>(m, cl, S, fac->d, a, st)
                            : cl == 1 ? launch_joint_s<16>(m, cl, S, fac->d, a, st)
                                      : launch_joint_s<24>(m, cl, S, fac->d, a, st);
    if (ok) continue;
    const int Sc = plan.S[SW_CONDENSE][cl] > 0 ? plan.S[SW_CONDENSE][cl] : def;
    if (cl == 0) {
      launch_cr_s<8>(false, m, cl, S, fac->d, a, st);
      launch_cr_s<8>(true, m, cl, Sc, fac->d, a, st);
    } else if (cl == 1) {
      launch_cr_s<16>(false, m, cl, S, fac->d, a, st);
      launch_cr_s<16>(true, m, cl, Sc, fac->d, a, st);
    } else {
      launch_cr_s<24>(false, m, cl, S, fac->d, a, st);
      launch_cr_s<24>(true, m, cl, Sc, fac->d, a, st);
    }
  }
}

}  // namespace

// interior r, w; nodal U, V, A, W and the predictor correction of the coarse solve
int64_t sbfwi_state_size(sbfwi_mesh_s* m, int NS) { return (2 * m->n_int + 5 * m->n_nodes) * (int64_t)NS; }

int sbfwi_step_work_alloc(StepWork* w, sbfwi_mesh_s* m, int NS) {
  w->NS = NS;
  int64_t ni = m->n_int * NS, nn = m->n_nodes * NS, nl = m->n_loop * NS;
  SBFWI_CHECK(sbfwi_alloc(&w->r, 2 * ni + 5 * nn));  // r, w, U, V, A, W, corr contiguous
  w->w = w->r + ni;
  w->U = w->w + ni;
  w->V = w->U + nn;
  w->A = w->V + nn;
  w->W = w->A + nn;
  w->corr = w->W + nn;
  SBFWI_CHECK(sbfwi_alloc(&w->q, ni));
  SBFWI_CHECK(sbfwi_alloc(&w->yn, nl));
  SBFWI_CHECK(sbfwi_alloc(&w->fhat, nl));
  SBFWI_CHECK(sbfwi_alloc(&w->F, nn));
  SBFWI_CHECK(sbfwi_alloc(&w->Unew, nn));
  SBFWI_CHECK(sbfwi_coarse_work_alloc(&w->cw, m, NS));
  SBFWI_CHECK(sbfwi_alloc(&w->kdev, 1));
  return SBFWI_OK;
}

void sbfwi_step_work_free(StepWork* w) {
  sbfwi_dev_free(w->r);
  sbfwi_dev_free(w->q);
  sbfwi_dev_free(w->yn);
  sbfwi_dev_free(w->fhat);
  sbfwi_dev_free(w->F);
  sbfwi_dev_free(w->Unew);
  sbfwi_coarse_work_free(&w->cw);
  sbfwi_dev_free(w->kdev);
  sbfwi_dev_free(w->env);
  if (w->g_pre) (void)hipGraphExecDestroy(w->g_pre);
  if (w->g_post) (void)hipGraphExecDestroy(w->g_post);
  *w = StepWork();
}

int sbfwi_step_zero(sbfwi_mesh_s* m, StepWork* w, hipStream_t s) {
  SBFWI_HIP(hipMemsetAsync(w->r, 0, sizeof(double) * sbfwi_state_size(m, w->NS), s));
  w->condensed = false;
  return SBFWI_OK;
}

int sbfwi_state_copy(sbfwi_mesh_s* m, StepWork* w, double* dst, int to_store, hipStream_t s) {
  size_t bytes = sizeof(double) * sbfwi_state_size(m, w->NS);
  if (to_store) {
    SBFWI_HIP(hipMemcpyAsync(dst, w->r, bytes, hipMemcpyDeviceToDevice, s));
  } else {
    SBFWI_HIP(hipMemcpyAsync(w->r, dst, bytes, hipMemcpyDeviceToDevice, s));
    w->condensed = false;   // a new state: its sources are not swept yet
  }
  return SBFWI_OK;
}

namespace {

StepArgs step_args(StepWork* w, double* xs, double* fs, int field_kind, double* vs) {
  StepArgs a;
  a.NS = w->NS;
  a.r = w->r; a.w = w->w;
  a.U = w->U; a.V = w->V; a.A = w->A; a.W = w->W;
  a.q = w->q; a.yn = w->yn; a.fhat = w->fhat; a.Unew = w->Unew;
  a.xs = xs; a.fs = fs; a.field_kind = field_kind; a.vs = vs;
  return a;
}

// gather of the coarse right-hand side and initial guess
int step_rhs(sbfwi_factors_s* f, StepWork* w, const StepArgs& a, int64_t k, const int64_t* kdev,
             const SourceTable& src, hipStream_t st) {
  sbfwi_mesh_s* m = f->m;
  int64_t nn = m->n_nodes * w->NS;
  {
    ProfScope ps(PK_RHS, st);
    hipLaunchKernelGGL(rhs_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, m->d, w->NS, w->fhat,
                       w->F, w->U, w->V, w->A, w->Unew, w->corr, f->dt, src, k, kdev);
  }
  SBFWI_HIP(hipGetLastError());
  return SBFWI_OK;
}

// nodal Newmark update and receivers (a.Unew: the step's coarse solution)
int step_nodal(sbfwi_factors_s* f, StepWork* w, const StepArgs& a, int64_t k, const int64_t* kdev, int n_rec,
               const int64_t* rec_node, double* traces, int64_t n_steps, hipStream_t st) {
  sbfwi_mesh_s* m = f->m;
  int64_t nn = m->n_nodes * w->NS;
  int64_t tot = nn + (int64_t)n_rec * w->NS;
  {
    ProfScope ps(PK_NODAL, st);
    hipLaunchKernelGGL(nodal_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, m->n_nodes, w->NS,
                       f->d, a.Unew, w->U, w->V, w->A, w->W, w->corr, n_rec, rec_node, traces, n_steps, k, kdev,
                       w->ustore, w->env, f->d.status);
  }
  SBFWI_HIP(hipGetLastError());
  return SBFWI_OK;
}

// the recover sweep of the step, joined with the condense of the next one when
// it follows and joint sweeps are on; returns whether the next step is condensed
int step_sweeps(sbfwi_factors_s* f, const StepArgs& a, bool next, hipStream_t st, bool* condensed) {
  if (next && f->joint_sweeps) {
    launch_joint(f, a, st);
    *condensed = true;
  } else {
    launch_sweep(false, f, a, st);
    *condensed = false;
  }
  SBFWI_HIP(hipGetLastError());
  return SBFWI_OK;
}

int capture(hipStream_t st, hipGraphExec_t* out, const std::function<int()>& body) {
  hipGraph_t g = nullptr;
  SBFWI_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  sbfwi_prof_suspend(1);
  int rc = body();
  sbfwi_prof_suspend(0);
  hipError_t e = hipStreamEndCapture(st, &g);
  if (rc != SBFWI_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return sbfwi_fail(SBFWI_EHIP, "graph capture failed: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return sbfwi_fail(SBFWI_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
  return SBFWI_OK;
}

}  // namespace

int sbfwi_forward_step(sbfwi_factors_s* f, StepWork* w, int64_t k, const SourceTable& src, int n_rec,
                       const int64_t* rec_node, double* traces, int64_t n_steps, double* xs, double* fs,
                       int field_kind, hipStream_t st, double* vs, const double* usol, bool next) {
  StepArgs a = step_args(w, xs, fs, field_kind, vs);
  if (!w->condensed) launch_sweep(true, f, a, st);
  if (usol) {   // the coarse solution is known: no gather, no coarse solve
    a.Unew = const_cast<double*>(usol);   // read only by the nodal update and the recover sweep
  } else {
    SBFWI_CHECK(step_rhs(f, w, a, k, nullptr, src, st));
    SBFWI_CHECK(sbfwi_coarse_solve(f, &w->cw, 0, w->F, w->Unew, k, st));
  }
  SBFWI_CHECK(step_nodal(f, w, a, k, nullptr, n_rec, rec_node, traces, n_steps, st));
  return step_sweeps(f, a, next, st, &w->condensed);
}

int sbfwi_graph_step_reset(StepWork* w, int64_t k, hipStream_t st) {
  hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, st, w->kdev, k);
  SBFWI_HIP(hipGetLastError());
  return SBFWI_OK;
}

int sbfwi_forward_step_graph(sbfwi_factors_s* f, StepWork* w, const SourceTable& src, int n_rec,
                             const int64_t* rec_node, double* traces, int64_t n_steps, hipStream_t st) {
  const StepArgs a = step_args(w, nullptr, nullptr, 0, nullptr);
  // with joint sweeps each replayed step ends by condensing the next one (the last
  // step's is unused), so only the first step needs a condense of its own
  const bool joint = f->joint_sweeps != 0;
  if (!w->g_pre) {
    if (joint && !w->condensed) launch_sweep(true, f, a, st);
    SBFWI_CHECK(capture(st, &w->g_pre, [&]() -> int {
      if (!joint) launch_sweep(true, f, a, st);
      SBFWI_CHECK(step_rhs(f, w, a, 0, w->kdev, src, st));
      return sbfwi_coarse_solve_parts(f, &w->cw, 0, w->F, w->Unew, 0, w->kdev, 1, st);
    }));
    SBFWI_CHECK(capture(st, &w->g_post, [&]() -> int {
      SBFWI_CHECK(sbfwi_coarse_solve_parts(f, &w->cw, 0, w->F, w->Unew, 0, w->kdev, 4, st));
      SBFWI_CHECK(step_nodal(f, w, a, 0, w->kdev, n_rec, rec_node, traces, n_steps, st));
      bool cd = false;
      SBFWI_CHECK(step_sweeps(f, a, joint, st, &cd));
      hipLaunchKernelGGL(advance_step_kernel, dim3(1), dim3(64), 0, st, w->kdev);
      SBFWI_HIP(hipGetLastError());
      return SBFWI_OK;
    }));
  }
  SBFWI_HIP(hipGraphLaunch(w->g_pre, st));
  SBFWI_CHECK(sbfwi_coarse_solve_parts(f, &w->cw, 0, w->F, w->Unew, 0, w->kdev, 2, st));
  SBFWI_HIP(hipGraphLaunch(w->g_post, st));
  w->condensed = joint;
  return SBFWI_OK;
}

namespace {

// Average time in ms of reps launches (after one untimed launch) on stream st.
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

void launch_cls(bool condense, sbfwi_mesh_s* m, int cl, int S, const FactorsDev& f, const StepArgs& a,
                hipStream_t st) {
  if (cl == 0) launch_cr_s<8>(condense, m, cl, S, f, a, st);
  else if (cl == 1) launch_cr_s<16>(condense, m, cl, S, f, a, st);
  else launch_cr_s<24>(condense, m, cl, S, f, a, st);
}

void launch_fused_s(bool condense, int S, sbfwi_mesh_s* m, const FactorsDev& f, const StepArgs& a,
                    hipStream_t st) {
  switch (S) {
    case 1: launch_fused<1>(condense, m, f, a, st); break;
    case 2: launch_fused<2>(condense, m, f, a, st); break;
    case 4: launch_fused<4>(condense, m, f, a, st); break;
    case 8: launch_fused<8>(condense, m, f, a, st); break;
    default: launch_fused<16>(condense, m, f, a, st); break;
  }
}

int tune_step(sbfwi_factors_s* f, StepWork& w, int NS, hipStream_t st, hipEvent_t e0, hipEvent_t e1, double* out) {
  sbfwi_mesh_s* m = f->m;
  StepArgs a;
  a.NS = NS;
  a.r = w.r; a.w = w.w;
  a.U = w.U; a.V = w.V; a.A = w.A; a.W = w.W;
  a.q = w.q; a.yn = w.yn; a.fhat = w.fhat; a.Unew = w.Unew;
  a.xs = nullptr; a.fs = nullptr; a.field_kind = 0; a.vs = nullptr;
  const int cands[5] = {1, 2, 4, 8, 16};
  int smax = 1;
  while (smax < NS) smax *= 2;
  for (int kind = SW_CONDENSE; kind <= SW_RECOVER; ++kind) {
    const bool cond = kind == SW_CONDENSE;
    double sum_best = 0.0;
    for (int cl = 0; cl < 3; ++cl) {
      f->plan.S[kind][cl] = 0;
      if (m->h_class_elems[cl].empty()) continue;
      float best = 1e30f;
      int bs = 0;
      for (int S : cands) {
        if (S > smax) break;
        float t = 0.f;
        SBFWI_CHECK(time_launch([&] { launch_cls(cond, m, cl, S, f->d, a, st); }, 3, st, e0, e1, &t));
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
      SBFWI_CHECK(time_launch([&] { launch_fused_s(cond, S, m, f->d, a, st); }, 3, st, e0, e1, &t));
      if (t < bestf) { bestf = t; bfs = S; }
    }
    // the single persistent launch is kept only when clearly faster
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

int sbfwi_tune_step_sweeps(sbfwi_factors_s* f, int NS, hipStream_t st, double* out) {
  StepWork w;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = sbfwi_step_work_alloc(&w, f->m, NS);
  if (rc == SBFWI_OK) rc = sbfwi_step_zero(f->m, &w, st);
  if (rc == SBFWI_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = sbfwi_fail(SBFWI_EHIP, "event creation failed");
  if (rc == SBFWI_OK) rc = tune_step(f, w, NS, st, e0, e1, out);
  (void)hipStreamSynchronize(st);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  sbfwi_step_work_free(&w);
  return rc;
}

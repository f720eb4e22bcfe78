// Element factorisation (once per model) and coarse assembly.
//
// One workgroup per element.  The coefficient matrices of eq. Es are built
// from per-segment geometric weights: with linear boundary segments and the
// density interpolated linearly between nodal values, every segment block of
// E0, E1, E2, M0 is a linear combination of the two end-node densities,
//   E^tau_seg(a, b) = sum_end alpha^tau[seg][end][a][b] rho_{seg+end},
// where alpha integrates (two-point Gauss, exact for the cubic integrands)
// c^2 det J_b (b1.b1 N N, b2.b1 dN N, b2.b2 dN dN) and det J_b N N times the
// end-node shape function.  The same alpha are the derivatives of the
// coefficient matrices with respect to the nodal densities, kept for the
// gradient.  All matrices are cyclic tridiagonal and are handled as bands.
//
// The radial rows follow the central-difference discretisation of the
// Newmark-discretised radial equation (eq. ODE_Newmark, eq. FD) with
// one-sided differences of E0, E1 at the end levels and the two ghost rows of
// the flux boundary conditions (eq. system).  The radial Galerkin scheme
// (scheme 1) replaces them by linear elements in xi with the radial mass
// lumped, written in the same row layout: the negated Galerkin rows of the
// interior levels, an identity row for the unused level n + 1 that carries
// the boundary level's mass source (u_{n+1} = M_n w_n), the boundary row
// (K_{n,n-1}, K_nn + a0 M_n, -I) and an identity row for the unused level -1;
// the elimination below then gives G = -I and the Galerkin Schur complement.  The elimination is the paper's
// block Gauss sweep, organised so that only phi~_j^-1 is stored per level:
// rho_j = theta_j phi~_{j-1}^-1 is applied as theta_j (phi~_{j-1}^-1 .), which
// halves the factor storage and lets the same stored block serve the forward
// and the transposed sweeps.
#include "fd_bands.h"
#include "sbfwi_internal.h"

namespace {

constexpr int FT = 256;  // threads per factor workgroup

struct ElemCtx {
  int nb, n;        // boundary nodes, intervals (levels 0..n)
  double xi0, h, c2, a0;
  const double* rho;  // element's [N_r][nb] densities (global)
  const double* alpha;  // LDS [4][nb][2][4]
  int scheme;           // 0 central differences, 1 radial Galerkin, 2 low-frequency expansion
  const double* rgw;    // Galerkin rows: weights of the element's intervals [n][kRgW]
  int lfe;              // radially constant coefficients: every level takes the boundary level's densities
};

__device__ __forceinline__ int md(int i, int nb) { return (i % nb + nb) % nb; }

// Band entry t (0 sub, 1 diag, 2 super) of row i of E^tau at level lev.
__device__ double e_band(const ElemCtx& c, int tau, int lev, int t, int i) {
  const int nb = c.nb;
  const double* r = c.rho + (int64_t)(c.lfe ? c.n : lev) * nb;
  const double* al = c.alpha + tau * nb * 8;
  auto A = [&](int seg, int end, int ab) { return al[seg * 8 + end * 4 + ab]; };
  if (t == 1) {
    int s0 = i, s1 = md(i - 1, nb);
    return A(s0, 0, 0) * r[i] + A(s0, 1, 0) * r[md(i + 1, nb)] +
           A(s1, 0, 3) * r[s1] + A(s1, 1, 3) * r[i];
  } else if (t == 2) {  // M[i][i+1]: segment i, (a, b) = (0, 1)
    return A(i, 0, 1) * r[i] + A(i, 1, 1) * r[md(i + 1, nb)];
  } else {              // M[i][i-1]: segment i-1, (a, b) = (1, 0)
    int s1 = md(i - 1, nb);
    return A(s1, 0, 2) * r[s1] + A(s1, 1, 2) * r[i];
  }
}

// Band entry t of the transpose of E^tau at level lev.
__device__ double e_band_T(const ElemCtx& c, int tau, int lev, int t, int i) {
  if (t == 1) return e_band(c, tau, lev, 1, i);
  if (t == 0) return e_band(c, tau, lev, 2, md(i - 1, c.nb));
  return e_band(c, tau, lev, 0, md(i + 1, c.nb));
}

__device__ __forceinline__ double xi_of(const ElemCtx& c, int j) { return c.xi0 + c.h * j; }

// d/dxi of E^tau at level j: central inside, one-sided at the end levels.
__device__ double d_band(const ElemCtx& c, int tau, int j, int t, int i, bool transpose) {
  auto E = [&](int lev) { return transpose ? e_band_T(c, tau, lev, t, i) : e_band(c, tau, lev, t, i); };
  if (j == 0) return (E(1) - E(0)) / c.h;
  if (j == c.n) return (E(c.n) - E(c.n - 1)) / c.h;
  return (E(j + 1) - E(j - 1)) / (2.0 * c.h);
}

// Galerkin rows.  Stiffness block (local row p, column q) of interval j and
// the lumped mass of its local level p, band entry t of row i.
__device__ double rg_k(const ElemCtx& c, int j, int p, int q, int t, int i) {
  const double* w = c.rgw + (int64_t)j * kRgW;
  const int o = 4 * p + 2 * q;
  double v = 0.0;
  for (int e = 0; e < 2; ++e) {
    const int lev = j + e;
    v += w[o + e] * e_band(c, 0, lev, t, i) + w[8 + o + e] * e_band_T(c, 1, lev, t, i) +
         w[16 + o + e] * e_band(c, 1, lev, t, i) + w[24 + o + e] * e_band(c, 2, lev, t, i);
  }
  return v;
}
__device__ double rg_m(const ElemCtx& c, int j, int p, int t, int i) {
  const double* w = c.rgw + (int64_t)j * kRgW;
  return w[32 + 2 * p] * e_band(c, 3, j, t, i) + w[33 + 2 * p] * e_band(c, 3, j + 1, t, i);
}

__device__ double row_band_rg(const ElemCtx& c, int which, int r, int t, int i) {
  const int n = c.n;
  const double id = t == 1 ? 1.0 : 0.0;
  if (r == -1) return which == 0 ? id : 0.0;
  if (r == n) return which == 2 ? id : (which == 3 ? rg_m(c, n - 1, 1, t, i) : 0.0);
  if (r == n + 1) {
    if (which == 0) return rg_k(c, n - 1, 1, 0, t, i);
    if (which == 1) return rg_k(c, n - 1, 1, 1, t, i) + c.a0 * rg_m(c, n - 1, 1, t, i);
    return which == 2 ? -id : 0.0;
  }
  // interior level r: intervals r - 1 (local level 1) and r (local level 0)
  if (which == 0) return r >= 1 ? -rg_k(c, r - 1, 1, 0, t, i) : 0.0;
  if (which == 2) return -rg_k(c, r, 0, 1, t, i);
  const double m = (r >= 1 ? rg_m(c, r - 1, 1, t, i) : 0.0) + rg_m(c, r, 0, t, i);
  if (which == 3) return -m;
  const double k = (r >= 1 ? rg_k(c, r - 1, 1, 1, t, i) : 0.0) + rg_k(c, r, 0, 0, t, i);
  return -(k + c.a0 * m);
}

// theta_r, psi_r, P_r (entry (t, i), level r = 0 .. n) of the central-difference
// rows through the helpers the sweeps use to form them on the fly.
__device__ FdRow fd_row_at(const ElemCtx& c, int r, int t, int i) {
  const int nb = c.nb;
  double k[kFdKappa];
  auto al = [&](int tau, int seg, int end, int ab) { return c.alpha[tau * nb * 8 + seg * 8 + end * 4 + ab]; };
  fd_kappa(al, nb, t, i, k);
  auto ent = [&](int lev) {
    const double* rr = c.rho + (int64_t)(c.lfe ? c.n : lev) * nb;
    return fd_entry(k, rr[md(i - 1, nb)], rr[i], rr[md(i + 1, nb)]);
  };
  const FdEntry v = ent(r);
  const double e0m = r > 0 ? ent(r - 1).e0 : 0.0, e0p = r < c.n ? ent(r + 1).e0 : 0.0;
  return fd_row(c.xi0, fd_step(c.xi0, c.n), r, c.n, e0m, v, e0p);
}

// Band entries of the rows: which = 0 theta, 1 phi, 2 psi, 3 P, for row r = -1 .. n+1.
template <int SCH>
__device__ double row_band(const ElemCtx& c, int which, int r, int t, int i) {
  if constexpr (SCH != SBFWI_SCHEME_PAPER_FD) return row_band_rg(c, which, r, t, i);
  const double h = c.h;
  if (r == -1 || r == c.n + 1) {
    int lev = (r == -1) ? 0 : c.n;
    double x = xi_of(c, lev);
    if (which == 0) return -x * e_band(c, 0, lev, t, i) / (2.0 * h);
    if (which == 1) return e_band_T(c, 1, lev, t, i);
    if (which == 2) return x * e_band(c, 0, lev, t, i) / (2.0 * h);
    return 0.0;
  }
  if (which == 1) {
    const double x = xi_of(c, r);
    const double e0 = e_band(c, 0, r, t, i);
    return -2.0 * x * x * e0 / (h * h) - e_band(c, 2, r, t, i) + x * d_band(c, 1, r, t, i, true) -
           c.a0 * x * x * e_band(c, 3, r, t, i);
  }
  const FdRow o = fd_row_at(c, r, t, i);
  return which == 0 ? o.th : (which == 2 ? o.ps : o.pm);
}

template <int NBT>
struct Lds {
  double alpha[4 * NBT * 8];
  double band[3][3 * NBT];    // scratch bands
  double A[NBT * NBT];        // dense work blocks
  double B[NBT * NBT];
  double Z[NBT * NBT];
  double Fp[NBT * NBT];       // phi~^-1 of the previous level
  double Pp[NBT * NBT];       // psi~ of the previous level (dense)
  double Ph[NBT * NBT];       // phi~_n
  double Ph1[NBT * NBT];      // phi~_{n+1}
  double W[NBT * 2 * NBT];    // Gauss-Jordan workspace
  double fac[NBT];
  int piv;
  int bad;
};

// dst = dense(band)
template <int NBT>
__device__ void band_to_dense(const double* band, double* dst, int nb) {
  for (int q = threadIdx.x; q < nb * nb; q += FT) {
    int i = q / nb, j = q % nb;
    double v = 0.0;
    if (j == i) v = band[nb + i];
    if (j == md(i + 1, nb)) v += band[2 * nb + i];
    if (j == md(i - 1, nb)) v += band[i];
    dst[i * NBT + j] = v;
  }
}

// dst = D * B (dense x band); dst may not alias D
template <int NBT>
__device__ void dense_band(const double* D, const double* band, double* dst, int nb) {
  for (int q = threadIdx.x; q < nb * nb; q += FT) {
    int i = q / nb, j = q % nb;
    int jm = md(j - 1, nb), jp = md(j + 1, nb);
    // B[jm][j] = super_{jm}, B[j][j] = diag_j, B[jp][j] = sub_{jp}
    dst[i * NBT + j] = D[i * NBT + j] * band[nb + j] + D[i * NBT + jm] * band[2 * nb + jm] +
                       D[i * NBT + jp] * band[jp];
  }
}

// dst = B * D (band x dense)
template <int NBT>
__device__ void band_dense(const double* band, const double* D, double* dst, int nb) {
  for (int q = threadIdx.x; q < nb * nb; q += FT) {
    int i = q / nb, j = q % nb;
    dst[i * NBT + j] = band[i] * D[md(i - 1, nb) * NBT + j] + band[nb + i] * D[i * NBT + j] +
                       band[2 * nb + i] * D[md(i + 1, nb) * NBT + j];
  }
}

// dst = X * Y (dense x dense)
template <int NBT>
__device__ void dense_dense(const double* X, const double* Y, double* dst, int nb) {
  for (int q = threadIdx.x; q < nb * nb; q += FT) {
    int i = q / nb, j = q % nb;
    double v = 0.0;
    for (int k = 0; k < nb; ++k) v += X[i * NBT + k] * Y[k * NBT + j];
    dst[i * NBT + j] = v;
  }
}

// inv = M^-1 by Gauss-Jordan with partial pivoting (M untouched).
template <int NBT>
__device__ void invert(Lds<NBT>& L, const double* M, double* inv, int nb) {
  const int W2 = 2 * NBT;
  for (int q = threadIdx.x; q < nb * 2 * nb; q += FT) {
    int i = q / (2 * nb), j = q % (2 * nb);
    L.W[i * W2 + j] = (j < nb) ? M[i * NBT + j] : (j - nb == i ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int col = 0; col < nb; ++col) {
    if (threadIdx.x == 0) {
      int p = col;
      double best = fabs(L.W[col * W2 + col]);
      for (int r = col + 1; r < nb; ++r) {
        double v = fabs(L.W[r * W2 + col]);
        if (v > best) { best = v; p = r; }
      }
      L.piv = p;
      if (!(best > 1e-300) || !isfinite(best)) L.bad = 1;
    }
    __syncthreads();
    int p = L.piv;
    if (p != col) {
      for (int j = threadIdx.x; j < 2 * nb; j += FT) {
        double t = L.W[col * W2 + j];
        L.W[col * W2 + j] = L.W[p * W2 + j];
        L.W[p * W2 + j] = t;
      }
    }
    __syncthreads();
    double f = 1.0 / L.W[col * W2 + col];
    __syncthreads();
    for (int j = threadIdx.x; j < 2 * nb; j += FT) L.W[col * W2 + j] *= f;
    __syncthreads();
    for (int r = threadIdx.x; r < nb; r += FT) L.fac[r] = L.W[r * W2 + col];
    __syncthreads();
    for (int q = threadIdx.x; q < nb * 2 * nb; q += FT) {
      int r = q / (2 * nb), j = q % (2 * nb);
      if (r != col) L.W[r * W2 + j] -= L.fac[r] * L.W[col * W2 + j];
    }
    __syncthreads();
  }
  for (int q = threadIdx.x; q < nb * nb; q += FT) {
    int i = q / nb, j = q % nb;
    inv[i * NBT + j] = L.W[i * W2 + nb + j];
  }
  __syncthreads();
}

template <int NBT>
__device__ void store_dense(const double* D, double* dst, int nb) {
  for (int q = threadIdx.x; q < nb * nb; q += FT) dst[q] = D[(q / nb) * NBT + (q % nb)];
}

template <int NBT, int SCH>
__device__ void load_rows(const ElemCtx& c, Lds<NBT>& L, int slot, int which, int r) {
  for (int q = threadIdx.x; q < 3 * c.nb; q += FT) L.band[slot][q] = row_band<SCH>(c, which, r, q / c.nb, q % c.nb);
}

// Per-segment geometric weights alpha[tau][seg][end][ab] of eq. Es for the
// element's nb segments, into alpha (LDS) and, if given, the gradient's copy
// gbasis: two-point Gauss-Legendre (exact for the cubic integrands) of
// c^2 det J_b (b1.b1 N N, b2.b1 dN N, b2.b2 dN dN) and det J_b N N, times the
// end-node shape function.
__device__ void segment_weights(const MeshDev& mm, int e, double c, double* alpha, double* gbasis) {
  const int nb = mm.nb[e];
  const int64_t lo = mm.loop_off[e];
  const double cx = mm.centre[2 * e], cy = mm.centre[2 * e + 1];
  for (int s = threadIdx.x; s < nb; s += FT) {
    int s1 = md(s + 1, nb);
    double ax = mm.loop_xy[2 * (lo + s)], ay = mm.loop_xy[2 * (lo + s) + 1];
    double bx = mm.loop_xy[2 * (lo + s1)], by = mm.loop_xy[2 * (lo + s1) + 1];
    double dx = 0.5 * (bx - ax), dy = 0.5 * (by - ay);
    double acc[32];
    for (int q = 0; q < 32; ++q) acc[q] = 0.0;
    const double gp = 0.57735026918962576451;  // 1/sqrt(3), weights 1
    for (int g = 0; g < 2; ++g) {
      double eta = g == 0 ? -gp : gp;
      double N[2] = {0.5 * (1.0 - eta), 0.5 * (1.0 + eta)};
      double dN[2] = {-0.5, 0.5};
      double xb = N[0] * ax + N[1] * bx - cx, yb = N[0] * ay + N[1] * by - cy;
      double det = xb * dy - yb * dx;
      double b1x = dy / det, b1y = -dx / det;
      double b2x = -yb / det, b2y = xb / det;
      double b11 = b1x * b1x + b1y * b1y, b21 = b2x * b1x + b2y * b1y, b22 = b2x * b2x + b2y * b2y;
      for (int end = 0; end < 2; ++end) {
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) {
            int ab = a * 2 + b;
            double wN = det * N[end];
            acc[0 * 8 + end * 4 + ab] += c * c * b11 * wN * N[a] * N[b];
            acc[1 * 8 + end * 4 + ab] += c * c * b21 * wN * dN[a] * N[b];
            acc[2 * 8 + end * 4 + ab] += c * c * b22 * wN * dN[a] * dN[b];
            acc[3 * 8 + end * 4 + ab] += wN * N[a] * N[b];
          }
      }
    }
    for (int tau = 0; tau < 4; ++tau)
      for (int q = 0; q < 8; ++q) {
        alpha[tau * nb * 8 + s * 8 + q] = acc[tau * 8 + q];
        if (gbasis) gbasis[32 * (lo + s) + tau * 8 + q] = acc[tau * 8 + q];
      }
  }
}

// SCH: the radial scheme, fixed at compile time so that each instance keeps
// only its own row builder.
template <int NBT, int SCH>
__global__ void __launch_bounds__(FT) factor_kernel(
    const int32_t* __restrict__ elems, const MeshDev mm, const double* __restrict__ rho,
    double c, double a0, FactorsDev ff, int* status) {
  __shared__ Lds<NBT> L;
  const int e = elems[blockIdx.x];
  const int nb = mm.nb[e];
  const int nr = mm.nr[e];
  const int n = nr - 1;
  const int64_t lo = mm.loop_off[e];
  if (threadIdx.x == 0) L.bad = 0;
  // per-segment geometric weights alpha[tau][seg][end][ab]
  segment_weights(mm, e, c, L.alpha, ff.gbasis);
  __syncthreads();
  ElemCtx ec;
  ec.nb = nb;
  ec.n = n;
  ec.xi0 = mm.xi0;
  ec.h = (1.0 - mm.xi0) / n;
  ec.c2 = c * c;
  ec.lfe = SCH == SBFWI_SCHEME_LFE_CONDENSED;
  ec.a0 = ec.lfe ? 0.0 : a0;   // the condensed expansion's K is the static condensation
  ec.rho = rho + mm.par_off[e];
  ec.alpha = L.alpha;
  ec.scheme = SCH;
  ec.rgw = SCH != SBFWI_SCHEME_PAPER_FD ? ff.rgw + ff.rgw_off[nr] : nullptr;
  const int64_t po = mm.par_off[e];
  // central differences: kappa of every band entry, for the sweeps that form theta_j,
  // psi_j, P_j on the fly, at ((loop slot) * 3 + t) * kFdKappa
  if constexpr (SCH == SBFWI_SCHEME_PAPER_FD) {
    auto al = [&](int tau, int seg, int end, int ab) { return L.alpha[tau * nb * 8 + seg * 8 + end * 4 + ab]; };
    for (int q = threadIdx.x; q < 3 * nb; q += FT) {
      const int t = q / nb, i = q % nb;
      fd_kappa(al, nb, t, i, ff.bkap + ((lo + i) * 3 + t) * kFdKappa);
    }
  }
  // persistent bands: theta_j, psi_j, P_j for j = 0..n; theta_{n+1}, phi_{-1}, psi_{-1}
  for (int q = threadIdx.x; q < 3 * nb * nr; q += FT) {
    int j = q / (3 * nb), rem = q % (3 * nb), t = rem / nb, i = rem % nb;
    ff.th_band[3 * po + j * 3 * nb + rem] = row_band<SCH>(ec, 0, j, t, i);
    ff.ps_band[3 * po + j * 3 * nb + rem] = row_band<SCH>(ec, 2, j, t, i);
    ff.pm_band[3 * po + j * 3 * nb + rem] = row_band<SCH>(ec, 3, j, t, i);
  }
  for (int q = threadIdx.x; q < 3 * nb; q += FT) {
    ff.th_np1[3 * lo + q] = row_band<SCH>(ec, 0, n + 1, q / nb, q % nb);
    ff.phim1[3 * lo + q] = row_band<SCH>(ec, 1, -1, q / nb, q % nb);
    ff.psim1[3 * lo + q] = row_band<SCH>(ec, 2, -1, q / nb, q % nb);
  }
  const int64_t dofs = mm.dense_off[e];
  const int64_t fo = mm.finv_off[e];
  // theta_{-1}^-1
  load_rows<NBT, SCH>(ec, L, 0, 0, -1);
  __syncthreads();
  band_to_dense<NBT>(L.band[0], L.A, nb);
  __syncthreads();
  invert<NBT>(L, L.A, L.B, nb);                 // B = theta_{-1}^-1
  store_dense<NBT>(L.B, ff.thm1_inv + dofs, nb);
  // rho_0 = theta_0 theta_{-1}^-1 ; phi~_0 = phi_0 - rho_0 phi_{-1} ; psi~_0 = psi_0 - rho_0 psi_{-1}
  load_rows<NBT, SCH>(ec, L, 0, 0, 0);   // theta_0
  load_rows<NBT, SCH>(ec, L, 1, 1, -1);  // phi_{-1}
  load_rows<NBT, SCH>(ec, L, 2, 2, -1);  // psi_{-1}
  __syncthreads();
  band_dense<NBT>(L.band[0], L.B, L.Z, nb);     // Z = rho_0
  __syncthreads();
  dense_band<NBT>(L.Z, L.band[1], L.A, nb);     // A = rho_0 phi_{-1}
  dense_band<NBT>(L.Z, L.band[2], L.B, nb);     // B = rho_0 psi_{-1}
  __syncthreads();
  load_rows<NBT, SCH>(ec, L, 0, 1, 0);   // phi_0
  load_rows<NBT, SCH>(ec, L, 1, 2, 0);   // psi_0
  __syncthreads();
  band_to_dense<NBT>(L.band[0], L.Ph, nb);
  band_to_dense<NBT>(L.band[1], L.Pp, nb);
  __syncthreads();
  for (int q = threadIdx.x; q < nb * nb; q += FT) {
    int i = q / nb, j = q % nb;
    L.Ph[i * NBT + j] -= L.A[i * NBT + j];      // phi~_0
    L.Pp[i * NBT + j] -= L.B[i * NBT + j];      // psi~_0
  }
  __syncthreads();
  store_dense<NBT>(L.Pp, ff.psit0 + dofs, nb);
  invert<NBT>(L, L.Ph, L.Fp, nb);               // Fp = phi~_0^-1
  store_dense<NBT>(L.Fp, ff.finv + fo, nb);
  // levels j = 1 .. n
  for (int j = 1; j <= n; ++j) {
    // Z = phi~_{j-1}^-1 psi~_{j-1}
    if (j == 1) {
      dense_dense<NBT>(L.Fp, L.Pp, L.Z, nb);
    } else {
      load_rows<NBT, SCH>(ec, L, 2, 2, j - 1);
      __syncthreads();
      dense_band<NBT>(L.Fp, L.band[2], L.Z, nb);
    }
    load_rows<NBT, SCH>(ec, L, 0, 0, j);   // theta_j
    load_rows<NBT, SCH>(ec, L, 1, 1, j);   // phi_j
    __syncthreads();
    band_dense<NBT>(L.band[0], L.Z, L.A, nb);   // A = theta_j Z
    band_to_dense<NBT>(L.band[1], L.Ph, nb);
    __syncthreads();
    for (int q = threadIdx.x; q < nb * nb; q += FT) {
      int i = q / nb, jj = q % nb;
      L.Ph[i * NBT + jj] -= L.A[i * NBT + jj];  // phi~_j
    }
    __syncthreads();
    if (j == n) {
      load_rows<NBT, SCH>(ec, L, 0, 0, n + 1);
      load_rows<NBT, SCH>(ec, L, 1, 1, n + 1);
      __syncthreads();
      band_dense<NBT>(L.band[0], L.Z, L.A, nb);
      band_to_dense<NBT>(L.band[1], L.Ph1, nb);
      __syncthreads();
      for (int q = threadIdx.x; q < nb * nb; q += FT) {
        int i = q / nb, jj = q % nb;
        L.Ph1[i * NBT + jj] -= L.A[i * NBT + jj];   // phi~_{n+1}
      }
      __syncthreads();
    } else {
      invert<NBT>(L, L.Ph, L.Fp, nb);
      store_dense<NBT>(L.Fp, ff.finv + fo + (int64_t)j * nb * nb, nb);
    }
  }
  store_dense<NBT>(L.Ph, ff.phit_n + dofs, nb);
  // G = psi_{n+1} psi_n^-1 ; S = phi~_{n+1} - G phi~_n
  load_rows<NBT, SCH>(ec, L, 0, 2, n);       // psi_n
  load_rows<NBT, SCH>(ec, L, 1, 2, n + 1);   // psi_{n+1}
  __syncthreads();
  band_to_dense<NBT>(L.band[0], L.A, nb);
  __syncthreads();
  invert<NBT>(L, L.A, L.B, nb);         // B = psi_n^-1
  store_dense<NBT>(L.B, ff.psin_inv + dofs, nb);
  band_dense<NBT>(L.band[1], L.B, L.Z, nb);   // Z = G
  __syncthreads();
  store_dense<NBT>(L.Z, ff.G + dofs, nb);
  dense_dense<NBT>(L.Z, L.Ph, L.A, nb);       // A = G phi~_n
  __syncthreads();
  for (int q = threadIdx.x; q < nb * nb; q += FT) {
    int i = q / nb, jj = q % nb;
    ff.S[dofs + q] = L.Ph1[i * NBT + jj] - L.A[i * NBT + jj];
  }
  if (ec.lfe) {
    // M = sum_i Phi_i^T M_i Phi_i over the static modes Phi_n = I,
    // Phi_i = -phi~_i^-1 psi_i Phi_{i+1}; M_i = -P_i inside, M_n = P_n
    __syncthreads();
    load_rows<NBT, SCH>(ec, L, 0, 3, n);
    __syncthreads();
    band_to_dense<NBT>(L.band[0], L.Ph1, nb);     // Ph1 = M accumulator
    for (int q = threadIdx.x; q < nb * nb; q += FT) {
      int i = q / nb, jj = q % nb;
      L.Ph[i * NBT + jj] = i == jj ? 1.0 : 0.0;   // Ph = Phi
    }
    __syncthreads();
    for (int j = n - 1; j >= 0; --j) {
      load_rows<NBT, SCH>(ec, L, 1, 2, j);             // psi_j
      load_rows<NBT, SCH>(ec, L, 2, 3, j);             // P_j
      for (int q = threadIdx.x; q < nb * nb; q += FT)
        L.Fp[(q / nb) * NBT + (q % nb)] = ff.finv[fo + (int64_t)j * nb * nb + q];
      __syncthreads();
      band_dense<NBT>(L.band[1], L.Ph, L.Z, nb);  // Z = psi_j Phi_{j+1}
      __syncthreads();
      dense_dense<NBT>(L.Fp, L.Z, L.A, nb);       // A = phi~_j^-1 Z = -Phi_j
      __syncthreads();
      for (int q = threadIdx.x; q < nb * nb; q += FT) {
        int i = q / nb, jj = q % nb;
        L.Ph[i * NBT + jj] = -L.A[i * NBT + jj];
      }
      __syncthreads();
      band_dense<NBT>(L.band[2], L.Ph, L.B, nb);  // B = P_j Phi_j = -M_j Phi_j
      __syncthreads();
      for (int q = threadIdx.x; q < nb * nb; q += FT) {
        int i = q / nb, jj = q % nb;
        double v = 0.0;
        for (int k = 0; k < nb; ++k) v += L.Ph[k * NBT + i] * L.B[k * NBT + jj];
        L.Ph1[i * NBT + jj] -= v;
      }
      __syncthreads();
    }
    store_dense<NBT>(L.Ph1, ff.Me + dofs, nb);
  }
  if (threadIdx.x == 0 && L.bad) atomicOr(status, 1);
}

__global__ void assemble_kernel(int64_t nnz, const int64_t* __restrict__ cptr,
                                const int64_t* __restrict__ csrc, const double* __restrict__ S,
                                double* __restrict__ K) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nnz) return;
  double v = 0.0;
  for (int64_t t = cptr[q]; t < cptr[q + 1]; ++t) v += S[csrc[t]];
  K[q] = v;
}

// Low-frequency expansion: K_g + a0 M_g (the Newmark system matrix) and M_g.
__global__ void assemble_lfe_kernel(int64_t nnz, const int64_t* __restrict__ cptr,
                                    const int64_t* __restrict__ csrc, const double* __restrict__ S,
                                    const double* __restrict__ Me, double a0, double* __restrict__ K,
                                    double* __restrict__ M) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nnz) return;
  double k = 0.0, m = 0.0;
  for (int64_t t = cptr[q]; t < cptr[q + 1]; ++t) {
    k += S[csrc[t]];
    m += Me[csrc[t]];
  }
  K[q] = k + a0 * m;
  M[q] = m;
}

// ---------------------------------------------------------------------------
// Low-frequency expansion (scheme 2, Section "Low-frequency expansion", eq. S):
// per element, with the boundary level's densities at every level, K solves
// the algebraic Riccati equation (K - E1) E0^-1 (K - E1^T) = E2 and M the
// Lyapunov equation A M + M A^T = M0, A = (K - E1) E0^-1 + I.
//
// K: the graph {[u; K u]} is the invariant subspace of the static radial
// matrix Z = [[-E0^-1 E1^T, E0^-1], [E2 - E1 E0^-1 E1^T, E1 E0^-1]] that
// belongs to its eigenvalues with positive real part (the modes bounded at the
// scaling centre) together with the constant mode [1; 0] (eigenvalue 0, whose
// partner completes a Jordan pair).  The linear fields are modes of eigenvalue
// 1, so the other positive eigenvalues are >= 1 and the shift Z - I/2 separates
// them from 0 and the negative ones.  Its matrix sign function, by the
// determinant-scaled Newton iteration X <- (mu X + (mu X)^-1) / 2, gives the
// spectral projector P = (I + sign(Z - I/2)) / 2 onto the positive modes;
// every column of P lies in the graph, [P11 P12] -> [P21 P22], and K 1 = 0, so
// K = (P21 P11^T + P22 P12^T) (P11 P11^T + P12 P12^T + s 1 1^T)^-1 (any s > 0;
// s = trace(P11 P11^T + P12 P12^T) / nb keeps the scales alike).
// M: the eigenvalues of A are 1 + (those of the modes) >= 1, so sign(A) = I
// and the Newton iteration on [[A, C], [0, -A^T]] -- A <- (mu A + (mu A)^-1)/2,
// C <- (mu C + A^-1 C A^-T / mu)/2 from C = M0 -- converges to C = 2 M.
// ---------------------------------------------------------------------------

template <int NBT>
struct RicLds {
  double alpha[4 * NBT * 8];
  double E0i[NBT * NBT];        // E0^-1 (compact, leading dimension nb)
  double E1[NBT * NBT];
  double M0[NBT * NBT];
  double R0[4 * NBT * NBT];     // sign iterate S (2nb x 2nb), later K, A, C, T
  double R1[4 * NBT * NBT];     // its inverse, later the nb x nb work blocks
  double fac[2 * NBT];
  double red[2 * FT];
  int perm[2 * NBT];
  int piv;
  int bad;
  double logdet;
};

// In-place Gauss-Jordan inversion with partial pivoting of the N x N matrix X
// (leading dimension N) in LDS; *logdet receives log |det X|, *bad is set on a
// zero or non-finite pivot.
template <int NBT>
__device__ void gj_invert(RicLds<NBT>& L, double* X, int N) {
  if (threadIdx.x == 0) L.logdet = 0.0;
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    if (threadIdx.x == 0) {
      int p = k;
      double best = fabs(X[k * N + k]);
      for (int r = k + 1; r < N; ++r) {
        const double v = fabs(X[r * N + k]);
        if (v > best) { best = v; p = r; }
      }
      L.piv = p;
      L.perm[k] = p;
      if (!(best > 1e-300) || !isfinite(best)) L.bad = 1;
      L.logdet += log(best > 1e-300 ? best : 1e-300);
    }
    __syncthreads();
    const int p = L.piv;
    if (p != k)
      for (int j = threadIdx.x; j < N; j += FT) {
        const double t = X[k * N + j];
        X[k * N + j] = X[p * N + j];
        X[p * N + j] = t;
      }
    __syncthreads();
    const double pv = X[k * N + k];
    __syncthreads();
    for (int j = threadIdx.x; j < N; j += FT) X[k * N + j] = (j == k ? 1.0 : X[k * N + j]) / pv;
    for (int i = threadIdx.x; i < N; i += FT) L.fac[i] = i == k ? 0.0 : X[i * N + k];
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += FT)
      if (i != k) X[i * N + k] = 0.0;
    __syncthreads();
    for (int q = threadIdx.x; q < N * N; q += FT) {
      const int i = q / N, j = q % N;
      if (i != k) X[q] -= L.fac[i] * X[k * N + j];
    }
    __syncthreads();
  }
  for (int k = N - 1; k >= 0; --k) {   // undo the row interchanges on the columns of the inverse
    const int p = L.perm[k];
    if (p != k)
      for (int i = threadIdx.x; i < N; i += FT) {
        const double t = X[i * N + k];
        X[i * N + k] = X[i * N + p];
        X[i * N + p] = t;
      }
    __syncthreads();
  }
}

// Largest |x| over the block's partial values (thread t holds a[t], b[t]).
template <int NBT>
__device__ void block_max2(RicLds<NBT>& L, double a, double b, double* ra, double* rb) {
  L.red[threadIdx.x] = a;
  L.red[FT + threadIdx.x] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = 0.0, y = 0.0;
    for (int t = 0; t < FT; ++t) {
      x = fmax(x, L.red[t]);
      y = fmax(y, L.red[FT + t]);
    }
    L.red[0] = x;
    L.red[FT] = y;
  }
  __syncthreads();
  *ra = L.red[0];
  *rb = L.red[FT];
  __syncthreads();
}

constexpr int kSignMaxIter = 60;

// One scaled Newton step of the sign iteration on the N x N iterate X (its
// inverse computed in Xi); returns the largest change and the largest entry.
template <int NBT>
__device__ void sign_step(RicLds<NBT>& L, double* X, double* Xi, int N, bool scale, double* change, double* norm) {
  for (int q = threadIdx.x; q < N * N; q += FT) Xi[q] = X[q];
  __syncthreads();
  gj_invert<NBT>(L, Xi, N);
  const double mu = scale ? exp(-L.logdet / N) : 1.0;
  double ch = 0.0, nm = 0.0;
  for (int q = threadIdx.x; q < N * N; q += FT) {
    const double v = 0.5 * (mu * X[q] + Xi[q] / mu);
    ch = fmax(ch, fabs(v - X[q]));
    nm = fmax(nm, fabs(v));
    X[q] = v;
  }
  block_max2<NBT>(L, ch, nm, change, norm);
}

template <int NBT>
__global__ void __launch_bounds__(FT) lfe_riccati_kernel(const int32_t* __restrict__ elems, const MeshDev mm,
                                                         const double* __restrict__ rho, double c, FactorsDev ff,
                                                         int* status) {
  __shared__ RicLds<NBT> L;
  const int e = elems[blockIdx.x];
  const int nb = mm.nb[e];
  const int n = mm.nr[e] - 1;
  const int nn = nb * nb;
  if (threadIdx.x == 0) L.bad = 0;
  segment_weights(mm, e, c, L.alpha, nullptr);
  __syncthreads();
  ElemCtx ec;
  ec.nb = nb;
  ec.n = n;
  ec.xi0 = mm.xi0;
  ec.h = (1.0 - mm.xi0) / n;
  ec.c2 = c * c;
  ec.lfe = 1;   // radially constant: the boundary level's densities
  ec.a0 = 0.0;
  ec.rho = rho + mm.par_off[e];
  ec.alpha = L.alpha;
  ec.scheme = SBFWI_SCHEME_LFE;
  ec.rgw = nullptr;
  // dense E0 (into R1, then inverted in place), E1, E2 (R1 + nn), M0
  auto dense_e = [&](int tau, double* dst) {
    for (int q = threadIdx.x; q < nn; q += FT) {
      const int i = q / nb, j = q % nb;
      double v = j == i ? e_band(ec, tau, n, 1, i) : 0.0;
      if (j == md(i + 1, nb)) v += e_band(ec, tau, n, 2, i);
      if (j == md(i - 1, nb)) v += e_band(ec, tau, n, 0, i);
      dst[q] = v;
    }
  };
  double* E2 = L.R1 + nn;
  dense_e(0, L.R1);
  dense_e(1, L.E1);
  dense_e(2, E2);
  dense_e(3, L.M0);
  __syncthreads();
  gj_invert<NBT>(L, L.R1, nb);
  for (int q = threadIdx.x; q < nn; q += FT) L.E0i[q] = L.R1[q];
  __syncthreads();
  // S = Z - I/2 (2nb x 2nb); blocks: Z11 = -E0^-1 E1^T, Z12 = E0^-1,
  // Z21 = E2 - E1 E0^-1 E1^T = E2 + E1 Z11, Z22 = E1 E0^-1
  const int N = 2 * nb;
  double* S = L.R0;
  for (int q = threadIdx.x; q < nn; q += FT) {
    const int i = q / nb, j = q % nb;
    double z11 = 0.0, z22 = 0.0;
    for (int k = 0; k < nb; ++k) {
      z11 -= L.E0i[i * nb + k] * L.E1[j * nb + k];
      z22 += L.E1[i * nb + k] * L.E0i[k * nb + j];
    }
    S[i * N + j] = z11 - (i == j ? 0.5 : 0.0);
    S[i * N + nb + j] = L.E0i[q];
    S[(nb + i) * N + nb + j] = z22 - (i == j ? 0.5 : 0.0);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nn; q += FT) {
    const int i = q / nb, j = q % nb;
    double v = E2[q];
    for (int k = 0; k < nb; ++k) v += L.E1[i * nb + k] * S[k * N + j];   // S11 = Z11 - I/2
    S[(nb + i) * N + j] = v + 0.5 * L.E1[i * nb + j];                      // E1 (S11 + I/2) = E1 Z11
  }
  __syncthreads();
  // sign(Z - I/2): scaled until the iterate settles, then plain Newton steps;
  // one more step after the change first falls below the tolerance
  bool done = false;
  int it = 0, extra = 0;
  bool scale = true;
  for (; it < kSignMaxIter && !done; ++it) {
    double ch, nm;
    sign_step<NBT>(L, S, L.R1, N, scale, &ch, &nm);
    if (ch <= 1e-2 * nm) scale = false;
    if (ch <= 1e-14 * nm) done = ++extra > 1;
  }
  if (!done && threadIdx.x == 0) atomicOr(status, 2);
  // P = (I + S) / 2; A = P11 P11^T + P12 P12^T + s 1 1^T (R1), Rm = P21 P11^T + P22 P12^T (R1 + nn)
  for (int q = threadIdx.x; q < N * N; q += FT) S[q] = 0.5 * (S[q] + ((q / N) == (q % N) ? 1.0 : 0.0));
  __syncthreads();
  double* A = L.R1;
  double* Rm = L.R1 + nn;
  double tr = 0.0;
  for (int q = threadIdx.x; q < nn; q += FT) {
    const int i = q / nb, j = q % nb;
    double a = 0.0, r = 0.0;
    for (int k = 0; k < N; ++k) {
      a += S[i * N + k] * S[j * N + k];
      r += S[(nb + i) * N + k] * S[j * N + k];
    }
    A[q] = a;
    Rm[q] = r;
    if (i == j) tr += a;
  }
  double trace, unused;
  {
    L.red[threadIdx.x] = tr;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int k = 0; k < FT; ++k) t += L.red[k];
      L.red[0] = t;
    }
    __syncthreads();
    trace = L.red[0];
    unused = 0.0;
    __syncthreads();
  }
  (void)unused;
  for (int q = threadIdx.x; q < nn; q += FT) A[q] += trace / nb;
  __syncthreads();
  gj_invert<NBT>(L, A, nb);
  // K = Rm A^-1 (R0 slot 0); Al = (K - E1) E0^-1 + I (slot 1); C = M0 (slot 2)
  double* K = L.R0;
  double* Al = L.R0 + nn;
  double* C = L.R0 + 2 * nn;
  double* T = L.R0 + 3 * nn;
  for (int q = threadIdx.x; q < nn; q += FT) {
    const int i = q / nb, j = q % nb;
    double v = 0.0;
    for (int k = 0; k < nb; ++k) v += Rm[i * nb + k] * A[k * nb + j];
    T[q] = v;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nn; q += FT) K[q] = T[q];
  __syncthreads();
  for (int q = threadIdx.x; q < nn; q += FT) {
    const int i = q / nb, j = q % nb;
    double v = i == j ? 1.0 : 0.0;
    for (int k = 0; k < nb; ++k) v += (K[i * nb + k] - L.E1[i * nb + k]) * L.E0i[k * nb + j];
    Al[q] = v;
    C[q] = L.M0[q];
  }
  __syncthreads();
  // Lyapunov by the Newton iteration on [[Al, C], [0, -Al^T]]
  double* X = L.R1;
  done = false;
  extra = 0;
  scale = true;
  for (it = 0; it < kSignMaxIter && !done; ++it) {
    for (int q = threadIdx.x; q < nn; q += FT) X[q] = Al[q];
    __syncthreads();
    gj_invert<NBT>(L, X, nb);
    const double mu = scale ? exp(-L.logdet / nb) : 1.0;
    for (int q = threadIdx.x; q < nn; q += FT) {   // T = X C
      const int i = q / nb, j = q % nb;
      double v = 0.0;
      for (int k = 0; k < nb; ++k) v += X[i * nb + k] * C[k * nb + j];
      T[q] = v;
    }
    __syncthreads();
    double ch = 0.0, nm = 0.0;
    for (int q = threadIdx.x; q < nn; q += FT) {
      const int i = q / nb, j = q % nb;
      double v = 0.0;
      for (int k = 0; k < nb; ++k) v += T[i * nb + k] * X[j * nb + k];   // X C X^T
      C[q] = 0.5 * (mu * C[q] + v / mu);
      const double a = 0.5 * (mu * Al[q] + X[q] / mu);
      ch = fmax(ch, fabs(a - Al[q]));
      nm = fmax(nm, fabs(a));
      Al[q] = a;
    }
    double chg, nrm;
    block_max2<NBT>(L, ch, nm, &chg, &nrm);
    if (chg <= 1e-2 * nrm) scale = false;
    if (chg <= 1e-14 * nrm) done = ++extra > 1;
  }
  if (!done && threadIdx.x == 0) atomicOr(status, 2);
  const int64_t dofs = mm.dense_off[e];
  for (int q = threadIdx.x; q < nn; q += FT) {
    ff.S[dofs + q] = K[q];
    ff.Me[dofs + q] = 0.5 * C[q];
  }
  if (threadIdx.x == 0 && L.bad) atomicOr(status, 1);
}

__global__ void transpose_diag_kernel(int64_t nnz, int64_t n_nodes, const int64_t* __restrict__ tr,
                                      const int64_t* __restrict__ diag, const int64_t* __restrict__ ell_pos,
                                      const double* __restrict__ K, double* __restrict__ KT,
                                      double* __restrict__ Kell, double* __restrict__ KTell,
                                      double* __restrict__ dinv) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nnz) {
    double kt = K[tr[q]];
    KT[q] = kt;
    Kell[ell_pos[q]] = K[q];
    KTell[ell_pos[q]] = kt;
  }
  if (q < n_nodes) dinv[q] = 1.0 / K[diag[q]];
}

}  // namespace

void sbfwi_factors_free(sbfwi_factors_s* f) {
  if (!f) return;
  FactorsDev& d = f->d;
  void* ptrs[] = {d.finv, d.th_band, d.ps_band, d.pm_band, d.th_np1, d.phim1, d.psim1, d.bkap, d.rho,
                  d.G, d.S, d.psit0, d.psin_inv, d.phit_n, d.thm1_inv, d.gbasis,
                  d.Kval, d.KTval, d.Kell, d.KTell, d.diag_inv, d.status, d.rgw, d.Me, d.Mval};
  sbfwi_dev_free(d.rgw_off);
  for (void* p : ptrs) sbfwi_dev_free(p);
  sbfwi_direct_num_free(f->dnum);
  delete f;
}

void sbfwi_rg_weights(double xi0, const std::vector<int>& level_counts, std::vector<double>& w,
                      std::vector<int>& off) {
  // Gauss-Legendre nodes and weights on [-1, 1], 4 points
  const double gx[4] = {-0.86113631159405257522, -0.33998104358485626480, 0.33998104358485626480,
                        0.86113631159405257522};
  const double gw[4] = {0.34785484513745385737, 0.65214515486254614263, 0.65214515486254614263,
                        0.34785484513745385737};
  off.assign(129, -1);
  w.clear();
  for (int nr : level_counts) {
    if (nr < 2 || nr > 128 || off[nr] >= 0) continue;
    off[nr] = (int)w.size();
    const int n = nr - 1;
    const double h = (1.0 - xi0) / n;
    for (int j = 0; j < n; ++j) {
      const double a = xi0 + h * j, b = a + h;
      double iv[kRgW] = {};
      for (int g = 0; g < 4; ++g) {
        const double x = 0.5 * (a + b) + 0.5 * (b - a) * gx[g], ww = 0.5 * (b - a) * gw[g];
        const double N[2] = {(b - x) / (b - a), (x - a) / (b - a)};
        const double dN[2] = {-1.0 / (b - a), 1.0 / (b - a)};
        for (int p = 0; p < 2; ++p) {
          for (int q = 0; q < 2; ++q)
            for (int e = 0; e < 2; ++e) {
              const int o = 4 * p + 2 * q + e;
              iv[o] += ww * x * dN[p] * dN[q] * N[e];
              iv[8 + o] += ww * dN[p] * N[q] * N[e];
              iv[16 + o] += ww * N[p] * dN[q] * N[e];
              iv[24 + o] += ww * N[p] * N[q] * N[e] / x;
            }
          for (int e = 0; e < 2; ++e) iv[32 + 2 * p + e] += ww * x * N[p] * N[e];
        }
      }
      w.insert(w.end(), iv, iv + kRgW);
    }
  }
}

template <int NBT>
static void launch_factor_nb(int scheme, dim3 grid, dim3 block, hipStream_t s, const int32_t* elems, const MeshDev& md,
                             const double* rho, double c, const FactorsDev& d) {
  if (scheme == SBFWI_SCHEME_RADIAL_GALERKIN)
    hipLaunchKernelGGL((factor_kernel<NBT, SBFWI_SCHEME_RADIAL_GALERKIN>), grid, block, 0, s, elems, md, rho, c, d.a0,
                       d, d.status);
  else if (scheme == SBFWI_SCHEME_LFE)
    hipLaunchKernelGGL((lfe_riccati_kernel<NBT>), grid, block, 0, s, elems, md, rho, c, d, d.status);
  else if (scheme == SBFWI_SCHEME_LFE_CONDENSED)
    hipLaunchKernelGGL((factor_kernel<NBT, SBFWI_SCHEME_LFE_CONDENSED>), grid, block, 0, s, elems, md, rho, c, d.a0,
                       d, d.status);
  else
    hipLaunchKernelGGL((factor_kernel<NBT, SBFWI_SCHEME_PAPER_FD>), grid, block, 0, s, elems, md, rho, c, d.a0, d,
                       d.status);
}

static void launch_factor(int cl, int scheme, dim3 grid, dim3 block, hipStream_t s, sbfwi_mesh_s* m,
                          const double* rho, double c, const FactorsDev& d) {
  if (cl == 0) launch_factor_nb<8>(scheme, grid, block, s, m->class_elems[0], m->d, rho, c, d);
  else if (cl == 1) launch_factor_nb<16>(scheme, grid, block, s, m->class_elems[1], m->d, rho, c, d);
  else launch_factor_nb<24>(scheme, grid, block, s, m->class_elems[2], m->d, rho, c, d);
}

int sbfwi_factor_impl(sbfwi_mesh_s* m, const double* rho, double c, double dt, double beta,
                      double gamma, int scheme, int coarse_solver, hipStream_t s, sbfwi_factors_s** out) {
  sbfwi_factors_s* f = new sbfwi_factors_s();
  f->m = m;
  f->c = c;
  f->dt = dt;
  f->beta = beta;
  f->gamma = gamma;
  FactorsDev& d = f->d;
  d.a0 = 1.0 / (beta * dt * dt);
  d.a1 = 1.0 / (beta * dt);
  d.a2 = 1.0 / (2.0 * beta) - 1.0;
  d.c1 = gamma / (beta * dt);
  d.c2 = 1.0 - gamma / beta;
  d.c3 = dt * (1.0 - gamma / (2.0 * beta));
  d.dt = dt;
  d.scheme = scheme;
  f->scheme = scheme;
  int rc = SBFWI_OK;
  auto A = [&](double** p, int64_t n) {
    if (rc == SBFWI_OK) {
      rc = sbfwi_alloc(p, n);
      f->bytes += n * 8;
    }
  };
  A(&d.finv, m->n_finv);
  A(&d.th_band, 3 * m->n_params);
  A(&d.ps_band, 3 * m->n_params);
  A(&d.pm_band, 3 * m->n_params);
  A(&d.th_np1, 3 * m->n_loop);
  A(&d.phim1, 3 * m->n_loop);
  A(&d.psim1, 3 * m->n_loop);
  A(&d.G, m->n_dense);
  A(&d.S, m->n_dense);
  A(&d.psit0, m->n_dense);
  A(&d.psin_inv, m->n_dense);
  A(&d.phit_n, m->n_dense);
  A(&d.thm1_inv, m->n_dense);
  A(&d.gbasis, 32 * m->n_loop);
  if (scheme == SBFWI_SCHEME_PAPER_FD) {   // what the sweeps need to form the rows on the fly
    A(&d.bkap, 3 * kFdKappa * m->n_loop);
    A(&d.rho, m->n_params);
  }
  A(&d.Kval, m->nnz);
  A(&d.KTval, m->nnz);
  A(&d.Kell, m->d.n_ell);
  A(&d.KTell, m->d.n_ell);
  A(&d.diag_inv, m->n_nodes);
  if (rc == SBFWI_OK) rc = sbfwi_alloc(&d.status, 8);
  if (sbfwi_is_lfe(scheme)) {
    A(&d.Me, m->n_dense);
    A(&d.Mval, m->nnz);
  }
  if (rc == SBFWI_OK && scheme != SBFWI_SCHEME_PAPER_FD) {
    std::vector<double> w;
    std::vector<int> off;
    sbfwi_rg_weights(m->xi0, m->h_nr, w, off);
    rc = sbfwi_upload(&d.rgw, w);
    if (rc == SBFWI_OK) rc = sbfwi_upload(&d.rgw_off, off);
    f->bytes += (int64_t)w.size() * 8 + (int64_t)off.size() * 4;
  }
  if (rc != SBFWI_OK) {
    sbfwi_factors_free(f);
    return rc;
  }
  auto hip_fail = [&](hipError_t e, const char* what) {
    sbfwi_factors_free(f);
    return sbfwi_fail(SBFWI_EHIP, "%s: %s", what, hipGetErrorString(e));
  };
  hipError_t he = hipMemsetAsync(d.status, 0, 8 * sizeof(int), s);
  if (he != hipSuccess) return hip_fail(he, "hipMemsetAsync");
  if (d.rho) {
    he = hipMemcpyAsync(d.rho, rho, sizeof(double) * m->n_params, hipMemcpyDeviceToDevice, s);
    if (he != hipSuccess) return hip_fail(he, "density copy");
  }
  {
    ProfScope ps_factor(PK_FACTOR, s);   // the element factorisation kernels
    for (int cl = 0; cl < 3; ++cl) {
      int64_t cnt = (int64_t)m->h_class_elems[cl].size();
      if (cnt == 0) continue;
      dim3 grid((unsigned)cnt), block(FT);
      launch_factor(cl, scheme, grid, block, s, m, rho, c, d);
      he = hipGetLastError();
      if (he != hipSuccess) return hip_fail(he, "factor_kernel launch");
    }
  }
  {
    unsigned g = (unsigned)((m->nnz + 255) / 256);
    if (sbfwi_is_lfe(scheme))
      hipLaunchKernelGGL(assemble_lfe_kernel, dim3(g), dim3(256), 0, s, m->nnz, m->d.contrib_ptr,
                         m->d.contrib_src, d.S, d.Me, d.a0, d.Kval, d.Mval);
    else
      hipLaunchKernelGGL(assemble_kernel, dim3(g), dim3(256), 0, s, m->nnz, m->d.contrib_ptr, m->d.contrib_src,
                         d.S, d.Kval);
    int64_t big = m->nnz > m->n_nodes ? m->nnz : m->n_nodes;
    unsigned g2 = (unsigned)((big + 255) / 256);
    he = hipMemsetAsync(d.Kell, 0, sizeof(double) * m->d.n_ell, s);
    if (he == hipSuccess) he = hipMemsetAsync(d.KTell, 0, sizeof(double) * m->d.n_ell, s);
    if (he != hipSuccess) return hip_fail(he, "hipMemsetAsync");
    hipLaunchKernelGGL(transpose_diag_kernel, dim3(g2), dim3(256), 0, s, m->nnz, m->n_nodes, m->d.tr_idx,
                       m->d.diag_idx, m->d.ell_pos, d.Kval, d.KTval, d.Kell, d.KTell, d.diag_inv);
    he = hipGetLastError();
    if (he != hipSuccess) return hip_fail(he, "assembly launch");
  }
  int st[4] = {0, 0, 0, 0};
  he = hipMemcpyAsync(st, d.status, sizeof(st), hipMemcpyDeviceToHost, s);
  if (he != hipSuccess) return hip_fail(he, "hipMemcpyAsync");
  he = hipStreamSynchronize(s);
  if (he != hipSuccess) return hip_fail(he, "hipStreamSynchronize");
  if (st[0] & 1) {
    sbfwi_factors_free(f);
    return sbfwi_fail(SBFWI_ESINGULAR, "a pivot block of the condensation sweep is singular");
  }
  if (st[0] & 2) {
    sbfwi_factors_free(f);
    return sbfwi_fail(SBFWI_ENOCONV, "the expansion's sign or Lyapunov iteration did not settle");
  }
  {   // response scale of the growth envelope: the largest 1 / |K_g,ii|
    std::vector<double> di(m->n_nodes);
    rc = sbfwi_copy_sync(di.data(), d.diag_inv, sizeof(double) * m->n_nodes, hipMemcpyDeviceToHost);
    if (rc != SBFWI_OK) {
      sbfwi_factors_free(f);
      return rc;
    }
    for (double v : di) f->env_r = std::max(f->env_r, std::fabs(v));
  }
  if (coarse_solver == 1) {
    rc = sbfwi_direct_factor(f, s);
    if (rc != SBFWI_OK) {
      sbfwi_factors_free(f);
      return rc;
    }
  }
  *out = f;
  return SBFWI_OK;
}

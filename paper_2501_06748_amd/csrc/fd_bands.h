// Rows theta_r, psi_r, P_r of the central-difference radial scheme (eq. FD,
// eq. system) evaluated from the nodal densities of the level.
//
// With linear boundary segments and the density interpolated linearly between
// nodal values, entry (t, i) of every cyclic tridiagonal block E^tau_r of
// eq. Es (t = 0: column i-1, 1: column i, 2: column i+1) is a fixed linear
// function of the densities of level r at the nodes i-1, i, i+1:
//   E^tau_r(t, i) = kappa^tau(t, i) . (rho_r[i-1], rho_r[i], rho_r[i+1]).
// The rows of interior level r (xi_r = xi_0 + r h) need E0 at levels r-1, r,
// r+1, the combination E1^T - E1 and M0 at level r:
//   C_r     = E0_r + (E1^T - E1)_r + xi_r dE0/dxi|_r,
//   theta_r = (xi_r / h)^2 E0_r - xi_r / (2 h) C_r,
//   psi_r   = (xi_r / h)^2 E0_r + xi_r / (2 h) C_r,
//   P_r     = -xi_r^2 M0_r,
// with the derivative of E0 by central differences inside and one-sided at
// r = 0 and r = n.  The element factorisation and the sweeps that form these
// rows on the fly evaluate them with the functions below, in the same order
// of operations (and no contraction of their own), so both see the same bits.
#pragma once

#include <hip/hip_runtime.h>

// kappa of one entry (t, i): E0, E1^T - E1 and M0, three coefficients each.
constexpr int kFdKappa = 9;

__host__ __device__ inline int fdb_md(int i, int nb) { return i < 0 ? i + nb : (i >= nb ? i - nb : i); }

// kappa of entry (t, i) from the per-segment weights alpha[tau][seg][end][ab]
// (alpha(tau, seg, end, ab) returns it): the segment block of E^tau is
// sum_end alpha[tau][seg][end][a][b] rho_{seg + end}, ab = 2 a + b.
template <typename Alpha>
__host__ __device__ inline void fd_kappa(const Alpha& alpha, int nb, int t, int i, double* k) {
  const int im = fdb_md(i - 1, nb);
  double E[4][3], ET[3];   // E^tau (tau = 0..3) and E1^T coefficients on (rho[i-1], rho[i], rho[i+1])
  for (int tau = 0; tau < 4; ++tau) {
    if (t == 1) {          // M[i][i]: segments i (a = b = 0) and i - 1 (a = b = 1)
      E[tau][0] = alpha(tau, im, 0, 3);
      E[tau][1] = alpha(tau, i, 0, 0) + alpha(tau, im, 1, 3);
      E[tau][2] = alpha(tau, i, 1, 0);
    } else if (t == 2) {   // M[i][i+1]: segment i, (a, b) = (0, 1)
      E[tau][0] = 0.0;
      E[tau][1] = alpha(tau, i, 0, 1);
      E[tau][2] = alpha(tau, i, 1, 1);
    } else {               // M[i][i-1]: segment i - 1, (a, b) = (1, 0)
      E[tau][0] = alpha(tau, im, 0, 2);
      E[tau][1] = alpha(tau, im, 1, 2);
      E[tau][2] = 0.0;
    }
  }
  if (t == 1) {            // transpose of E1: its own diagonal
    ET[0] = E[1][0]; ET[1] = E[1][1]; ET[2] = E[1][2];
  } else if (t == 0) {     // (E1^T)[i][i-1] = E1[i-1][i]: segment i - 1, (a, b) = (0, 1)
    ET[0] = alpha(1, im, 0, 1); ET[1] = alpha(1, im, 1, 1); ET[2] = 0.0;
  } else {                 // (E1^T)[i][i+1] = E1[i+1][i]: segment i, (a, b) = (1, 0)
    ET[0] = 0.0; ET[1] = alpha(1, i, 0, 2); ET[2] = alpha(1, i, 1, 2);
  }
  for (int c = 0; c < 3; ++c) {
    k[c] = E[0][c];
    k[3 + c] = ET[c] - E[1][c];
    k[6 + c] = E[3][c];
  }
}

__host__ __device__ inline double fd_kdot(const double* k, double rm, double r0, double rp) {
#pragma clang fp contract(off)
  return fma(k[0], rm, fma(k[1], r0, k[2] * rp));
}

// Entries of E0, E1^T - E1 and M0 at one level from the densities at i-1, i, i+1.
struct FdEntry {
  double e0, ed, em;
};

__host__ __device__ inline FdEntry fd_entry(const double* k, double rm, double r0, double rp) {
  FdEntry v;
  v.e0 = fd_kdot(k, rm, r0, rp);
  v.ed = fd_kdot(k + 3, rm, r0, rp);
  v.em = fd_kdot(k + 6, rm, r0, rp);
  return v;
}

// theta_r, psi_r, P_r of entry (t, i) at level r of n from E0 at r-1, r, r+1
// (e0m is not used at r = 0, e0p not at r = n) and the entry of level r; the
// element's radial step h = (1 - xi_0) / n enters as h, 1/h and 1/(2h)
// (FdStep), so that a level needs no division.
struct FdRow {
  double th, ps, pm;
};

struct FdStep {
  double h, ih, i2h;
};

__host__ __device__ inline FdStep fd_step(double xi0, int n) {
  FdStep s;
  s.h = (1.0 - xi0) / n;
  s.ih = 1.0 / s.h;
  s.i2h = 0.5 * s.ih;
  return s;
}

__host__ __device__ inline FdRow fd_row(double xi0, const FdStep& st, int r, int n, double e0m, const FdEntry& v,
                                        double e0p) {
#pragma clang fp contract(off)   // no fusion beyond the explicit fma: the same bits in every file
  const double x = fma(st.h, (double)r, xi0);
  const double d0 = r == 0 ? (e0p - v.e0) * st.ih : (r == n ? (v.e0 - e0m) * st.ih : (e0p - e0m) * st.i2h);
  const double xh = x * st.ih;
  const double s2 = xh * xh;
  const double s1 = x * st.i2h;
  const double C = fma(x, d0, v.e0 + v.ed);
  const double a = s2 * v.e0, b = s1 * C;
  FdRow o;
  o.th = a - b;
  o.ps = a + b;
  o.pm = -((x * x) * v.em);
  return o;
}

// The rows of one element formed level by level inside a sweep (one 64-lane
// wavefront, n_b <= 21): lane l < 3 n_b evaluates entry (t, i) = (l / n_b,
// l % n_b) of theta_r, psi_r and P_r, the layout of a stored band row, so the
// lanes that hold items take their row's entries by cross-lane shuffles just
// as from a loaded row.  Lanes past 3 n_b evaluate entry 0.  Each density row
// is loaded (lane l < n_b holds node l, the others reread node 0) one row
// ahead of the one it completes, and the lanes take the densities of their
// entry's three nodes by shuffles.  Up: rows r = 0, 1, .., n in turn; down:
// rows r = n, n - 1, .., 0 (a call past the last row returns values nobody
// uses).
struct FdSweepRows {
  double k[kFdKappa];
  const double* rho;   // the element's density rows, [n + 1][n_b]
  double xi0;
  FdStep st;
  int n, nb, i;
  double e0o;          // E0 of the row formed before (up: r - 1, down: r + 1)
  FdEntry v;           // entries of row r
  double pend;         // density row in flight
  int r;               // the next row formed

  __device__ void load_row(int lev) {
    const int l = (int)threadIdx.x;
    lev = lev < 0 ? 0 : (lev > n ? n : lev);
    pend = rho[(int64_t)lev * nb + (l < nb ? l : 0)];
  }
  __device__ FdEntry entry_of(double row) const {
    const double rm = __shfl(row, fdb_md(i - 1, nb), 64), r0 = __shfl(row, i, 64),
                 rp = __shfl(row, fdb_md(i + 1, nb), 64);
    return fd_entry(k, rm, r0, rp);
  }
  // kap: kappa of the element's loop slots, [n_b][3][kFdKappa]; rho_e: its density rows
  __device__ void setup(const double* kap, const double* rho_e, double xi0_, int n_, int nb_) {
    const int l = (int)threadIdx.x;
    const int q = l < 3 * nb_ ? l : 0;
    const int t = q / nb_;
    i = q % nb_;
    for (int c = 0; c < kFdKappa; ++c) k[c] = kap[(i * 3 + t) * kFdKappa + c];
    rho = rho_e;
    xi0 = xi0_;
    n = n_;
    nb = nb_;
    st = fd_step(xi0_, n_);
    e0o = 0.0;
  }
  // up from row 0: v = row 0, row 1 in flight
  __device__ void init_up(const double* kap, const double* rho_e, double xi0_, int n_, int nb_) {
    setup(kap, rho_e, xi0_, n_, nb_);
    load_row(0);
    v = entry_of(pend);
    load_row(1);
    r = 0;
  }
  // down from row n (the row after it is not needed there): v = row n, row n - 1 in flight
  __device__ void init_down(const double* kap, const double* rho_e, double xi0_, int n_, int nb_) {
    setup(kap, rho_e, xi0_, n_, nb_);
    load_row(n);
    v = entry_of(pend);
    load_row(n - 1);
    r = n;
  }
  __device__ FdRow next_up() {
    const FdEntry vp = entry_of(pend);          // row r + 1
    const FdRow o = fd_row(xi0, st, r, n, e0o, v, vp.e0);
    e0o = v.e0;
    v = vp;
    load_row(r + 2);
    ++r;
    return o;
  }
  __device__ FdRow next_down() {
    const FdEntry vm = entry_of(pend);          // row r - 1
    const FdRow o = fd_row(xi0, st, r, n, vm.e0, v, e0o);
    e0o = v.e0;
    v = vm;
    load_row(r - 2);
    --r;
    return o;
  }
};

// Checks the host dense kernels of the coarse factorisation against the
// textbook loops they replace: the same bits for every entry (blocked LU with
// and without a thread team, multiply-accumulate with either sign and strided
// left factors, row-oriented triangular inverses), and the pivot failure.
// Built and run by tests/test_dense_host.py; prints "ok" and exits 0 on
// success.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "dense_host.h"

// the reference loops never fuse a product into an addition, whatever the
// flags of this file: a library built with fused multiply-add fails the check
#define REF __attribute__((optimize("fp-contract=off"), noinline))

namespace {

int failures = 0;

void expect(bool ok, const char* what, int a, int b) {
  if (!ok) {
    std::printf("FAIL %s (%d, %d)\n", what, a, b);
    ++failures;
  }
}

bool same_bits(const std::vector<double>& x, const std::vector<double>& y) {
  return x.size() == y.size() && std::memcmp(x.data(), y.data(), x.size() * sizeof(double)) == 0;
}

// a front with some exact zeros (the skip rule matters) and a dominant diagonal
std::vector<double> front(int mf, std::mt19937_64& g) {
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  std::vector<double> F((size_t)mf * mf);
  for (int i = 0; i < mf; ++i)
    for (int j = 0; j < mf; ++j) {
      const double v = u(g);
      F[(size_t)i * mf + j] = i == j ? 3.0 * mf + v : (std::fabs(v) < 0.3 ? 0.0 : v);
    }
  return F;
}

REF int textbook_lu(std::vector<double>& F, int mf, int nj) {
  for (int k = 0; k < nj; ++k) {
    const double piv = F[(size_t)k * mf + k];
    if (!(std::fabs(piv) > 0.0) || !std::isfinite(piv)) return k;
    for (int i = k + 1; i < mf; ++i) {
      double* ri = &F[(size_t)i * mf];
      const double l = ri[k] / piv;
      ri[k] = l;
      if (l != 0.0)
        for (int j = k + 1; j < mf; ++j) ri[j] -= l * F[(size_t)k * mf + j];
    }
  }
  return -1;
}

REF void textbook_inverses(const std::vector<double>& A, int mf, int nj, std::vector<double>& P,
                           std::vector<double>& Q) {
  for (int j = 0; j < nj; ++j) {   // column by column
    P[(size_t)j * nj + j] = 1.0;
    for (int i = j + 1; i < nj; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s -= A[(size_t)i * mf + k] * P[(size_t)k * nj + j];
      P[(size_t)i * nj + j] = s;
    }
  }
  for (int j = nj - 1; j >= 0; --j) {
    Q[(size_t)j * nj + j] = 1.0 / A[(size_t)j * mf + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= j; ++k) s -= A[(size_t)i * mf + k] * Q[(size_t)k * nj + j];
      Q[(size_t)i * nj + j] = s / A[(size_t)i * mf + i];
    }
  }
}

REF void textbook_mac(bool sub, std::vector<double>& R, const std::vector<double>& A, const std::vector<double>& B,
                      int m, int n, int K) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 1; k < K; ++k) {   // steps k0 = 1 .. K - 1
        const double a = A[(size_t)i * K + k];
        if (a == 0.0) continue;
        if (sub)
          R[(size_t)i * n + j] -= a * B[(size_t)k * n + j];
        else
          R[(size_t)i * n + j] += a * B[(size_t)k * n + j];
      }
}

}  // namespace

int main() {
  std::mt19937_64 g(20250106);
  DenseTeam team(4);
  // LU: square fronts, fronts with a trailing block, sizes around the panel width
  const int sizes[][2] = {{1, 1}, {5, 3}, {31, 31}, {32, 32}, {33, 20}, {70, 64}, {97, 45}, {130, 130}, {200, 77}};
  for (const auto& sz : sizes) {
    const int mf = sz[0], nj = sz[1];
    std::vector<double> F = front(mf, g), A = F, B = F, C = F;
    expect(textbook_lu(A, mf, nj) == -1, "textbook pivots", mf, nj);
    expect(dense_lu(B.data(), mf, nj, nullptr) == -1, "blocked pivots", mf, nj);
    expect(dense_lu(C.data(), mf, nj, &team) == -1, "team pivots", mf, nj);
    expect(same_bits(A, B), "blocked LU bits", mf, nj);
    expect(same_bits(A, C), "team LU bits", mf, nj);
    // inverses of the eliminated leading block, whole and in column blocks
    std::vector<double> P((size_t)nj * nj, 0.0), Q((size_t)nj * nj, 0.0), P2 = P, Q2 = Q;
    textbook_inverses(A, mf, nj, P, Q);
    for (int c0 = 0; c0 < nj; c0 += 7) {
      const int c1 = c0 + 7 < nj ? c0 + 7 : nj;
      dense_inv_unit_lower(B.data(), mf, nj, P2.data(), c0, c1);
      dense_inv_upper(B.data(), mf, nj, Q2.data(), c0, c1);
    }
    expect(same_bits(P, P2), "unit lower inverse bits", mf, nj);
    expect(same_bits(Q, Q2), "upper inverse bits", mf, nj);
    // the inverses are inverses (a pin independent of the loops above)
    double worst = 0.0;
    for (int i = 0; i < nj; ++i)
      for (int j = 0; j < nj; ++j) {
        double l = 0.0, u = 0.0;
        for (int k = 0; k < nj; ++k) {
          const double lik = k < i ? A[(size_t)i * mf + k] : (k == i ? 1.0 : 0.0);
          l += lik * P[(size_t)k * nj + j];
          const double uik = k >= i ? A[(size_t)i * mf + k] : 0.0;
          u += uik * Q[(size_t)k * nj + j];
        }
        worst = std::fmax(worst, std::fabs(l - (i == j)));
        worst = std::fmax(worst, std::fabs(u - (i == j)));
      }
    expect(worst < 1e-12, "inverse residual", mf, nj);
  }
  // multiply-accumulate: both signs, strided left factor, ragged shapes
  const int shapes[][3] = {{1, 1, 1}, {3, 5, 2}, {4, 4, 4}, {7, 9, 13}, {16, 33, 40}, {41, 6, 29}};
  for (const auto& sh : shapes) {
    const int m = sh[0], n = sh[1], K = sh[2];
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    std::vector<double> A((size_t)m * K), At((size_t)K * m), B((size_t)K * n), C0((size_t)m * n);
    for (int i = 0; i < m; ++i)
      for (int k = 0; k < K; ++k) {
        const double v = u(g);
        A[(size_t)i * K + k] = At[(size_t)k * m + i] = std::fabs(v) < 0.25 ? 0.0 : v;
      }
    for (double& x : B) x = u(g);
    for (double& x : C0) x = u(g);
    if (K > 2) {   // column 2 of A zero and row 2 of B infinite: only the skip keeps C finite
      for (int i = 0; i < m; ++i) A[(size_t)i * K + 2] = At[(size_t)2 * m + i] = 0.0;
      for (int j = 0; j < n; ++j) B[(size_t)2 * n + j] = (j % 2 ? 1.0 : -1.0) * INFINITY;
    }
    for (int sub = 0; sub < 2; ++sub) {
      std::vector<double> R = C0, D = C0, E = C0;
      textbook_mac(sub != 0, R, A, B, m, n, K);
      dense_mac(sub != 0, D.data(), n, A.data(), K, 1, B.data(), n, m, n, 1, K);
      dense_mac(sub != 0, E.data(), n, At.data(), 1, m, B.data(), n, m, n, 1, K);
      expect(same_bits(R, D), "mac bits", m, n);
      expect(same_bits(R, E), "strided mac bits", m, n);
    }
  }
  // a zero pivot is reported at its index, by both paths
  {
    const int mf = 50, nj = 40;
    std::vector<double> F = front(mf, g);
    for (int j = 0; j < mf; ++j) F[(size_t)37 * mf + j] = 0.0;   // row 37 zero: pivot 37 is zero
    std::vector<double> A = F, B = F;
    expect(textbook_lu(A, mf, nj) == 37, "textbook zero pivot", mf, nj);
    expect(dense_lu(B.data(), mf, nj, &team) == 37, "blocked zero pivot", mf, nj);
  }
  if (failures) return 1;
  std::printf("ok\n");
  return 0;
}

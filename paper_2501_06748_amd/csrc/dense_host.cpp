// Dense kernels of the host factorisation of K_g (declarations and the
// operation-order contract in dense_host.h).  Plain host C++, built without
// fused multiply-add: every result entry takes exactly the products and
// additions of the textbook loops, in the same order.
#include "dense_host.h"

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <immintrin.h>
#include <mutex>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

namespace {

typedef double v2d __attribute__((vector_size(16)));

inline v2d ld2(const double* p) {
  v2d v;
  std::memcpy(&v, p, sizeof v);
  return v;
}
inline void st2(double* p, v2d v) { std::memcpy(p, &v, sizeof v); }

template <bool SUB>
inline void mac(v2d& c, double a, v2d b) {
  const v2d s = {a, a};
  if (SUB)
    c -= s * b;
  else
    c += s * b;
}

template <bool SUB>
inline void mac1(double& c, double a, double b) {
  if (SUB)
    c -= a * b;
  else
    c += a * b;
}

// R rows x 4 columns of C, steps k0 .. k1 - 1, accumulators in registers
template <bool SUB, int R>
void tile(double* C, int64_t ldc, const double* A, int64_t sai, int64_t sak, const double* B, int64_t ldb,
          int64_t k0, int64_t k1) {
  v2d c[R][2];
  const double* a[R];
  for (int r = 0; r < R; ++r) {
    c[r][0] = ld2(C + r * ldc);
    c[r][1] = ld2(C + r * ldc + 2);
    a[r] = A + r * sai;
  }
  for (int64_t k = k0; k < k1; ++k) {
    const v2d b0 = ld2(B + k * ldb), b1 = ld2(B + k * ldb + 2);
    for (int r = 0; r < R; ++r) {
      const double x = a[r][k * sak];
      if (x != 0.0) {
        mac<SUB>(c[r][0], x, b0);
        mac<SUB>(c[r][1], x, b1);
      }
    }
  }
  for (int r = 0; r < R; ++r) {
    st2(C + r * ldc, c[r][0]);
    st2(C + r * ldc + 2, c[r][1]);
  }
}

// rows x one column, one step after the other
template <bool SUB>
void column(double* C, int64_t ldc, const double* A, int64_t sai, int64_t sak, const double* B, int64_t ldb,
            int64_t m, int64_t k0, int64_t k1) {
  for (int64_t i = 0; i < m; ++i) {
    double c = C[i * ldc];
    const double* a = A + i * sai;
    for (int64_t k = k0; k < k1; ++k) {
      const double x = a[k * sak];
      if (x != 0.0) mac1<SUB>(c, x, B[k * ldb]);
    }
    C[i * ldc] = c;
  }
}

template <bool SUB>
void mac_block(double* C, int64_t ldc, const double* A, int64_t sai, int64_t sak, const double* B, int64_t ldb,
               int64_t m, int64_t n, int64_t k0, int64_t k1) {
  const int64_t n4 = n & ~int64_t(3), m4 = m & ~int64_t(3);
  for (int64_t i = 0; i < m4; i += 4)
    for (int64_t j = 0; j < n4; j += 4)
      tile<SUB, 4>(C + i * ldc + j, ldc, A + i * sai, sai, sak, B + j, ldb, k0, k1);
  for (int64_t i = m4; i < m; ++i)
    for (int64_t j = 0; j < n4; j += 4)
      tile<SUB, 1>(C + i * ldc + j, ldc, A + i * sai, sai, sak, B + j, ldb, k0, k1);
  for (int64_t j = n4; j < n; ++j) column<SUB>(C + j, ldc, A, sai, sak, B + j, ldb, m, k0, k1);
}

}  // namespace

struct DenseTeam::State {
  std::vector<std::thread> workers;
  std::atomic<uint64_t> gen{0};
  std::atomic<int> done{0};
  std::atomic<bool> stop{false};
  const std::function<void(int)>* fn = nullptr;
  std::mutex mu;
  std::condition_variable cv;
};

namespace {
constexpr int kSpins = 4096;   // polls (each with a pause hint) before a worker sleeps
}

DenseTeam::DenseTeam(int threads) : st_(new State), n_(std::max(1, threads)) {
  for (int t = 1; t < n_; ++t)
    st_->workers.emplace_back([this, t] {
      uint64_t seen = 0;
      for (;;) {
        uint64_t g = st_->gen.load(std::memory_order_acquire);
        for (int spin = 0; g == seen && spin < kSpins; ++spin) {
          _mm_pause();
          g = st_->gen.load(std::memory_order_acquire);
        }
        if (g == seen) {
          std::unique_lock<std::mutex> lk(st_->mu);
          st_->cv.wait(lk, [&] { return st_->gen.load(std::memory_order_acquire) != seen; });
          g = st_->gen.load(std::memory_order_acquire);
        }
        seen = g;
        if (st_->stop.load(std::memory_order_acquire)) return;
        (*st_->fn)(t);
        st_->done.fetch_add(1, std::memory_order_acq_rel);
      }
    });
}

DenseTeam::~DenseTeam() {
  st_->stop.store(true, std::memory_order_release);
  {
    std::lock_guard<std::mutex> lk(st_->mu);
    st_->gen.fetch_add(1, std::memory_order_acq_rel);
  }
  st_->cv.notify_all();
  for (auto& w : st_->workers) w.join();
  delete st_;
}

void DenseTeam::run(const std::function<void(int)>& fn) {
  if (n_ == 1) {
    fn(0);
    return;
  }
  st_->fn = &fn;
  st_->done.store(0, std::memory_order_relaxed);
  {
    std::lock_guard<std::mutex> lk(st_->mu);
    st_->gen.fetch_add(1, std::memory_order_acq_rel);
  }
  st_->cv.notify_all();
  fn(0);
  while (st_->done.load(std::memory_order_acquire) != n_ - 1) _mm_pause();
}

int dense_threads() { return (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency())); }

void dense_mac(bool sub, double* C, int64_t ldc, const double* A, int64_t sai, int64_t sak, const double* B,
               int64_t ldb, int64_t m, int64_t n, int64_t k0, int64_t k1) {
  if (m <= 0 || n <= 0 || k1 <= k0) return;
  if (sub)
    mac_block<true>(C, ldc, A, sai, sak, B, ldb, m, n, k0, k1);
  else
    mac_block<false>(C, ldc, A, sai, sak, B, ldb, m, n, k0, k1);
}

int dense_lu(double* F, int64_t mf, int nj, DenseTeam* team) {
  constexpr int kPanel = 32;                // pivots per panel
  constexpr int64_t kTeamWork = 1 << 18;    // multiply-adds below a panel worth sharing among threads
  for (int p0 = 0; p0 < nj; p0 += kPanel) {
    const int p1 = std::min(p0 + kPanel, nj);
    // the panel's own rows: pivots p0 .. p1 - 1 on the panel's columns
    for (int k = p0; k < p1; ++k) {
      const double piv = F[(int64_t)k * mf + k];
      if (!(std::fabs(piv) > 0.0) || !std::isfinite(piv)) return k;
      const double* rk = F + (int64_t)k * mf;
      for (int64_t i = k + 1; i < p1; ++i) {
        double* ri = F + i * mf;
        const double l = ri[k] / piv;
        ri[k] = l;
        if (l != 0.0)
          for (int64_t j = k + 1; j < p1; ++j) ri[j] -= l * rk[j];
      }
    }
    const int64_t nc = mf - p1;
    if (nc <= 0) continue;
    // the panel's rows after its columns: row r takes pivots p0 .. r - 1 in turn
    for (int64_t r = p0 + 1; r < p1; ++r)
      dense_mac(true, F + r * mf + p1, mf, F + r * mf, mf, 1, F + p1, mf, 1, nc, p0, r);
    // rows [a, b) below the panel: their multipliers (pivots in turn, panel columns),
    // then the updates of their columns after the panel
    auto below = [&](int64_t a, int64_t b) {
      for (int64_t i = a; i < b; ++i) {
        double* ri = F + i * mf;
        for (int k = p0; k < p1; ++k) {
          const double l = ri[k] / F[(int64_t)k * mf + k];
          ri[k] = l;
          if (l != 0.0) {
            const double* rk = F + (int64_t)k * mf;
            for (int64_t j = k + 1; j < p1; ++j) ri[j] -= l * rk[j];
          }
        }
      }
      dense_mac(true, F + a * mf + p1, mf, F + a * mf, mf, 1, F + p1, mf, b - a, nc, p0, p1);
    };
    if (team && team->size() > 1 && nc * nc * (p1 - p0) > kTeamWork) {
      const int T = team->size();
      team->run([&](int t) { below(p1 + nc * t / T, p1 + nc * (t + 1) / T); });
    } else {
      below(p1, mf);
    }
  }
  return -1;
}

// Row-oriented triangular inverses: row i of X is formed from the rows before
// (lower) or after (upper) it, vectorised along the row; each entry still
// takes its terms in increasing k, as the column-by-column textbook loops do.
void dense_inv_unit_lower(const double* A, int64_t lda, int n, double* X, int c0, int c1) {
  for (int i = 0; i < n; ++i) {
    double* xi = X + (size_t)i * n;
    const int j1 = std::min(c1, i);
    for (int j = c0; j < j1; ++j) xi[j] = 0.0;
    // X[i][j] = -sum_{k = j}^{i-1} A[i][k] X[k][j]: step k touches the entries j <= k
    for (int k = c0; k < i; ++k) {
      const double a = A[i * lda + k];
      const double* xk = X + (size_t)k * n;
      const int je = std::min(j1 - 1, k);
      for (int j = c0; j <= je; ++j) xi[j] -= a * xk[j];
    }
    if (i >= c0 && i < c1) xi[i] = 1.0;
  }
}

void dense_inv_upper(const double* A, int64_t lda, int n, double* X, int c0, int c1) {
  for (int i = n - 1; i >= 0; --i) {
    double* xi = X + (size_t)i * n;
    const int j0 = std::max(c0, i + 1);
    for (int j = j0; j < c1; ++j) xi[j] = 0.0;
    // X[i][j] = -(sum_{k = i+1}^{j} A[i][k] X[k][j]) / A[i][i]: step k touches the entries j >= k
    for (int k = i + 1; k < c1; ++k) {
      const double a = A[i * lda + k];
      const double* xk = X + (size_t)k * n;
      for (int j = std::max(j0, k); j < c1; ++j) xi[j] -= a * xk[j];
    }
    const double d = A[i * lda + i];
    for (int j = j0; j < c1; ++j) xi[j] = xi[j] / d;
    if (i >= c0 && i < c1) xi[i] = 1.0 / d;
  }
}

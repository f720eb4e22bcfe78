// Dense kernels of the host factorisation of the coarse matrix K_g (the
// multifrontal LU in a nested-dissection order, factored once per model).
//
// Every kernel here computes each result entry with the same sequence of
// floating-point operations as the plain loops it replaces (one product and
// one addition or subtraction per step, steps in increasing k, a step skipped
// where the left factor is zero; no fused multiply-add), so the factors do not
// depend on blocking, vector width or the number of threads.
#pragma once

#include <cstdint>
#include <functional>

// A fixed set of host threads for one factorisation: run(fn) calls fn(t) for
// t = 0 .. size() - 1, t = 0 on the calling thread, and returns when all
// have finished.  Between calls the workers poll briefly, then sleep.
class DenseTeam {
 public:
  explicit DenseTeam(int threads);
  ~DenseTeam();
  DenseTeam(const DenseTeam&) = delete;
  DenseTeam& operator=(const DenseTeam&) = delete;
  int size() const { return n_; }
  void run(const std::function<void(int)>& fn);

 private:
  struct State;
  State* st_;
  int n_;
};

// Host threads for the factorisation: the hardware concurrency, at most 16.
int dense_threads();

// C[i][j] = C[i][j] + A[i][k] B[k][j] (sub false) or - A[i][k] B[k][j] (sub
// true) for k = k0, .., k1 - 1 in turn, skipping k where A[i][k] == 0, over
// rows i < m and columns j < n.  C and B are row-major with leading
// dimensions ldc and ldb; A[i][k] is A[i sai + k sak] (k absolute, as in B).
// The regions of C, A and B may lie in one array but must not overlap.
void dense_mac(bool sub, double* C, int64_t ldc, const double* A, int64_t sai, int64_t sak, const double* B,
               int64_t ldb, int64_t m, int64_t n, int64_t k0, int64_t k1);

// LU without pivoting of the first nj pivots of the row-major mf x mf front F:
// for k < nj, l_ik = F[i][k] / F[k][k] replaces F[i][k] (i > k) and
// F[i][j] -= l_ik F[k][j] (j > k, skipped where l_ik == 0).  Returns -1, or
// the first k whose pivot is zero or not finite (F is then partly eliminated).
// The trailing updates are shared among the team's threads (team may be null).
int dense_lu(double* F, int64_t mf, int nj, DenseTeam* team);

// Columns [c0, c1) of X = inverse of the unit lower triangle of the leading
// n x n block of A (row-major, leading dimension lda); X is n x n row-major.
void dense_inv_unit_lower(const double* A, int64_t lda, int n, double* X, int c0, int c1);

// Columns [c0, c1) of X = inverse of the upper triangle (with its diagonal).
void dense_inv_upper(const double* A, int64_t lda, int n, double* X, int c0, int c1);

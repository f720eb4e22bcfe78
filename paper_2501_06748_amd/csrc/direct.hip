// Direct coarse solve: nested-dissection LU of K_g, factored once per model.
//
// The paper condenses every element onto its boundary nodes and assembles the
// dynamic stiffnesses into one global nodal system (Section "Radial
// discretization"); K_g stays the same for every time step of a run with
// fixed dt.  Here K_g is factored once, K_g = L U, in a nested-dissection
// order built from the node coordinates, and every step solves with the
// factors (K_g^T = U^T L^T for the adjoint).
//
// Ordering (per mesh, host): the node set is split recursively by the median
// coordinate along its wider extent; the separator is the set of nodes on the
// lower side that couple to the upper side.  Both halves are ordered before
// their separator, so the supernodes (separators and leaves of at most
// kLeaf nodes) come out in postorder and each covers a contiguous range of
// positions.  B_J, the later positions coupled to supernode J after the
// elimination of its subtree, follows from J's own couplings and the B sets
// of its children.
//
// Factorisation (per model, host, multifrontal): the front of J (rows and
// columns J then B_J) is assembled from the entries of K_g whose first index
// in elimination order lies in J and from the children's update matrices;
// its first |J| pivots are eliminated without pivoting (K_g is dominated by
// the a0-weighted mass term), giving L11, U11, L21 = F21 U11^-1,
// U12 = L11^-1 F12 and the update F22 - L21 U12 for J's parent.  The device
// keeps, per supernode and column-major, P = L11^-1, C = L21, Q = U11^-1 and
// E = U12 (and the transposed set for K_g^T).
//
// Solve (device, per level of the dissection tree, one block per supernode):
// forward, deepest level first: t_J = b_J - (sum of the contributions
// L21^(D) y_D of J's descendants D to J's rows, added in a fixed order),
// y_J = P_J t_J, then J's own contribution C_J y_J to its B_J rows;
// backward, root first: x_J = Q_J (y_J - E_J x_{B_J}).  No atomics: results
// are bit-reproducible.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "sbfwi_internal.h"

namespace {

constexpr int kLeaf = 24;     // nodes per leaf supernode
constexpr int DT = 256;       // threads per block of the solve kernels

// ------------------------------------------------------------------ ordering

struct Dissect {
  const std::vector<int64_t>& rp;
  const std::vector<int64_t>& col;
  const double* xy;
  std::vector<int64_t> order;            // node ids in elimination order
  std::vector<int64_t> sn_ptr{0};        // supernode position ranges (postorder)
  std::vector<int32_t> parent;           // filled after
  std::vector<std::vector<int32_t>> kids;
  std::vector<char> side;                // scratch: 1 = upper half of the current split
  std::vector<char> member;              // scratch: in the current set

  Dissect(const std::vector<int64_t>& r, const std::vector<int64_t>& c, const double* p, int64_t n)
      : rp(r), col(c), xy(p), side(n, 0), member(n, 0) {}

  int emit(const std::vector<int64_t>& nodes, std::vector<int32_t> children) {
    for (int64_t v : nodes) order.push_back(v);
    sn_ptr.push_back((int64_t)order.size());
    kids.push_back(std::move(children));
    return (int)kids.size() - 1;
  }

  // returns the supernode id of the subtree's root, or -1 for an empty set
  int run(std::vector<int64_t> V) {
    if (V.empty()) return -1;
    if ((int64_t)V.size() <= kLeaf) return emit(V, {});
    double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
    for (int64_t v : V)
      for (int a = 0; a < 2; ++a) {
        lo[a] = std::min(lo[a], xy[2 * v + a]);
        hi[a] = std::max(hi[a], xy[2 * v + a]);
      }
    int ax = (hi[0] - lo[0]) >= (hi[1] - lo[1]) ? 0 : 1;
    std::vector<double> vals;
    vals.reserve(V.size());
    for (int64_t v : V) vals.push_back(xy[2 * v + ax]);
    std::sort(vals.begin(), vals.end());
    vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
    if (vals.size() < 2) {   // all on one line across this axis: try the other one
      ax = 1 - ax;
      vals.clear();
      for (int64_t v : V) vals.push_back(xy[2 * v + ax]);
      std::sort(vals.begin(), vals.end());
      vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
      if (vals.size() < 2) return emit(V, {});
    }
    const double med = vals[(vals.size() - 1) / 2];
    for (int64_t v : V) {
      member[v] = 1;
      side[v] = xy[2 * v + ax] > med ? 1 : 0;
    }
    std::vector<int64_t> V1, V2, S;
    for (int64_t v : V) {
      if (side[v]) {
        V2.push_back(v);
        continue;
      }
      bool cut = false;
      for (int64_t q = rp[v]; q < rp[v + 1] && !cut; ++q) {
        const int64_t w = col[q];
        cut = member[w] && side[w];
      }
      (cut ? S : V1).push_back(v);
    }
    for (int64_t v : V) member[v] = side[v] = 0;
    if (S.empty()) {   // the halves do not touch: any node separates them
      S.push_back(V1.back());
      V1.pop_back();
    }
    std::vector<int32_t> ch;
    int c1 = run(std::move(V1));
    int c2 = run(std::move(V2));
    if (c1 >= 0) ch.push_back(c1);
    if (c2 >= 0) ch.push_back(c2);
    return emit(S, ch);
  }
};

__global__ void fwd_level_kernel(const int32_t* __restrict__ lvl_sn, DirectDev d, const double* __restrict__ P,
                                 const double* __restrict__ Cm, int NS, const double* __restrict__ b,
                                 double* __restrict__ tb, double* __restrict__ yb, double* __restrict__ cb,
                                 int* __restrict__ status) {
  const int J = lvl_sn[blockIdx.x];
  const int64_t j0 = d.sn_ptr[J];
  const int nj = (int)(d.sn_ptr[J + 1] - j0);
  const int64_t b0 = d.b_ptr[J];
  const int nb = (int)(d.b_ptr[J + 1] - b0);
  const double* Pj = P + d.mm_off[J];
  const double* Cj = Cm + d.mb_off[J];
  for (int it = threadIdx.x; it < nj * NS; it += DT) {
    const int i = it / NS, s = it - i * NS;
    const int64_t p = j0 + i;
    double t = b[d.inv[p] * NS + s];
    for (int64_t q = d.cl_ptr[p]; q < d.cl_ptr[p + 1]; ++q) t -= cb[d.cl_idx[q] * NS + s];
    tb[p * NS + s] = t;
  }
  __syncthreads();
  bool bad = false;
  for (int it = threadIdx.x; it < nj * NS; it += DT) {
    const int i = it / NS, s = it - i * NS;
    double y = 0.0;
    for (int k = 0; k < nj; ++k) y += Pj[(int64_t)k * nj + i] * tb[(j0 + k) * NS + s];
    yb[(j0 + i) * NS + s] = y;
    bad = bad || !isfinite(y);
  }
  if (bad) atomicOr(&status[0], 4);
  __syncthreads();
  for (int it = threadIdx.x; it < nb * NS; it += DT) {
    const int r = it / NS, s = it - r * NS;
    double c = 0.0;
    for (int k = 0; k < nj; ++k) c += Cj[(int64_t)k * nb + r] * yb[(j0 + k) * NS + s];
    cb[(b0 + r) * NS + s] = c;
  }
}

__global__ void bwd_level_kernel(const int32_t* __restrict__ lvl_sn, DirectDev d, const double* __restrict__ Q,
                                 const double* __restrict__ E, int NS, const double* __restrict__ yb,
                                 double* __restrict__ tb, double* __restrict__ xp, double* __restrict__ x) {
  const int J = lvl_sn[blockIdx.x];
  const int64_t j0 = d.sn_ptr[J];
  const int nj = (int)(d.sn_ptr[J + 1] - j0);
  const int64_t b0 = d.b_ptr[J];
  const int nb = (int)(d.b_ptr[J + 1] - b0);
  const double* Qj = Q + d.mm_off[J];
  const double* Ej = E + d.mb_off[J];
  for (int it = threadIdx.x; it < nj * NS; it += DT) {
    const int i = it / NS, s = it - i * NS;
    double t = yb[(j0 + i) * NS + s];
    for (int r = 0; r < nb; ++r) t -= Ej[(int64_t)r * nj + i] * xp[d.bpos[b0 + r] * NS + s];
    tb[(j0 + i) * NS + s] = t;
  }
  __syncthreads();
  for (int it = threadIdx.x; it < nj * NS; it += DT) {
    const int i = it / NS, s = it - i * NS;
    double v = 0.0;
    for (int k = 0; k < nj; ++k) v += Qj[(int64_t)k * nj + i] * tb[(j0 + k) * NS + s];
    xp[(j0 + i) * NS + s] = v;
    x[d.inv[j0 + i] * NS + s] = v;
  }
}

__global__ void count_solve_kernel(int* status) {
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&status[5], 1);
}

}  // namespace

// ------------------------------------------------------------------ symbolic (per mesh)

int sbfwi_direct_symbolic(sbfwi_mesh_s* m, const double* node_xy) {
  DirectSym* ds = new DirectSym();
  m->dsym = ds;
  const int64_t n = m->n_nodes;
  Dissect dis(m->h_row_ptr, m->h_col64, node_xy, n);
  std::vector<int64_t> all(n);
  std::iota(all.begin(), all.end(), 0);
  const int root = dis.run(std::move(all));
  if ((int64_t)dis.order.size() != n || root < 0) return sbfwi_fail(SBFWI_EINVAL, "nested dissection lost nodes");
  const int nS = (int)dis.kids.size();
  ds->nS = nS;
  ds->inv = dis.order;
  ds->sn_ptr = dis.sn_ptr;
  ds->pos.assign(n, 0);
  for (int64_t p = 0; p < n; ++p) ds->pos[ds->inv[p]] = p;
  ds->children = dis.kids;
  ds->level.assign(nS, 0);
  for (int J = nS - 1; J >= 0; --J)   // parents come after their children
    for (int c : ds->children[J]) ds->level[c] = ds->level[J] + 1;
  ds->depth = *std::max_element(ds->level.begin(), ds->level.end());
  // B sets
  std::vector<int64_t> stamp(n, -1);
  ds->b_ptr.assign(nS + 1, 0);
  std::vector<std::vector<int64_t>> B(nS);
  for (int J = 0; J < nS; ++J) {
    const int64_t j0 = ds->sn_ptr[J], j1 = ds->sn_ptr[J + 1];
    std::vector<int64_t>& bj = B[J];
    auto add = [&](int64_t p) {
      if (p >= j1 && stamp[p] != J) {
        stamp[p] = J;
        bj.push_back(p);
      }
    };
    for (int64_t p = j0; p < j1; ++p) {
      const int64_t v = ds->inv[p];
      for (int64_t q = m->h_row_ptr[v]; q < m->h_row_ptr[v + 1]; ++q) add(ds->pos[m->h_col64[q]]);
    }
    for (int c : ds->children[J])
      for (int64_t p : B[c]) add(p);
    std::sort(bj.begin(), bj.end());
    ds->b_ptr[J + 1] = ds->b_ptr[J] + (int64_t)bj.size();
  }
  ds->bpos.resize(ds->b_ptr[nS]);
  for (int J = 0; J < nS; ++J) std::copy(B[J].begin(), B[J].end(), ds->bpos.begin() + ds->b_ptr[J]);
  // contribution lists per position: (D, k) with B_D[k] = p, D ascending
  std::vector<int64_t> cnt(n + 1, 0);
  for (int64_t q = 0; q < ds->b_ptr[nS]; ++q) cnt[ds->bpos[q] + 1]++;
  for (int64_t p = 0; p < n; ++p) cnt[p + 1] += cnt[p];
  ds->cl_ptr = cnt;
  ds->cl_idx.assign(cnt[n], 0);
  {
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int D = 0; D < nS; ++D)
      for (int64_t q = ds->b_ptr[D]; q < ds->b_ptr[D + 1]; ++q) ds->cl_idx[fill[ds->bpos[q]]++] = q;
  }
  // dense block offsets and level lists
  ds->mm_off.assign(nS + 1, 0);
  ds->mb_off.assign(nS + 1, 0);
  ds->max_nj = 0;
  for (int J = 0; J < nS; ++J) {
    const int64_t nj = ds->sn_ptr[J + 1] - ds->sn_ptr[J], nb = ds->b_ptr[J + 1] - ds->b_ptr[J];
    ds->mm_off[J + 1] = ds->mm_off[J] + nj * nj;
    ds->mb_off[J + 1] = ds->mb_off[J] + nj * nb;
    ds->max_nj = std::max<int64_t>(ds->max_nj, nj);
  }
  ds->lvl_ptr.assign(ds->depth + 2, 0);
  for (int J = 0; J < nS; ++J) ds->lvl_ptr[ds->level[J] + 1]++;
  for (int l = 0; l <= ds->depth; ++l) ds->lvl_ptr[l + 1] += ds->lvl_ptr[l];
  ds->lvl_sn.assign(nS, 0);
  {
    std::vector<int32_t> fill(ds->lvl_ptr.begin(), ds->lvl_ptr.end() - 1);
    for (int J = 0; J < nS; ++J) ds->lvl_sn[fill[ds->level[J]]++] = J;
  }
  DirectDev& d = ds->d;
  SBFWI_CHECK(sbfwi_upload(&d.inv, ds->inv));
  SBFWI_CHECK(sbfwi_upload(&d.sn_ptr, ds->sn_ptr));
  SBFWI_CHECK(sbfwi_upload(&d.b_ptr, ds->b_ptr));
  SBFWI_CHECK(sbfwi_upload(&d.bpos, ds->bpos));
  SBFWI_CHECK(sbfwi_upload(&d.cl_ptr, ds->cl_ptr));
  SBFWI_CHECK(sbfwi_upload(&d.cl_idx, ds->cl_idx));
  SBFWI_CHECK(sbfwi_upload(&d.mm_off, ds->mm_off));
  SBFWI_CHECK(sbfwi_upload(&d.mb_off, ds->mb_off));
  SBFWI_CHECK(sbfwi_upload(&ds->lvl_sn_dev, ds->lvl_sn));
  return SBFWI_OK;
}

void sbfwi_direct_sym_free(DirectSym* ds) {
  if (!ds) return;
  DirectDev& d = ds->d;
  void* ptrs[] = {d.inv, d.sn_ptr, d.b_ptr, d.bpos, d.cl_ptr, d.cl_idx, d.mm_off, d.mb_off, ds->lvl_sn_dev};
  for (void* p : ptrs) sbfwi_dev_free(p);
  delete ds;
}

// ------------------------------------------------------------------ numeric (per model)

namespace {

// Unit-lower-triangular inverse of the strictly-lower part of A (n x n, row-major,
// leading dimension lda) into column-major out; upper-triangular inverse likewise.
void inv_unit_lower(const double* A, int64_t lda, int n, double* out) {
  std::vector<double> X((size_t)n * n, 0.0);   // row-major
  for (int j = 0; j < n; ++j) {
    X[(size_t)j * n + j] = 1.0;
    for (int i = j + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s -= A[i * lda + k] * X[(size_t)k * n + j];
      X[(size_t)i * n + j] = s;
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[(size_t)j * n + i] = X[(size_t)i * n + j];
}

void inv_upper(const double* A, int64_t lda, int n, double* out) {
  std::vector<double> X((size_t)n * n, 0.0);   // row-major
  for (int j = n - 1; j >= 0; --j) {
    X[(size_t)j * n + j] = 1.0 / A[j * lda + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= j; ++k) s -= A[i * lda + k] * X[(size_t)k * n + j];
      X[(size_t)i * n + j] = s / A[i * lda + i];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[(size_t)j * n + i] = X[(size_t)i * n + j];
}

}  // namespace

int sbfwi_direct_factor(sbfwi_factors_s* f, hipStream_t s) {
  sbfwi_mesh_s* m = f->m;
  DirectSym* ds = m->dsym;
  if (!ds) return sbfwi_fail(SBFWI_EINVAL, "mesh has no dissection order");
  const int64_t nnz = m->nnz, n = m->n_nodes;
  std::vector<double> K(nnz), KT(nnz);
  SBFWI_HIP(hipMemcpyAsync(K.data(), f->d.Kval, nnz * sizeof(double), hipMemcpyDeviceToHost, s));
  SBFWI_HIP(hipMemcpyAsync(KT.data(), f->d.KTval, nnz * sizeof(double), hipMemcpyDeviceToHost, s));
  SBFWI_HIP(hipStreamSynchronize(s));
  const int nS = ds->nS;
  const int64_t nmm = ds->mm_off[nS], nmb = ds->mb_off[nS];
  std::vector<double> Pn(nmm), Qn(nmm), Pt(nmm), Qt(nmm), Cn(nmb), En(nmb), Ct(nmb), Et(nmb);
  std::vector<std::vector<double>> upd(nS);
  std::vector<int64_t> loc(n, -1);
  for (int J = 0; J < nS; ++J) {
    const int64_t j0 = ds->sn_ptr[J], j1 = ds->sn_ptr[J + 1];
    const int nj = (int)(j1 - j0);
    const int64_t b0 = ds->b_ptr[J];
    const int nb = (int)(ds->b_ptr[J + 1] - b0);
    const int64_t mf = nj + nb;
    for (int64_t p = j0; p < j1; ++p) loc[p] = p - j0;
    for (int r = 0; r < nb; ++r) loc[ds->bpos[b0 + r]] = nj + r;
    std::vector<double> F((size_t)mf * mf, 0.0);   // row-major front
    for (int64_t p = j0; p < j1; ++p) {
      const int64_t v = ds->inv[p], lp = p - j0;
      for (int64_t q = m->h_row_ptr[v]; q < m->h_row_ptr[v + 1]; ++q) {
        const int64_t pc = ds->pos[m->h_col64[q]];
        if (pc < j0) continue;                    // belongs to a descendant's front
        const int64_t lc = loc[pc];
        if (lc < 0) return sbfwi_fail(SBFWI_EINVAL, "dissection structure misses a coupling");
        F[(size_t)lp * mf + lc] += K[q];          // row in J
        if (pc >= j1) F[(size_t)lc * mf + lp] += KT[q];   // column in J, row in B_J: K[c][v]
      }
    }
    for (int c : ds->children[J]) {
      const int64_t cb0 = ds->b_ptr[c];
      const int cnb = (int)(ds->b_ptr[c + 1] - cb0);
      const std::vector<double>& U = upd[c];
      for (int a = 0; a < cnb; ++a) {
        const int64_t la = loc[ds->bpos[cb0 + a]];
        for (int bb = 0; bb < cnb; ++bb) F[(size_t)la * mf + loc[ds->bpos[cb0 + bb]]] += U[(size_t)a * cnb + bb];
      }
      std::vector<double>().swap(upd[c]);
    }
    // eliminate the first nj pivots
    for (int k = 0; k < nj; ++k) {
      const double piv = F[(size_t)k * mf + k];
      if (!(std::fabs(piv) > 0.0) || !std::isfinite(piv))
        return sbfwi_fail(SBFWI_ESINGULAR, "coarse matrix: zero pivot in the direct factorisation");
      const double* rk = &F[(size_t)k * mf];
      for (int64_t i = k + 1; i < mf; ++i) {
        double* ri = &F[(size_t)i * mf];
        const double l = ri[k] / piv;
        ri[k] = l;
        if (l != 0.0)
          for (int64_t j = k + 1; j < mf; ++j) ri[j] -= l * rk[j];
      }
    }
    double* pn = &Pn[ds->mm_off[J]];
    double* qn = &Qn[ds->mm_off[J]];
    inv_unit_lower(F.data(), mf, nj, pn);
    inv_upper(F.data(), mf, nj, qn);
    double* pt = &Pt[ds->mm_off[J]];
    double* qt = &Qt[ds->mm_off[J]];
    for (int i = 0; i < nj; ++i)
      for (int k = 0; k < nj; ++k) {
        pt[(size_t)k * nj + i] = qn[(size_t)i * nj + k];   // (U11^-1)^T
        qt[(size_t)k * nj + i] = pn[(size_t)i * nj + k];   // (L11^-1)^T
      }
    double* cn = &Cn[ds->mb_off[J]];
    double* en = &En[ds->mb_off[J]];
    double* ct = &Ct[ds->mb_off[J]];
    double* et = &Et[ds->mb_off[J]];
    for (int r = 0; r < nb; ++r)
      for (int k = 0; k < nj; ++k) {
        const double l21 = F[(size_t)(nj + r) * mf + k];
        const double u12 = F[(size_t)k * mf + nj + r];
        cn[(size_t)k * nb + r] = l21;     // C = L21 (nb x nj)
        en[(size_t)r * nj + k] = u12;     // E = U12 (nj x nb)
        ct[(size_t)k * nb + r] = u12;     // C^T-solve = U12^T (nb x nj)
        et[(size_t)r * nj + k] = l21;     // E^T-solve = L21^T (nj x nb)
      }
    if (nb > 0) {
      std::vector<double>& U = upd[J];
      U.resize((size_t)nb * nb);
      for (int a = 0; a < nb; ++a)
        for (int bb = 0; bb < nb; ++bb) U[(size_t)a * nb + bb] = F[(size_t)(nj + a) * mf + nj + bb];
    }
    for (int64_t p = j0; p < j1; ++p) loc[p] = -1;
    for (int r = 0; r < nb; ++r) loc[ds->bpos[b0 + r]] = -1;
  }
  DirectNum* dn = new DirectNum();
  f->dnum = dn;
  SBFWI_CHECK(sbfwi_upload(&dn->P[0], Pn));
  SBFWI_CHECK(sbfwi_upload(&dn->C[0], Cn));
  SBFWI_CHECK(sbfwi_upload(&dn->Q[0], Qn));
  SBFWI_CHECK(sbfwi_upload(&dn->E[0], En));
  SBFWI_CHECK(sbfwi_upload(&dn->P[1], Pt));
  SBFWI_CHECK(sbfwi_upload(&dn->C[1], Ct));
  SBFWI_CHECK(sbfwi_upload(&dn->Q[1], Qt));
  SBFWI_CHECK(sbfwi_upload(&dn->E[1], Et));
  f->bytes += 8 * 4 * (nmm + nmb);
  return SBFWI_OK;
}

void sbfwi_direct_num_free(DirectNum* dn) {
  if (!dn) return;
  for (int t = 0; t < 2; ++t) {
    sbfwi_dev_free(dn->P[t]);
    sbfwi_dev_free(dn->C[t]);
    sbfwi_dev_free(dn->Q[t]);
    sbfwi_dev_free(dn->E[t]);
  }
  delete dn;
}

// ------------------------------------------------------------------ solve

int sbfwi_direct_solve(sbfwi_factors_s* f, CoarseWork* w, int transpose, const double* b, double* x,
                       hipStream_t s) {
  DirectSym* ds = f->m->dsym;
  DirectNum* dn = f->dnum;
  const int t = transpose ? 1 : 0;
  ProfScope ps(PK_SOLVE, s);
  for (int l = ds->depth; l >= 0; --l) {
    const int cnt = ds->lvl_ptr[l + 1] - ds->lvl_ptr[l];
    hipLaunchKernelGGL(fwd_level_kernel, dim3(cnt), dim3(DT), 0, s, ds->lvl_sn_dev + ds->lvl_ptr[l], ds->d,
                       dn->P[t], dn->C[t], w->NS, b, w->dtb, w->dyb, w->dcb, f->d.status);
  }
  for (int l = 0; l <= ds->depth; ++l) {
    const int cnt = ds->lvl_ptr[l + 1] - ds->lvl_ptr[l];
    hipLaunchKernelGGL(bwd_level_kernel, dim3(cnt), dim3(DT), 0, s, ds->lvl_sn_dev + ds->lvl_ptr[l], ds->d,
                       dn->Q[t], dn->E[t], w->NS, w->dyb, w->dtb, w->dxp, x);
  }
  hipLaunchKernelGGL(count_solve_kernel, dim3(1), dim3(64), 0, s, f->d.status);
  SBFWI_HIP(hipGetLastError());
  return SBFWI_OK;
}

extern "C" int sbfwi_direct_info(sbfwi_mesh m, int64_t* out) {
  if (!m || !out) return sbfwi_fail(SBFWI_EINVAL, "NULL argument");
  const DirectSym* ds = m->dsym;
  if (!ds) return sbfwi_fail(SBFWI_EINVAL, "mesh has no dissection order");
  out[0] = ds->nS;
  out[1] = ds->depth;
  out[2] = ds->max_nj;
  out[3] = ds->mm_off[ds->nS];
  out[4] = ds->mb_off[ds->nS];
  out[5] = ds->b_ptr[ds->nS];
  int64_t mx = 0;
  for (int l = 0; l <= ds->depth; ++l) mx = std::max<int64_t>(mx, ds->lvl_ptr[l + 1] - ds->lvl_ptr[l]);
  out[6] = mx;
  return SBFWI_OK;
}

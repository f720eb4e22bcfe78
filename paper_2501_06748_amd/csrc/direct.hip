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
// U12 = L11^-1 F12 and the update F22 - L21 U12 for J's parent.
//
// The device keeps, per supernode, two folded row blocks: forward
// FM_J = [P | -P Lrow_J] with P = L11^-1 and Lrow_J the rows of L that J's
// rows hold in the columns of earlier supernodes (its contributors), so that
// y_J = FM_J [b_J ; y_contributors]; backward BM_J = [Q | -Q U12] with
// Q = U11^-1, so that x_J = BM_J [y_J ; x_{B_J}].  K_g^T = U^T L^T has its own
// pair.  Every row of a block is one dot product of a dense row with values
// gathered at a column list.
//
// Solve (device): per level of the dissection tree one launch over all rows
// of that level's supernodes -- forward deepest level first, backward root
// first -- with the levels below the cut (where the tree has kSubtrees
// supernodes) solved by one block per subtree.  No atomics: results are
// bit-reproducible.
#include <algorithm>
#include <cmath>
#include <atomic>
#include <numeric>
#include <mutex>
#include <thread>

#include "sbfwi_internal.h"

namespace {

constexpr int kLeaf = 24;     // nodes per leaf supernode
constexpr int DT = 256;       // threads per block of the solve kernels
constexpr int kSubtrees = 512;// subtrees solved one per block at the bottom of the tree

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

// out[(J, i)] = sum_k M_J[i][k] src_k over the row of (J, i): the first n_J
// entries read the vector `own` at J's own positions (the right-hand side by
// node forward, y backward), the rest read `done` at the row's column list
// (the contributors' positions forward, B_J backward), values solved at
// earlier levels.  G lanes per row (G a power of two up to the block) split
// the entries lane-strided in chunks of U loads issued before their use; a
// fixed butterfly inside each wavefront, then (rows wider than a wavefront)
// the wavefronts of the row in index order, sum them.
template <int NSM, bool FWD>
__device__ __forceinline__ void row_dot(const DirectDev& d, const RowMeta& rm, bool valid, int lane, int G,
                                        const double* __restrict__ vals, int NS, const double* __restrict__ own,
                                        const double* __restrict__ done, double (&acc)[NSM]) {
  constexpr int U = NSM <= 4 ? 8 : 4;
#pragma unroll
  for (int s = 0; s < NSM; ++s) acc[s] = 0.0;
  if (valid) {
    const int64_t j0 = rm.j0, len = rm.len;
    const int nj = rm.nj;
    const double* v = vals + rm.val_off;
    const int64_t* cols = (FWD ? d.col_idx : d.bpos) + rm.col_off - nj;
    for (int64_t k0 = lane; k0 < len; k0 += (int64_t)G * U) {
      double a[U];
      const double* src[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t k = k0 + (int64_t)u * G;
        const bool ok = k < len;
        a[u] = ok ? v[k] : 0.0;
        if (FWD)   // own = the right-hand side by node: position j0 + k holds node inv[j0 + k]
          src[u] = !ok ? own : (k < nj ? own + d.inv[j0 + k] * NS : done + cols[k] * NS);
        else
          src[u] = !ok ? own + j0 * NS : (k < nj ? own + (j0 + k) * NS : done + cols[k] * NS);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int s = 0; s < NSM; ++s)
          if (s < NS) acc[s] += a[u] * src[u][s];
    }
  }
  const int gw = G < 64 ? G : 64;
  for (int m = 1; m < gw; m <<= 1)
#pragma unroll
    for (int s = 0; s < NSM; ++s) acc[s] += __shfl_xor(acc[s], m, 64);
}

template <int NSM, bool FWD>
__device__ __forceinline__ void row_store(const RowMeta& rm, int NS, const double (&acc)[NSM],
                                          double* __restrict__ out_pos, double* __restrict__ out_node,
                                          int* __restrict__ status) {
  bool bad = false;
  for (int s = 0; s < NS; ++s) {
    out_pos[rm.pos * NS + s] = acc[s];
    if (!FWD) out_node[rm.node * NS + s] = acc[s];
    bad = bad || !isfinite(acc[s]);
  }
  if (bad) atomicOr(&status[0], 4);
}

// out[(J, i)] = sum_k M_J[i][k] src_k over the row of (J, i): the first n_J
// entries read the vector `own` at J's own positions (the right-hand side by
// node forward, y backward), the rest read `done` at the row's column list
// (the contributors' positions forward, B_J backward), values solved at
// earlier levels.  G lanes per row (G a power of two up to the block) split
// the entries lane-strided in chunks of U loads issued before their use; a
// fixed butterfly inside each wavefront, then (rows wider than a wavefront)
// the wavefronts of the row in index order, sum them.  One launch per level.
template <int NSM, bool FWD>
__global__ void __launch_bounds__(DT) direct_rows_kernel(DirectDev d, int64_t row0, int64_t nrows, int G,
                                                         const double* __restrict__ vals, int NS,
                                                         const double* __restrict__ own,
                                                         const double* __restrict__ done,
                                                         double* __restrict__ out_pos,
                                                         double* __restrict__ out_node, int* __restrict__ status,
                                                         int count) {
  __shared__ double red[DT / 64][NSM];
  if (count && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&status[5], 1);   // solves done
  const int64_t gt = (int64_t)blockIdx.x * DT + threadIdx.x;
  const int64_t r = gt / G;
  const int lane = (int)(gt - r * G);
  const bool valid = r < nrows;
  RowMeta rm{};
  if (valid) rm = (FWD ? d.fwd_rows : d.bwd_rows)[row0 + r];   // one 48-byte load per row
  double acc[NSM];
  row_dot<NSM, FWD>(d, rm, valid, lane, G, vals, NS, own, done, acc);
  if (G > 64) {   // rows wider than a wavefront: add the row's wavefronts in index order
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
      for (int s = 0; s < NSM; ++s) red[wave][s] = acc[s];
    __syncthreads();
    if (lane == 0) {
      const int nw = G / 64;
#pragma unroll
      for (int s = 0; s < NSM; ++s) {
        double t = 0.0;
        for (int q = 0; q < nw; ++q) t += red[wave + q][s];
        acc[s] = t;
      }
    }
  }
  if (valid && lane == 0) row_store<NSM, FWD>(rm, NS, acc, out_pos, out_node, status);
}

// The bottom of the dissection tree: one block per subtree (rooted at the cut
// level) walks its levels in order -- deepest first forward, cut level first
// backward -- with a block barrier between levels instead of a launch; rows
// of a level use SG lanes each.
template <int NSM, bool FWD>
__global__ void __launch_bounds__(DT) direct_subtree_kernel(DirectDev d, const int64_t* __restrict__ seg, int NL,
                                                            const int64_t* __restrict__ sub_rows,
                                                            const double* __restrict__ vals, int NS,
                                                            const double* __restrict__ own,
                                                            const double* __restrict__ done,
                                                            double* __restrict__ out_pos,
                                                            double* __restrict__ out_node, int* __restrict__ status,
                                                            int count) {
  constexpr int SG = 16;
  if (count && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&status[5], 1);   // solves done
  const int64_t* sg = seg + (int64_t)blockIdx.x * (NL + 1);
  const int lane = threadIdx.x % SG;
  for (int q = 0; q < NL; ++q) {
    const int li = FWD ? q : NL - 1 - q;   // segment li holds the rows of the li-th deepest level
    const int64_t a = sg[li], e = sg[li + 1];
    for (int64_t base = a; base < e; base += DT / SG) {
      const int64_t r = base + threadIdx.x / SG;
      const bool valid = r < e;
      RowMeta rm{};
      if (valid) rm = (FWD ? d.fwd_rows : d.bwd_rows)[sub_rows[r]];
      double acc[NSM];
      row_dot<NSM, FWD>(d, rm, valid, lane, SG, vals, NS, own, done, acc);
      if (valid && lane == 0) row_store<NSM, FWD>(rm, NS, acc, out_pos, out_node, status);
    }
    __syncthreads();   // this level's results are read by the next level of the block
  }
}


// Runs fn(i) for i in [0, n) on up to `threads` host threads (dynamic assignment).
template <typename Fn>
void parallel_for(int64_t n, Fn&& fn) {
  int threads = (int)std::min<int64_t>(n, std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
  if (threads <= 1) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int64_t> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&] {
      for (int64_t i = next++; i < n; i = next++) fn(i);
    });
  for (auto& th : pool) th.join();
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
  ds->snp.assign(n, 0);
  for (int J = 0; J < nS; ++J)
    for (int64_t p = ds->sn_ptr[J]; p < ds->sn_ptr[J + 1]; ++p) ds->snp[p] = J;
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
  // contributors of every supernode: the descendants D whose B_D meets J (D ascending)
  ds->ctr.assign(nS, {});
  for (int D = 0; D < nS; ++D) {
    int last = -1;
    for (int64_t q = ds->b_ptr[D]; q < ds->b_ptr[D + 1]; ++q) {
      const int J = ds->sn_of(ds->bpos[q]);
      if (J != last) ds->ctr[J].push_back(D);   // bpos is sorted, so each J appears in one run
      last = J;
    }
  }
  for (auto& c : ds->ctr) {
    std::sort(c.begin(), c.end());
    c.erase(std::unique(c.begin(), c.end()), c.end());
  }
  // forward rows of J read its own nodes, then the positions of its contributors;
  // backward rows read J's positions, then B_J
  ds->ncols.assign(nS, 0);
  ds->cf_off.assign(nS + 1, 0);
  ds->fm_off.assign(nS + 1, 0);
  ds->bm_off.assign(nS + 1, 0);
  ds->max_nj = 0;
  for (int J = 0; J < nS; ++J) {
    const int64_t nj = ds->sn_ptr[J + 1] - ds->sn_ptr[J], nb = ds->b_ptr[J + 1] - ds->b_ptr[J];
    int64_t nc = 0;
    for (int D : ds->ctr[J]) nc += ds->sn_ptr[D + 1] - ds->sn_ptr[D];
    ds->ncols[J] = nc;
    ds->cf_off[J + 1] = ds->cf_off[J] + nc;
    ds->fm_off[J + 1] = ds->fm_off[J] + nj * (nj + nc);
    ds->bm_off[J + 1] = ds->bm_off[J] + nj * (nj + nb);
    ds->max_nj = std::max<int64_t>(ds->max_nj, nj);
  }
  ds->col_idx.assign(ds->cf_off[nS], 0);
  for (int J = 0; J < nS; ++J) {
    int64_t o = ds->cf_off[J];
    for (int D : ds->ctr[J])
      for (int64_t p = ds->sn_ptr[D]; p < ds->sn_ptr[D + 1]; ++p) ds->col_idx[o++] = p;
  }
  // levels: supernodes, their rows, and lanes per row from the longest row of the level
  ds->lvl_ptr.assign(ds->depth + 2, 0);
  for (int J = 0; J < nS; ++J) ds->lvl_ptr[ds->level[J] + 1]++;
  for (int l = 0; l <= ds->depth; ++l) ds->lvl_ptr[l + 1] += ds->lvl_ptr[l];
  ds->lvl_sn.assign(nS, 0);
  {
    std::vector<int32_t> fill(ds->lvl_ptr.begin(), ds->lvl_ptr.end() - 1);
    for (int J = 0; J < nS; ++J) ds->lvl_sn[fill[ds->level[J]]++] = J;
  }
  ds->row_ptr.assign(ds->depth + 2, 0);
  ds->g_fwd.assign(ds->depth + 1, 1);
  ds->g_bwd.assign(ds->depth + 1, 1);
  auto lanes = [](int64_t len) {
    int g = 1;
    while (g < DT && g * 16 < len) g *= 2;   // about 16 entries per lane, at most a block per row
    return g;
  };
  for (int l = 0; l <= ds->depth; ++l) {
    int64_t lf = 0, lb = 0;
    for (int q = ds->lvl_ptr[l]; q < ds->lvl_ptr[l + 1]; ++q) {
      const int J = ds->lvl_sn[q];
      const int64_t nj = ds->sn_ptr[J + 1] - ds->sn_ptr[J];
      for (int64_t i = 0; i < nj; ++i) {
        ds->row_sn.push_back(J);
        ds->row_i.push_back((int32_t)i);
      }
      lf = std::max(lf, nj + ds->ncols[J]);
      lb = std::max(lb, nj + ds->b_ptr[J + 1] - ds->b_ptr[J]);
    }
    ds->row_ptr[l + 1] = (int64_t)ds->row_sn.size();
    ds->g_fwd[l] = lanes(lf);
    ds->g_bwd[l] = lanes(lb);
  }
  // cut level: the shallowest level with at least kSubtrees supernodes; the
  // subtrees rooted there are solved by one block each
  ds->cut = ds->depth + 1;
  for (int l = 0; l <= ds->depth; ++l)
    if (ds->lvl_ptr[l + 1] - ds->lvl_ptr[l] >= kSubtrees) {
      ds->cut = l;
      break;
    }
  ds->n_sub = 0;
  ds->NL = ds->depth - ds->cut + 1;
  if (ds->cut <= ds->depth) {
    ds->n_sub = ds->lvl_ptr[ds->cut + 1] - ds->lvl_ptr[ds->cut];
    // row range of every supernode in the level-ordered row arrays
    std::vector<int64_t> first_row(nS, 0);
    for (int l = 0; l <= ds->depth; ++l) {
      int64_t r = ds->row_ptr[l];
      for (int q = ds->lvl_ptr[l]; q < ds->lvl_ptr[l + 1]; ++q) {
        const int J = ds->lvl_sn[q];
        first_row[J] = r;
        r += ds->sn_ptr[J + 1] - ds->sn_ptr[J];
      }
    }
    ds->seg.assign((size_t)ds->n_sub * (ds->NL + 1), 0);
    for (int b = 0; b < ds->n_sub; ++b) {
      const int R = ds->lvl_sn[ds->lvl_ptr[ds->cut] + b];
      std::vector<std::vector<int32_t>> by_level(ds->NL);   // index = depth - level
      std::vector<int32_t> stack{R};
      while (!stack.empty()) {
        const int J = stack.back();
        stack.pop_back();
        by_level[ds->depth - ds->level[J]].push_back(J);
        for (int c : ds->children[J]) stack.push_back(c);
      }
      for (int li = 0; li < ds->NL; ++li) {
        ds->seg[(size_t)b * (ds->NL + 1) + li] = (int64_t)ds->sub_rows.size();
        std::sort(by_level[li].begin(), by_level[li].end());
        for (int J : by_level[li])
          for (int64_t i = 0; i < ds->sn_ptr[J + 1] - ds->sn_ptr[J]; ++i) ds->sub_rows.push_back(first_row[J] + i);
      }
      ds->seg[(size_t)b * (ds->NL + 1) + ds->NL] = (int64_t)ds->sub_rows.size();
    }
  }
  const int64_t nrows = (int64_t)ds->row_sn.size();
  std::vector<RowMeta> fr(nrows), br(nrows);
  for (int64_t q = 0; q < nrows; ++q) {
    const int J = ds->row_sn[q], i = ds->row_i[q];
    const int64_t j0 = ds->sn_ptr[J], nj = ds->sn_ptr[J + 1] - j0, nb = ds->b_ptr[J + 1] - ds->b_ptr[J];
    RowMeta a{};
    a.j0 = j0;
    a.pos = j0 + i;
    a.node = ds->inv[j0 + i];
    a.nj = (int32_t)nj;
    a.len = (int32_t)(nj + ds->ncols[J]);
    a.val_off = ds->fm_off[J] + (int64_t)i * a.len;
    a.col_off = ds->cf_off[J];
    fr[q] = a;
    a.len = (int32_t)(nj + nb);
    a.val_off = ds->bm_off[J] + (int64_t)i * a.len;
    a.col_off = ds->b_ptr[J];
    br[q] = a;
  }
  DirectDev& d = ds->d;
  SBFWI_CHECK(sbfwi_upload(&d.inv, ds->inv));
  SBFWI_CHECK(sbfwi_upload(&d.sn_ptr, ds->sn_ptr));
  SBFWI_CHECK(sbfwi_upload(&d.b_ptr, ds->b_ptr));
  SBFWI_CHECK(sbfwi_upload(&d.bpos, ds->bpos));
  SBFWI_CHECK(sbfwi_upload(&d.ncols, ds->ncols));
  SBFWI_CHECK(sbfwi_upload(&d.cf_off, ds->cf_off));
  SBFWI_CHECK(sbfwi_upload(&d.col_idx, ds->col_idx));
  SBFWI_CHECK(sbfwi_upload(&d.fm_off, ds->fm_off));
  SBFWI_CHECK(sbfwi_upload(&d.bm_off, ds->bm_off));
  SBFWI_CHECK(sbfwi_upload(&d.fwd_rows, fr));
  SBFWI_CHECK(sbfwi_upload(&d.bwd_rows, br));
  if (ds->n_sub > 0) {
    SBFWI_CHECK(sbfwi_upload(&ds->seg_dev, ds->seg));
    SBFWI_CHECK(sbfwi_upload(&ds->sub_rows_dev, ds->sub_rows));
  }
  return SBFWI_OK;
}

void sbfwi_direct_sym_free(DirectSym* ds) {
  if (!ds) return;
  DirectDev& d = ds->d;
  void* ptrs[] = {d.inv, d.sn_ptr, d.b_ptr, d.bpos, d.ncols, d.cf_off, d.col_idx, d.fm_off, d.bm_off,
                  d.fwd_rows, d.bwd_rows, ds->seg_dev, ds->sub_rows_dev};
  for (void* p : ptrs) sbfwi_dev_free(p);
  delete ds;
}

// ------------------------------------------------------------------ numeric (per model)

namespace {

// Unit-lower-triangular inverse of the strictly-lower part of the leading n x n
// block of A (row-major, leading dimension lda) into row-major out (n x n).
void inv_unit_lower(const double* A, int64_t lda, int n, double* X) {
  std::fill(X, X + (size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    X[(size_t)j * n + j] = 1.0;
    for (int i = j + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s -= A[i * lda + k] * X[(size_t)k * n + j];
      X[(size_t)i * n + j] = s;
    }
  }
}

// Inverse of the upper triangle (with diagonal) of the leading n x n block of A.
void inv_upper(const double* A, int64_t lda, int n, double* X) {
  std::fill(X, X + (size_t)n * n, 0.0);
  for (int j = n - 1; j >= 0; --j) {
    X[(size_t)j * n + j] = 1.0 / A[j * lda + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= j; ++k) s -= A[i * lda + k] * X[(size_t)k * n + j];
      X[(size_t)i * n + j] = s / A[i * lda + i];
    }
  }
}

// Per-supernode results of the elimination (row-major): P = L11^-1, Q = U11^-1,
// L21 (nb x nj), U12 (nj x nb).
struct FrontOut {
  std::vector<double> P, Q, L21, U12, upd;
};

int eliminate_front(const DirectSym* ds, sbfwi_mesh_s* m, const std::vector<double>& K,
                    const std::vector<double>& KT, std::vector<FrontOut>& fo, int J, std::vector<int64_t>& loc) {
  const int64_t j0 = ds->sn_ptr[J], j1 = ds->sn_ptr[J + 1];
  const int nj = (int)(j1 - j0);
  const int64_t b0 = ds->b_ptr[J];
  const int nb = (int)(ds->b_ptr[J + 1] - b0);
  const int64_t mf = nj + nb;
  for (int64_t p = j0; p < j1; ++p) loc[p] = p - j0;
  for (int r = 0; r < nb; ++r) loc[ds->bpos[b0 + r]] = nj + r;
  int rc = SBFWI_OK;
  std::vector<double> F((size_t)mf * mf, 0.0);   // row-major front: rows and columns J then B_J
  for (int64_t p = j0; p < j1 && rc == SBFWI_OK; ++p) {
    const int64_t v = ds->inv[p], lp = p - j0;
    for (int64_t q = m->h_row_ptr[v]; q < m->h_row_ptr[v + 1]; ++q) {
      const int64_t pc = ds->pos[m->h_col64[q]];
      if (pc < j0) continue;                         // assembled in a descendant's front
      const int64_t lc = loc[pc];
      if (lc < 0) {
        rc = sbfwi_fail(SBFWI_EINVAL, "dissection structure misses a coupling");
        break;
      }
      F[(size_t)lp * mf + lc] += K[q];                // row in J
      if (pc >= j1) F[(size_t)lc * mf + lp] += KT[q]; // row in B_J, column in J: K[c][v]
    }
  }
  for (int c : ds->children[J]) {
    const int64_t cb0 = ds->b_ptr[c];
    const int cnb = (int)(ds->b_ptr[c + 1] - cb0);
    const std::vector<double>& U = fo[c].upd;
    for (int a = 0; a < cnb; ++a) {
      const int64_t la = loc[ds->bpos[cb0 + a]];
      for (int bb = 0; bb < cnb; ++bb) F[(size_t)la * mf + loc[ds->bpos[cb0 + bb]]] += U[(size_t)a * cnb + bb];
    }
    std::vector<double>().swap(fo[c].upd);
  }
  for (int64_t p = j0; p < j1; ++p) loc[p] = -1;
  for (int r = 0; r < nb; ++r) loc[ds->bpos[b0 + r]] = -1;
  if (rc != SBFWI_OK) return rc;
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
  FrontOut& o = fo[J];
  o.P.resize((size_t)nj * nj);
  o.Q.resize((size_t)nj * nj);
  inv_unit_lower(F.data(), mf, nj, o.P.data());
  inv_upper(F.data(), mf, nj, o.Q.data());
  o.L21.resize((size_t)nb * nj);
  o.U12.resize((size_t)nj * nb);
  for (int r = 0; r < nb; ++r)
    for (int k = 0; k < nj; ++k) {
      o.L21[(size_t)r * nj + k] = F[(size_t)(nj + r) * mf + k];
      o.U12[(size_t)k * nb + r] = F[(size_t)k * mf + nj + r];
    }
  o.upd.resize((size_t)nb * nb);
  for (int a = 0; a < nb; ++a)
    for (int bb = 0; bb < nb; ++bb) o.upd[(size_t)a * nb + bb] = F[(size_t)(nj + a) * mf + nj + bb];
  return SBFWI_OK;
}

// rows [r0, r1) of out = [A | -A R]: A (nj x nj), R (nj x nc), both row-major; out rows have nj + nc entries
void fold_rows(const double* A, const double* R, int nj, int64_t nc, int r0, int r1, double* out) {
  const int64_t len = nj + nc;
  for (int i = r0; i < r1; ++i) {
    double* o = out + (size_t)i * len;
    for (int k = 0; k < nj; ++k) o[k] = A[(size_t)i * nj + k];
    double* t = o + nj;
    for (int64_t c = 0; c < nc; ++c) t[c] = 0.0;
    for (int k = 0; k < nj; ++k) {
      const double a = A[(size_t)i * nj + k];
      if (a == 0.0) continue;
      const double* rk = R + (size_t)k * nc;
      for (int64_t c = 0; c < nc; ++c) t[c] -= a * rk[c];
    }
  }
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
  std::vector<FrontOut> fo(nS);
  // eliminate level by level from the leaves (the fronts of one level are independent)
  for (int l = ds->depth; l >= 0; --l) {
    const int q0 = ds->lvl_ptr[l], cnt = ds->lvl_ptr[l + 1] - q0;
    std::atomic<int> rc{SBFWI_OK};
    parallel_for(cnt, [&](int64_t q) {
      thread_local std::vector<int64_t> loc;
      if ((int64_t)loc.size() != n) loc.assign(n, -1);
      int r = eliminate_front(ds, m, K, KT, fo, ds->lvl_sn[q0 + q], loc);
      if (r != SBFWI_OK) rc = r;
    });
    if (rc != SBFWI_OK)   // the message was recorded on a worker thread
      return sbfwi_fail(rc.load(), rc == SBFWI_ESINGULAR ? "coarse matrix: zero pivot in the direct factorisation"
                                                         : "direct factorisation: dissection misses a coupling");
  }
  // folded row blocks: forward FM_J = [P_J | -P_J Lrow_J], backward BM_J = [Q_J | -Q_J U12_J]
  // and for K^T: [Q_J^T | -Q_J^T Lrow'_J], [P_J^T | -P_J^T L21_J^T]
  const int64_t nf = ds->fm_off[nS], nbm = ds->bm_off[nS];
  std::vector<double> FM(nf), BM(nbm), FMt(nf), BMt(nbm);
  struct Item {
    int J, r0, r1;
  };
  std::vector<Item> items;
  for (int J = 0; J < nS; ++J) {
    const int nj = (int)(ds->sn_ptr[J + 1] - ds->sn_ptr[J]);
    const int64_t work = (int64_t)nj * (nj + ds->ncols[J]);
    const int chunk = work > (1 << 16) ? std::max(1, (int)((1 << 16) / std::max<int64_t>(1, nj + ds->ncols[J]))) : nj;
    for (int r0 = 0; r0 < nj; r0 += chunk) items.push_back({J, r0, std::min(nj, r0 + chunk)});
  }
  // Lrow_J / Lrow'_J (nj x ncols): rows of the contributors' L21 (U12^T) that fall in J
  std::vector<std::vector<double>> lrow(nS), lrowt(nS);
  parallel_for(nS, [&](int64_t Jq) {
    const int J = (int)Jq;
    const int64_t j0 = ds->sn_ptr[J];
    const int nj = (int)(ds->sn_ptr[J + 1] - j0);
    const int64_t nc = ds->ncols[J];
    lrow[J].assign((size_t)nj * nc, 0.0);
    lrowt[J].assign((size_t)nj * nc, 0.0);
    int64_t c0 = 0;
    for (int D : ds->ctr[J]) {
      const int nd = (int)(ds->sn_ptr[D + 1] - ds->sn_ptr[D]);
      const int64_t db0 = ds->b_ptr[D];
      const int dnb = (int)(ds->b_ptr[D + 1] - db0);
      for (int k = 0; k < dnb; ++k) {
        const int64_t p = ds->bpos[db0 + k];
        if (p < j0 || p >= j0 + nj) continue;
        const int i = (int)(p - j0);
        for (int mm = 0; mm < nd; ++mm) {
          lrow[J][(size_t)i * nc + c0 + mm] = fo[D].L21[(size_t)k * nd + mm];
          lrowt[J][(size_t)i * nc + c0 + mm] = fo[D].U12[(size_t)mm * dnb + k];
        }
      }
      c0 += nd;
    }
  });
  parallel_for((int64_t)items.size(), [&](int64_t q) {
    const Item it = items[q];
    const int J = it.J;
    const int nj = (int)(ds->sn_ptr[J + 1] - ds->sn_ptr[J]);
    const int nb = (int)(ds->b_ptr[J + 1] - ds->b_ptr[J]);
    const int64_t nc = ds->ncols[J];
    const FrontOut& o = fo[J];
    std::vector<double> Pt((size_t)nj * nj), Qt((size_t)nj * nj), L21t((size_t)nj * nb);
    for (int i = 0; i < nj; ++i)
      for (int k = 0; k < nj; ++k) {
        Pt[(size_t)i * nj + k] = o.Q[(size_t)k * nj + i];   // (U11^-1)^T
        Qt[(size_t)i * nj + k] = o.P[(size_t)k * nj + i];   // (L11^-1)^T
      }
    for (int r = 0; r < nb; ++r)
      for (int k = 0; k < nj; ++k) L21t[(size_t)k * nb + r] = o.L21[(size_t)r * nj + k];
    fold_rows(o.P.data(), lrow[J].data(), nj, nc, it.r0, it.r1, &FM[ds->fm_off[J]]);
    fold_rows(Pt.data(), lrowt[J].data(), nj, nc, it.r0, it.r1, &FMt[ds->fm_off[J]]);
    fold_rows(o.Q.data(), o.U12.data(), nj, nb, it.r0, it.r1, &BM[ds->bm_off[J]]);
    fold_rows(Qt.data(), L21t.data(), nj, nb, it.r0, it.r1, &BMt[ds->bm_off[J]]);
  });
  DirectNum* dn = new DirectNum();
  f->dnum = dn;
  SBFWI_CHECK(sbfwi_upload(&dn->FM[0], FM));
  SBFWI_CHECK(sbfwi_upload(&dn->BM[0], BM));
  SBFWI_CHECK(sbfwi_upload(&dn->FM[1], FMt));
  SBFWI_CHECK(sbfwi_upload(&dn->BM[1], BMt));
  f->bytes += 8 * 2 * (nf + nbm);
  return SBFWI_OK;
}

void sbfwi_direct_num_free(DirectNum* dn) {
  if (!dn) return;
  for (int t = 0; t < 2; ++t) {
    sbfwi_dev_free(dn->FM[t]);
    sbfwi_dev_free(dn->BM[t]);
  }
  delete dn;
}

// ------------------------------------------------------------------ solve

namespace {

template <int NSM>
void launch_rows(bool fwd, DirectSym* ds, int l, const double* vals, int NS, const double* vin,
                 const double* vdone, double* out_pos, double* out_node, int* status, int count, hipStream_t s) {
  if (l < 0) {   // the subtree blocks below the cut level
    if (fwd)
      hipLaunchKernelGGL((direct_subtree_kernel<NSM, true>), dim3(ds->n_sub), dim3(DT), 0, s, ds->d, ds->seg_dev,
                         ds->NL, ds->sub_rows_dev, vals, NS, vin, vdone, out_pos, out_node, status, count);
    else
      hipLaunchKernelGGL((direct_subtree_kernel<NSM, false>), dim3(ds->n_sub), dim3(DT), 0, s, ds->d, ds->seg_dev,
                         ds->NL, ds->sub_rows_dev, vals, NS, vin, vdone, out_pos, out_node, status, count);
    return;
  }
  const int64_t r0 = ds->row_ptr[l], nr = ds->row_ptr[l + 1] - r0;
  const int G = fwd ? ds->g_fwd[l] : ds->g_bwd[l];
  const unsigned blocks = (unsigned)((nr * G + DT - 1) / DT);
  if (fwd)
    hipLaunchKernelGGL((direct_rows_kernel<NSM, true>), dim3(blocks), dim3(DT), 0, s, ds->d, r0, nr, G, vals, NS,
                       vin, vdone, out_pos, out_node, status, count);
  else
    hipLaunchKernelGGL((direct_rows_kernel<NSM, false>), dim3(blocks), dim3(DT), 0, s, ds->d, r0, nr, G, vals, NS,
                       vin, vdone, out_pos, out_node, status, count);
}

void launch_rows_ns(bool fwd, DirectSym* ds, int l, const double* vals, int NS, const double* vin,
                    const double* vdone, double* out_pos, double* out_node, int* status, int count, hipStream_t s) {
  if (NS == 1) launch_rows<1>(fwd, ds, l, vals, NS, vin, vdone, out_pos, out_node, status, count, s);
  else if (NS == 2) launch_rows<2>(fwd, ds, l, vals, NS, vin, vdone, out_pos, out_node, status, count, s);
  else if (NS <= 4) launch_rows<4>(fwd, ds, l, vals, NS, vin, vdone, out_pos, out_node, status, count, s);
  else if (NS <= 8) launch_rows<8>(fwd, ds, l, vals, NS, vin, vdone, out_pos, out_node, status, count, s);
  else launch_rows<16>(fwd, ds, l, vals, NS, vin, vdone, out_pos, out_node, status, count, s);
}

}  // namespace

int sbfwi_direct_solve(sbfwi_factors_s* f, CoarseWork* w, int transpose, const double* b, double* x,
                       hipStream_t s) {
  DirectSym* ds = f->m->dsym;
  DirectNum* dn = f->dnum;
  const int t = transpose ? 1 : 0;
  const int NS = w->NS;
  int* st = f->d.status;
  ProfScope ps(PK_SOLVE, s);
  const int top = std::min(ds->depth, ds->cut - 1);   // deepest level launched on its own
  // forward, deepest level first: y (by position) from b (by node) and the contributors' y;
  // the levels at and below the cut level run in one launch of subtree blocks (level -1)
  if (ds->n_sub > 0) launch_rows_ns(true, ds, -1, dn->FM[t], NS, b, w->dyb, w->dyb, nullptr, st, 0, s);
  for (int l = top; l >= 0; --l) launch_rows_ns(true, ds, l, dn->FM[t], NS, b, w->dyb, w->dyb, nullptr, st, 0, s);
  // backward, root first: x (by position and by node) from y and the solved B sets; the
  // last launch counts the solve
  for (int l = 0; l <= top; ++l)
    launch_rows_ns(false, ds, l, dn->BM[t], NS, w->dyb, w->dxp, w->dxp, x, st, ds->n_sub == 0 && l == top, s);
  if (ds->n_sub > 0) launch_rows_ns(false, ds, -1, dn->BM[t], NS, w->dyb, w->dxp, w->dxp, x, st, 1, s);
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
  out[3] = ds->fm_off[ds->nS];
  out[4] = ds->bm_off[ds->nS];
  out[5] = ds->b_ptr[ds->nS];
  int64_t mx = 0;
  for (int l = 0; l <= ds->depth; ++l) mx = std::max<int64_t>(mx, ds->lvl_ptr[l + 1] - ds->lvl_ptr[l]);
  out[6] = mx;
  return SBFWI_OK;
}

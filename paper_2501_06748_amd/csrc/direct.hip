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
// U12 = L11^-1 F12 and the update F22 - L21 U12 for J's parent.  Levels with
// many fronts take one host thread per front; the few large fronts near the
// root take every thread in turn (dense kernels in dense_host.cpp, with the
// textbook loops' operation order, so the factors do not depend on it).
//
// Solve (device, multifrontal).  Forward, L y = b, leaves first: with the
// children's update vectors u_c (over their B sets), the front vector of J is
// t_J = b_J - sum_c u_c[J] and y_J = P_J t_J with P_J = L11^-1; J passes on
// u_J = sum_c u_c[B_J] + C_J y_J with C_J = L21, so each supernode reads only
// its children.  The device keeps FW_J = [P_J ; C_J P_J] ((|J| + |B_J|) x |J|)
// and evaluates y_J and u_J - sum_c u_c[B_J] as FW_J t_J.  Backward, U x = y,
// root first: x_J = Q_J y_J - Q_J U12 x_{B_J} with Q_J = U11^-1 from
// BM_J = [Q_J | -Q_J U12] and the vector [y_J ; x_{B_J}].  K_g^T = U^T L^T
// uses the same structure with (U11^-T, U12^T) forward and (L11^-T, L21^T)
// backward.  One launch per level of the dissection tree above the cut level
// (the shallowest with kSubtrees supernodes), one block per subtree below it;
// every block assembles a supernode's vector in LDS once and then runs its
// rows against it.  No atomics: results are bit-reproducible.
#include <algorithm>
#include <memory>
#include <cmath>
#include <atomic>
#include <numeric>
#include <mutex>
#include <thread>

#include "dense_host.h"
#include "sbfwi_internal.h"

namespace {

constexpr int kLeaf = 24;     // nodes per leaf supernode
constexpr int DT = 256;       // threads per block of the solve kernels
constexpr int kSubtrees = 512;// subtrees solved one per block at the bottom of the tree
constexpr int kLevelU = 8;    // row values per lane in flight, level launches
constexpr int kSubtreeU = 16; // and subtree launches

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

// One block of a solve program.  For each of its steps: the slot records
// assemble vectors in LDS (forward: the right-hand side at the supernode's
// nodes minus the children's update entries of the slot; backward: y at J's
// positions, then x at B_J), then G lanes per row dot each dense row with its
// supernode's vector (lane-strided, chunks of U values per lane in flight: a
// whole row when it has at most U G entries; U = 8 for the level launches,
// 16 for the subtree launches, whose steps hold many short rows; a fixed
// butterfly to sum) and write it: forward to y by position (kind 0) or, plus
// the children's update entries of the row, to the update vector (kind 1);
// backward to x by position and by node.  A step costs three memory round
// trips: the step record; a thread's first slot record and first row record;
// then the row's values, its pass-through entries and the slot's entries of
// every shot, all requested before any is used.  A later pass of a subtree
// step loads its rows as it starts.  Shots s0 .. s0 + NSM - 1 of NS are
// handled.  A block barrier separates the steps, whose later ones read what
// earlier ones wrote.
template <int NSM, bool FWD, int U>
__global__ void __launch_bounds__(DT) direct_prog_kernel(DProgDev p, int64_t blk0, int64_t st0, int G,
                                                         const double* __restrict__ vals, int NS, int s0,
                                                         const double* __restrict__ in, double* __restrict__ upd,
                                                         double* __restrict__ out, int* __restrict__ status,
                                                         int count) {
  extern __shared__ double vec[];   // [slot][NSM]
  if (count && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&status[5], 1);   // solves done
  const int ns = min(NSM, NS - s0);
  const int lane = threadIdx.x % G;
  int64_t sa, sb;
  if (st0 >= 0) {
    sa = st0 + blockIdx.x;
    sb = sa + 1;
  } else {
    sa = p.blk[blk0 + blockIdx.x];
    sb = p.blk[blk0 + blockIdx.x + 1];
  }
  bool bad = false;
  for (int64_t st = sa; st < sb; ++st) {
    const DStep S = p.steps[st];
    DRRec rr{};
    // the pass-through entries are kept as loaded and added at the row's write, so
    // that no wait for them comes before the other loads of the step are issued
    // (not with 16 shots in a subtree launch's wide rows: the registers would not
    // leave two waves per SIMD)
    constexpr bool kDefer = NSM < 16 || U <= 8;
    constexpr int NP2 = kDefer ? NSM : 1;
    double a[U], pass[NSM], pass2[NP2];
    auto load_row = [&](int64_t r, DRRec& w, double (&x)[U], double (&ps)[NSM], double (&ps2)[NP2]) {
      w = r < S.r1 ? p.rrec[r] : DRRec{};
      const double* v = vals + w.val;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = lane + u * G;
        x[u] = k < w.len ? v[k] : 0.0;
      }
#pragma unroll
      for (int s = 0; s < NSM; ++s) ps[s] = 0.0;
#pragma unroll
      for (int s = 0; s < NP2; ++s) ps2[s] = 0.0;
      if (FWD && lane == 0 && w.ngl > 0) {
        // every shot's entries are loaded before any is used (shots past ns reread shot
        // s0, a second entry is read again from the first when there is none), so that
        // the loads are in flight together
        const int64_t g1 = w.ngl > 1 ? w.g1 : w.g0;
        double t0[NSM], t1[NSM];
#pragma unroll
        for (int s = 0; s < NSM; ++s) {
          t0[s] = upd[w.g0 * NS + s0 + (s < ns ? s : 0)];
          t1[s] = upd[g1 * NS + s0 + (s < ns ? s : 0)];
        }
        if constexpr (kDefer) {
#pragma unroll
          for (int s = 0; s < NSM; ++s) {
            ps[s] = t0[s];
            ps2[s] = t1[s];
          }
        } else {
          const bool two = w.ngl > 1;
#pragma unroll
          for (int s = 0; s < NSM; ++s) {   // selects, not branches: both loads are used
            const double p1 = ps[s] + t0[s], p2 = p1 + t1[s];
            ps[s] = s < ns ? (two ? p2 : p1) : ps[s];
          }
        }
      }
    };
    // this thread's first slot record is requested with the first row record, before
    // the row's values, so that the gather's entries and the row's values are in
    // flight together
    const int64_t q0 = S.v0 + threadIdx.x;
    const DVRec v0 = p.vrec[q0 < S.v1 ? q0 : S.v0];
    load_row(S.r0 + threadIdx.x / G, rr, a, pass, pass2);
    for (int64_t q = q0; q < S.v1; q += DT) {
      const DVRec v = q == q0 ? v0 : p.vrec[q];
      double acc[NSM];
      const double* src = FWD ? in : (v.ngl ? upd : in);
      // as in load_row: every load issued before any value is used (a missing
      // child entry reads entry 0, which always exists, and is not used)
      double t[NSM];
#pragma unroll
      for (int s = 0; s < NSM; ++s) t[s] = src[v.src * NS + s0 + (s < ns ? s : 0)];
      if (FWD) {
        const int64_t g0 = v.ngl > 0 ? v.g0 : 0, g1 = v.ngl > 1 ? v.g1 : g0;
        double t0[NSM], t1[NSM];
#pragma unroll
        for (int s = 0; s < NSM; ++s) {
          t0[s] = upd[g0 * NS + s0 + (s < ns ? s : 0)];
          t1[s] = upd[g1 * NS + s0 + (s < ns ? s : 0)];
        }
#pragma unroll
        for (int s = 0; s < NSM; ++s) {
          const double a1 = t[s] - t0[s], a2 = a1 - t1[s];
          acc[s] = s < ns ? (v.ngl > 1 ? a2 : (v.ngl > 0 ? a1 : t[s])) : 0.0;
        }
      } else {
#pragma unroll
        for (int s = 0; s < NSM; ++s) acc[s] = s < ns ? t[s] : 0.0;
      }
#pragma unroll
      for (int s = 0; s < NSM; ++s) vec[v.slot * NSM + s] = acc[s];
    }
    __syncthreads();
    for (int64_t base = S.r0; base < S.r1; base += DT / G) {
      const int64_t r = base + threadIdx.x / G;
      const bool valid = r < S.r1;
      // a later pass loads its rows here (a level launch's block has one pass)
      if (base != S.r0) load_row(r, rr, a, pass, pass2);
      double acc[NSM];
#pragma unroll
      for (int s = 0; s < NSM; ++s) acc[s] = 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = lane + u * G;
        if (k < rr.len) {
          const double* x = vec + (int64_t)(rr.slot0 + k) * NSM;
#pragma unroll
          for (int s = 0; s < NSM; ++s) acc[s] += a[u] * x[s];
        }
      }
      const double* v = vals + rr.val;
      for (int k0 = lane + G * U; k0 < rr.len; k0 += G * U) {
        double b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int k = k0 + u * G;
          b[u] = k < rr.len ? v[k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int k = k0 + u * G;
          if (k < rr.len) {
            const double* x = vec + (int64_t)(rr.slot0 + k) * NSM;
#pragma unroll
            for (int s = 0; s < NSM; ++s) acc[s] += b[u] * x[s];
          }
        }
      }
      for (int m = 1; m < G; m <<= 1)
#pragma unroll
        for (int s = 0; s < NSM; ++s) acc[s] += __shfl_xor(acc[s], m, 64);
      if (valid && lane == 0) {
        if (FWD) {
          if (rr.kind == 0) {
#pragma unroll
            for (int s = 0; s < NSM; ++s)
              if (s < ns) out[rr.out * NS + s0 + s] = acc[s];
          } else {
#pragma unroll
            for (int s = 0; s < NSM; ++s) {
              double add = pass[s];
              if constexpr (kDefer) {   // the running sum load_row forms otherwise: (0 + e0) + e1
                const double p1 = 0.0 + pass[s], p2 = p1 + pass2[s];
                add = rr.ngl > 1 ? p2 : (rr.ngl > 0 ? p1 : 0.0);
              }
              acc[s] += add;
              if (s < ns) upd[rr.out * NS + s0 + s] = acc[s];
            }
          }
        } else {
#pragma unroll
          for (int s = 0; s < NSM; ++s)
            if (s < ns) {
              upd[rr.out * NS + s0 + s] = acc[s];
              out[rr.g0 * NS + s0 + s] = acc[s];
            }
        }
#pragma unroll
        for (int s = 0; s < NSM; ++s) bad = bad || (s < ns && !isfinite(acc[s]));
      }
    }
    __syncthreads();   // the next step reads this one's results and reuses the LDS vectors
  }
  if (bad) atomicOr(&status[0], 4);
}


// Runs fn(i) for i in [0, n) on up to `threads` host threads (dynamic assignment).
template <typename Fn>
void parallel_for(int64_t n, Fn&& fn) {
  int threads = (int)std::min<int64_t>(n, dense_threads());
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
  // row blocks: forward FW_J (|J| + |B_J|) x |J|, backward BM_J |J| x (|J| + |B_J|)
  ds->fw_off.assign(nS + 1, 0);
  ds->bm_off.assign(nS + 1, 0);
  std::vector<int64_t>& fr_off = ds->fr_off;   // front rows (J then B_J) of every supernode
  fr_off.assign(nS + 1, 0);
  for (int J = 0; J < nS; ++J) {
    const int64_t nj = ds->sn_ptr[J + 1] - ds->sn_ptr[J], nb = ds->b_ptr[J + 1] - ds->b_ptr[J];
    ds->fw_off[J + 1] = ds->fw_off[J] + (nj + nb) * nj;
    ds->bm_off[J + 1] = ds->bm_off[J] + nj * (nj + nb);
    fr_off[J + 1] = fr_off[J] + nj + nb;
    ds->max_nj = std::max<int64_t>(ds->max_nj, nj);
    ds->sum_j2 += nj * nj;
    ds->sum_jb += nj * nb;
  }
  // the children's update entries that land in each front row of J (B_c lies in J and B_J),
  // listed child by child
  std::vector<int64_t>& gl_ptr = ds->gl_ptr;
  std::vector<int64_t>& gl = ds->gl;
  gl_ptr.assign(fr_off[nS] + 1, 0);
  gl.clear();
  auto front_row = [&](int J, int64_t p) -> int64_t {   // front row of position p in J, or -1
    const int64_t j0 = ds->sn_ptr[J], j1 = ds->sn_ptr[J + 1];
    if (p >= j0 && p < j1) return p - j0;
    const auto b0 = ds->bpos.begin() + ds->b_ptr[J], b1 = ds->bpos.begin() + ds->b_ptr[J + 1];
    const auto it = std::lower_bound(b0, b1, p);
    return (it != b1 && *it == p) ? (j1 - j0) + (it - b0) : -1;
  };
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int64_t> fill;
    if (pass == 1) {
      for (int64_t r = 0; r < fr_off[nS]; ++r) gl_ptr[r + 1] += gl_ptr[r];
      gl.assign(gl_ptr[fr_off[nS]], 0);
      fill.assign(gl_ptr.begin(), gl_ptr.end() - 1);
    }
    for (int J = 0; J < nS; ++J)
      for (int c : ds->children[J])
        for (int64_t k = ds->b_ptr[c]; k < ds->b_ptr[c + 1]; ++k) {
          const int64_t fr = front_row(J, ds->bpos[k]);
          if (fr < 0) return sbfwi_fail(SBFWI_EINVAL, "nested dissection: a child's coupling leaves its parent's front");
          if (pass == 0) gl_ptr[fr_off[J] + fr + 1]++;
          else gl[fill[fr_off[J] + fr]++] = k;
        }
  }
  // levels
  ds->lvl_ptr.assign(ds->depth + 2, 0);
  for (int J = 0; J < nS; ++J) ds->lvl_ptr[ds->level[J] + 1]++;
  for (int l = 0; l <= ds->depth; ++l) ds->lvl_ptr[l + 1] += ds->lvl_ptr[l];
  ds->lvl_sn.assign(nS, 0);
  {
    std::vector<int32_t> fill(ds->lvl_ptr.begin(), ds->lvl_ptr.end() - 1);
    for (int J = 0; J < nS; ++J) ds->lvl_sn[fill[ds->level[J]]++] = J;
  }
  return sbfwi_direct_programs(m, kSubtrees);
}

// Solve programs of the mesh's dissection with the subtree launches cut at the
// shallowest level that has at least min_subtrees supernodes (none if no level
// has that many); replaces programs built before.
int sbfwi_direct_programs(sbfwi_mesh_s* m, int min_subtrees) {
  DirectSym* ds = m->dsym;
  if (!ds) return sbfwi_fail(SBFWI_EINVAL, "mesh has no dissection order");
  if (min_subtrees < 1) return sbfwi_fail(SBFWI_EINVAL, "the subtree cut needs at least 1 supernode per level");
  const int64_t n = m->n_nodes;
  const int nS = ds->nS;
  const std::vector<int64_t>& fr_off = ds->fr_off;
  const std::vector<int64_t>& gl_ptr = ds->gl_ptr;
  const std::vector<int64_t>& gl = ds->gl;
  for (int t = 0; t < 2; ++t) {
    sbfwi_dev_free(ds->prog[t].vrec);
    sbfwi_dev_free(ds->prog[t].rrec);
    sbfwi_dev_free(ds->prog[t].steps);
    sbfwi_dev_free(ds->prog[t].blk);
    ds->prog[t] = DProgDev();
    ds->launches[t].clear();
  }
  ds->max_slots = 0;
  // cut level: the shallowest level with at least min_subtrees supernodes; the
  // subtrees rooted there are solved by one block each
  ds->cut = ds->depth + 1;
  for (int l = 0; l <= ds->depth; ++l)
    if (ds->lvl_ptr[l + 1] - ds->lvl_ptr[l] >= min_subtrees) {
      ds->cut = l;
      break;
    }
  ds->n_sub = ds->cut <= ds->depth ? ds->lvl_ptr[ds->cut + 1] - ds->lvl_ptr[ds->cut] : 0;
  const int top = std::min(ds->depth, ds->cut - 1);   // deepest level with a launch of its own
  // programs (t = 0 forward, 1 backward)
  struct Prog {
    std::vector<DVRec> v;
    std::vector<DRRec> r;
    std::vector<DStep> st;
    std::vector<int64_t> blk{0};
  } P[2];
  auto lanes = [](int64_t len, int per_lane) {   // per_lane entries per lane, at most a wavefront per row
    int g = 1;
    while (g < 64 && g * per_lane < len) g *= 2;
    return g;
  };
  auto nrows = [&](int t, int J) {
    const int64_t nj = ds->sn_ptr[J + 1] - ds->sn_ptr[J];
    return t == 0 ? nj + ds->b_ptr[J + 1] - ds->b_ptr[J] : nj;
  };
  auto row_len = [&](int t, int J) {
    const int64_t nj = ds->sn_ptr[J + 1] - ds->sn_ptr[J];
    return t == 0 ? nj : nj + ds->b_ptr[J + 1] - ds->b_ptr[J];
  };
  auto emit_slots = [&](int t, int J, int base) -> int {   // J's vector at LDS slots base ..
    const int64_t j0 = ds->sn_ptr[J], nj = ds->sn_ptr[J + 1] - j0, b0 = ds->b_ptr[J];
    const int64_t nb = ds->b_ptr[J + 1] - b0;
    for (int64_t i = 0; i < nj; ++i) {
      DVRec v{};
      v.slot = base + (int32_t)i;
      if (t == 0) {
        v.src = ds->inv[j0 + i];
        const int64_t g = gl_ptr[fr_off[J] + i];
        v.ngl = (int32_t)(gl_ptr[fr_off[J] + i + 1] - g);
        v.g0 = v.ngl > 0 ? gl[g] : 0;
        v.g1 = v.ngl > 1 ? gl[g + 1] : 0;
      } else {
        v.src = j0 + i;
      }
      P[t].v.push_back(v);
    }
    if (t == 1)
      for (int64_t r = 0; r < nb; ++r) {
        DVRec v{};
        v.src = ds->bpos[b0 + r];
        v.ngl = 1;
        v.slot = base + (int32_t)(nj + r);
        P[t].v.push_back(v);
      }
    return (int)(t == 0 ? nj : nj + nb);
  };
  auto emit_rows = [&](int t, int J, int base, int64_t r0, int64_t r1) {
    const int64_t j0 = ds->sn_ptr[J], nj = ds->sn_ptr[J + 1] - j0, nb = ds->b_ptr[J + 1] - ds->b_ptr[J];
    for (int64_t r = r0; r < r1; ++r) {
      DRRec w{};
      w.slot0 = base;
      if (t == 0) {
        w.val = ds->fw_off[J] + r * nj;
        w.len = (int32_t)nj;
        if (r < nj) {
          w.out = j0 + r;
        } else {
          w.kind = 1;
          w.out = ds->b_ptr[J] + (r - nj);
          const int64_t g = gl_ptr[fr_off[J] + r];
          w.ngl = (int32_t)(gl_ptr[fr_off[J] + r + 1] - g);
          w.g0 = w.ngl > 0 ? gl[g] : 0;
          w.g1 = w.ngl > 1 ? gl[g + 1] : 0;
        }
      } else {
        w.val = ds->bm_off[J] + r * (nj + nb);
        w.len = (int32_t)(nj + nb);
        w.out = j0 + r;
        w.g0 = ds->inv[j0 + r];
      }
      P[t].r.push_back(w);
    }
  };
  auto level_launch = [&](int t, int l) {   // one block per (supernode, slice of its rows)
    DLaunch L;
    L.blk0 = (int64_t)P[t].blk.size() - 1;
    int64_t len = 1;
    for (int q = ds->lvl_ptr[l]; q < ds->lvl_ptr[l + 1]; ++q) len = std::max(len, row_len(t, ds->lvl_sn[q]));
    L.G = lanes(len, kLevelU);
    L.st0 = (int64_t)P[t].st.size();
    const int64_t per = DT / L.G;   // one pass of rows per block
    for (int q = ds->lvl_ptr[l]; q < ds->lvl_ptr[l + 1]; ++q) {
      const int J = ds->lvl_sn[q];
      const int64_t v0 = (int64_t)P[t].v.size();
      L.slots = std::max(L.slots, emit_slots(t, J, 0));
      const int64_t v1 = (int64_t)P[t].v.size(), nr = nrows(t, J);
      for (int64_t a = 0; a < nr; a += per) {
        const int64_t r0 = (int64_t)P[t].r.size();
        emit_rows(t, J, 0, a, std::min(nr, a + per));
        P[t].st.push_back({v0, v1, r0, (int64_t)P[t].r.size()});
        P[t].blk.push_back((int64_t)P[t].st.size());
      }
    }
    L.nblk = (int64_t)P[t].blk.size() - 1 - L.blk0;
    ds->launches[t].push_back(L);
  };
  auto subtree_launch = [&](int t) {   // one block per subtree rooted at the cut level
    DLaunch L;
    L.blk0 = (int64_t)P[t].blk.size() - 1;
    const int NL = ds->depth - ds->cut + 1;
    int64_t len = 1;
    for (int b = 0; b < ds->n_sub; ++b) {
      std::vector<std::vector<int32_t>> by_level(NL);   // index = depth - level
      std::vector<int32_t> stack{ds->lvl_sn[ds->lvl_ptr[ds->cut] + b]};
      while (!stack.empty()) {
        const int J = stack.back();
        stack.pop_back();
        by_level[ds->depth - ds->level[J]].push_back(J);
        for (int c : ds->children[J]) stack.push_back(c);
      }
      for (int q = 0; q < NL; ++q) {
        const int li = t == 0 ? q : NL - 1 - q;   // forward deepest first, backward cut level first
        if (by_level[li].empty()) continue;
        std::sort(by_level[li].begin(), by_level[li].end());
        const int64_t v0 = (int64_t)P[t].v.size();
        std::vector<int> base;
        int slots = 0;
        for (int J : by_level[li]) {
          base.push_back(slots);
          slots += emit_slots(t, J, slots);
        }
        const int64_t v1 = (int64_t)P[t].v.size(), r0 = (int64_t)P[t].r.size();
        for (size_t k = 0; k < by_level[li].size(); ++k) {
          const int J = by_level[li][k];
          emit_rows(t, J, base[k], 0, nrows(t, J));
          len = std::max(len, row_len(t, J));
        }
        P[t].st.push_back({v0, v1, r0, (int64_t)P[t].r.size()});
        L.slots = std::max(L.slots, slots);
      }
      P[t].blk.push_back((int64_t)P[t].st.size());
    }
    L.G = lanes(len, kSubtreeU);
    L.nblk = ds->n_sub;
    ds->launches[t].push_back(L);
  };
  if (ds->n_sub > 0) subtree_launch(0);
  for (int l = top; l >= 0; --l) level_launch(0, l);
  for (int l = 0; l <= top; ++l) level_launch(1, l);
  if (ds->n_sub > 0) subtree_launch(1);
  for (int t = 0; t < 2; ++t)
    for (DLaunch& L : ds->launches[t]) {
      ds->max_slots = std::max(ds->max_slots, L.slots);
      for (int64_t b = L.blk0; b < L.blk0 + L.nblk; ++b)
        for (int64_t q = P[t].blk[b]; q < P[t].blk[b + 1]; ++q) {
          const DStep& S = P[t].st[q];
          L.steps++;
          L.rows += S.r1 - S.r0;
          L.vrecs += S.v1 - S.v0;
          L.max_step_rows = std::max(L.max_step_rows, S.r1 - S.r0);
        }
    }
  // every record stays inside the arrays and LDS vectors it addresses
  const int64_t n_upd = ds->b_ptr[nS];
  for (int t = 0; t < 2; ++t) {
    const int64_t vals = t == 0 ? ds->fw_off[nS] : ds->bm_off[nS];
    bool ok = true;
    int64_t blocks = 0;
    for (const DLaunch& L : ds->launches[t]) {
      ok = ok && L.blk0 == blocks && L.nblk >= 0 && L.blk0 + L.nblk < (int64_t)P[t].blk.size();
      for (int64_t b = L.blk0; ok && L.st0 >= 0 && b < L.blk0 + L.nblk; ++b)   // single-step blocks
        ok = P[t].blk[b] == L.st0 + (b - L.blk0) && P[t].blk[b + 1] == P[t].blk[b] + 1;
      blocks += L.nblk;
      for (int64_t b = L.blk0; ok && b < L.blk0 + L.nblk; ++b)
        for (int64_t q = P[t].blk[b]; ok && q < P[t].blk[b + 1]; ++q) {
          const DStep& S = P[t].st[q];
          ok = S.v0 <= S.v1 && S.v1 <= (int64_t)P[t].v.size() && S.r0 <= S.r1 && S.r1 <= (int64_t)P[t].r.size();
          for (int64_t i = S.v0; ok && i < S.v1; ++i) {
            const DVRec& v = P[t].v[i];
            ok = v.src >= 0 && v.src < n && v.slot >= 0 && v.slot < L.slots &&
                 (t == 1 ? (v.ngl == 0 || v.ngl == 1)
                         : (v.ngl >= 0 && v.ngl <= 2 && (v.ngl < 1 || (v.g0 >= 0 && v.g0 < n_upd)) &&
                            (v.ngl < 2 || (v.g1 >= 0 && v.g1 < n_upd))));
          }
          for (int64_t i = S.r0; ok && i < S.r1; ++i) {
            const DRRec& w = P[t].r[i];
            ok = w.len >= 0 && w.val >= 0 && w.val + w.len <= vals && w.slot0 >= 0 && w.slot0 + w.len <= L.slots;
            if (t == 1) ok = ok && w.out >= 0 && w.out < n && w.g0 >= 0 && w.g0 < n;
            else if (w.kind == 0) ok = ok && w.out >= 0 && w.out < n;
            else
              ok = ok && w.out >= 0 && w.out < n_upd && w.ngl >= 0 && w.ngl <= 2 &&
                   (w.ngl < 1 || (w.g0 >= 0 && w.g0 < n_upd)) && (w.ngl < 2 || (w.g1 >= 0 && w.g1 < n_upd));
          }
        }
    }
    if (!ok || blocks + 1 != (int64_t)P[t].blk.size())
      return sbfwi_fail(SBFWI_EINVAL, "direct solve program out of bounds (internal error)");
  }
  for (int t = 0; t < 2; ++t) {
    SBFWI_CHECK(sbfwi_upload(&ds->prog[t].vrec, P[t].v));
    SBFWI_CHECK(sbfwi_upload(&ds->prog[t].rrec, P[t].r));
    SBFWI_CHECK(sbfwi_upload(&ds->prog[t].steps, P[t].st));
    SBFWI_CHECK(sbfwi_upload(&ds->prog[t].blk, P[t].blk));
  }
  return SBFWI_OK;
}

void sbfwi_direct_sym_free(DirectSym* ds) {
  if (!ds) return;
  for (int t = 0; t < 2; ++t) {
    sbfwi_dev_free(ds->prog[t].vrec);
    sbfwi_dev_free(ds->prog[t].rrec);
    sbfwi_dev_free(ds->prog[t].steps);
    sbfwi_dev_free(ds->prog[t].blk);
  }
  delete ds;
}

// ------------------------------------------------------------------ numeric (per model)

namespace {

// Per-supernode results of the elimination (row-major): P = L11^-1, Q = U11^-1,
// L21 (nb x nj), U12 (nj x nb).
struct FrontOut {
  std::vector<double> P, Q, L21, U12, upd;
};

// Assembles and eliminates the front of J; the dense work is shared among the
// team's threads (team may be null).
int eliminate_front(const DirectSym* ds, sbfwi_mesh_s* m, const std::vector<double>& K,
                    const std::vector<double>& KT, std::vector<FrontOut>& fo, int J, std::vector<int64_t>& loc,
                    DenseTeam* team) {
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
  if (dense_lu(F.data(), mf, nj, team) >= 0)
    return sbfwi_fail(SBFWI_ESINGULAR, "coarse matrix: zero pivot in the direct factorisation");
  FrontOut& o = fo[J];
  o.P.assign((size_t)nj * nj, 0.0);
  o.Q.assign((size_t)nj * nj, 0.0);
  const int T = team ? team->size() : 1;
  auto invert = [&](int t) {   // P = L11^-1 and Q = U11^-1, blocks of 16 columns dealt round the threads
    for (int c0 = 16 * t; c0 < nj; c0 += 16 * T) {
      const int c1 = std::min(nj, c0 + 16);
      dense_inv_unit_lower(F.data(), mf, nj, o.P.data(), c0, c1);
      dense_inv_upper(F.data(), mf, nj, o.Q.data(), c0, c1);
    }
  };
  if (T > 1)
    team->run(invert);
  else
    invert(0);
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

// Eliminates the fronts level by level from the leaves (the fronts of one
// level are independent).
int eliminate_levels(const DirectSym* ds, sbfwi_mesh_s* m, const std::vector<double>& K,
                     const std::vector<double>& KT, std::vector<FrontOut>& fo) {
  const int64_t n = m->n_nodes;
  const int T = dense_threads();
  std::unique_ptr<DenseTeam> team;
  std::vector<int64_t> team_loc;
  for (int l = ds->depth; l >= 0; --l) {
    const int q0 = ds->lvl_ptr[l], cnt = ds->lvl_ptr[l + 1] - q0;
    if (cnt <= 4 && 2 * cnt <= T) {   // a few fronts (near the root, the largest): one at a time, every thread on it
      if (!team) {
        team.reset(new DenseTeam(T));
        team_loc.assign(n, -1);
      }
      for (int q = q0; q < q0 + cnt; ++q) SBFWI_CHECK(eliminate_front(ds, m, K, KT, fo, ds->lvl_sn[q], team_loc, team.get()));
      continue;
    }
    // many fronts: one thread per front
    std::atomic<int> rc{SBFWI_OK};
    parallel_for(cnt, [&](int64_t q) {
      thread_local std::vector<int64_t> loc;
      if ((int64_t)loc.size() != n) loc.assign(n, -1);
      int r = eliminate_front(ds, m, K, KT, fo, ds->lvl_sn[q0 + q], loc, nullptr);
      if (r != SBFWI_OK) rc = r;
    });
    if (rc != SBFWI_OK)   // the message was recorded on a worker thread
      return sbfwi_fail(rc.load(), rc == SBFWI_ESINGULAR ? "coarse matrix: zero pivot in the direct factorisation"
                                                         : "direct factorisation: dissection misses a coupling");
  }
  return SBFWI_OK;
}

// Row blocks of every supernode, K_g (index 0) and K_g^T (index 1), in host
// buffers (not initialised: every entry is written once).
struct RowBlocks {
  std::unique_ptr<double[]> fw[2], bm[2];
  int64_t nfw = 0, nbm = 0;
};

// Row blocks from the eliminated fronts: forward FW_J = [P_J ; L21_J P_J] and
// FW^t_J = [Q_J^T ; U12_J^T Q_J^T]; backward BM_J = [Q_J | -Q_J U12_J] and
// BM^t_J = [P_J^T | -P_J^T L21_J^T].  The right blocks of BM_J and BM^t_J are
// the negated transposes of the lower blocks of FW^t_J and FW_J: each entry
// takes the same products in the same order (a running sum from zero, steps
// with a zero factor skipped), and 0 - s equals the running difference from
// zero bit for bit.  The work is cut into tasks of a few rows each (the fronts
// near the root hold most of it), largest first; every row is formed as a
// whole by one task.
void row_blocks(const DirectSym* ds, const std::vector<FrontOut>& fo, RowBlocks& rb) {
  const int nS = ds->nS;
  rb.nfw = ds->fw_off[nS];
  rb.nbm = ds->bm_off[nS];
  for (int t = 0; t < 2; ++t) {
    rb.fw[t].reset(new double[std::max<int64_t>(rb.nfw, 1)]);
    rb.bm[t].reset(new double[std::max<int64_t>(rb.nbm, 1)]);
  }
  auto nj_of = [&](int J) { return (int)(ds->sn_ptr[J + 1] - ds->sn_ptr[J]); };
  auto nb_of = [&](int J) { return (int)(ds->b_ptr[J + 1] - ds->b_ptr[J]); };
  struct Task {
    int J, r0, r1;
    int64_t cost;
  };
  constexpr int64_t kTaskWork = 1 << 17;   // multiply-adds (or moves) per task, about
  auto make_tasks = [&](bool products) {
    std::vector<Task> tasks;
    for (int J = 0; J < nS; ++J) {
      const int nj = nj_of(J), nb = nb_of(J);
      const int rows = products ? nb : nj;
      const int64_t row_cost = products ? 2 * (int64_t)nj * nj : 2 * (int64_t)(nj + nb);
      const int chunk = (int)std::max<int64_t>(1, kTaskWork / std::max<int64_t>(row_cost, 1));
      for (int r = 0; r < rows; r += chunk) {
        const int r1 = std::min(rows, r + chunk);
        tasks.push_back({J, r, r1, row_cost * (r1 - r)});
      }
    }
    std::stable_sort(tasks.begin(), tasks.end(), [](const Task& a, const Task& b) { return a.cost > b.cost; });
    return tasks;
  };
  // leading blocks of FW and FW^t: P_J and Q_J^T
  parallel_for(nS, [&](int64_t Jq) {
    const int J = (int)Jq, nj = nj_of(J);
    const FrontOut& o = fo[J];
    double* fw = rb.fw[0].get() + ds->fw_off[J];
    double* fwt = rb.fw[1].get() + ds->fw_off[J];
    std::copy(o.P.begin(), o.P.end(), fw);
    for (int i = 0; i < nj; ++i)
      for (int k = 0; k < nj; ++k) fwt[(size_t)i * nj + k] = o.Q[(size_t)k * nj + i];
  });
  // lower blocks: L21 P and U12^T Q^T, rows r0 .. r1 of each
  const std::vector<Task> prod = make_tasks(true);
  parallel_for((int64_t)prod.size(), [&](int64_t ti) {
    const Task& t = prod[ti];
    const int J = t.J, nj = nj_of(J), nb = nb_of(J), rows = t.r1 - t.r0;
    const FrontOut& o = fo[J];
    double* fw = rb.fw[0].get() + ds->fw_off[J];
    double* fwt = rb.fw[1].get() + ds->fw_off[J];
    double* c0 = fw + (int64_t)(nj + t.r0) * nj;
    double* c1 = fwt + (int64_t)(nj + t.r0) * nj;
    std::fill(c0, c0 + (int64_t)rows * nj, 0.0);
    std::fill(c1, c1 + (int64_t)rows * nj, 0.0);
    dense_mac(false, c0, nj, o.L21.data() + (size_t)t.r0 * nj, nj, 1, o.P.data(), nj, rows, nj, 0, nj);
    dense_mac(false, c1, nj, o.U12.data() + t.r0, 1, nb, fwt, nj, rows, nj, 0, nj);
  });
  // BM and BM^t, rows r0 .. r1 of each
  const std::vector<Task> back = make_tasks(false);
  parallel_for((int64_t)back.size(), [&](int64_t ti) {
    const Task& t = back[ti];
    const int J = t.J, nj = nj_of(J), nb = nb_of(J);
    const int64_t len = nj + nb;
    const FrontOut& o = fo[J];
    const double* fwl = rb.fw[0].get() + ds->fw_off[J] + (int64_t)nj * nj;    // L21 P, nb x nj
    const double* fwtl = rb.fw[1].get() + ds->fw_off[J] + (int64_t)nj * nj;   // U12^T Q^T, nb x nj
    double* bm = rb.bm[0].get() + ds->bm_off[J];
    double* bmt = rb.bm[1].get() + ds->bm_off[J];
    for (int i = t.r0; i < t.r1; ++i) {
      double* b0 = bm + i * len;
      double* b1 = bmt + i * len;
      for (int k = 0; k < nj; ++k) {
        b0[k] = o.Q[(size_t)i * nj + k];
        b1[k] = o.P[(size_t)k * nj + i];
      }
    }
    for (int c = 0; c < nb; ++c) {
      const double* x0 = fwtl + (int64_t)c * nj;
      const double* x1 = fwl + (int64_t)c * nj;
      for (int i = t.r0; i < t.r1; ++i) {
        bm[i * len + nj + c] = 0.0 - x0[i];
        bmt[i * len + nj + c] = 0.0 - x1[i];
      }
    }
  });
}

}  // namespace

int sbfwi_direct_factor(sbfwi_factors_s* f, hipStream_t s) {
  sbfwi_mesh_s* m = f->m;
  DirectSym* ds = m->dsym;
  if (!ds) return sbfwi_fail(SBFWI_EINVAL, "mesh has no dissection order");
  const int64_t nnz = m->nnz;
  std::vector<double> K(nnz), KT(nnz);
  SBFWI_HIP(hipMemcpyAsync(K.data(), f->d.Kval, nnz * sizeof(double), hipMemcpyDeviceToHost, s));
  SBFWI_HIP(hipMemcpyAsync(KT.data(), f->d.KTval, nnz * sizeof(double), hipMemcpyDeviceToHost, s));
  SBFWI_HIP(hipStreamSynchronize(s));
  std::vector<FrontOut> fo(ds->nS);
  SBFWI_CHECK(eliminate_levels(ds, m, K, KT, fo));
  RowBlocks rb;
  row_blocks(ds, fo, rb);
  std::vector<FrontOut>().swap(fo);
  DirectNum* dn = new DirectNum();
  f->dnum = dn;
  for (int t = 0; t < 2; ++t) {
    SBFWI_CHECK(sbfwi_alloc(&dn->FW[t], rb.nfw));
    SBFWI_CHECK(sbfwi_alloc(&dn->BM[t], rb.nbm));
    SBFWI_CHECK(sbfwi_copy_sync(dn->FW[t], rb.fw[t].get(), rb.nfw * sizeof(double), hipMemcpyHostToDevice));
    SBFWI_CHECK(sbfwi_copy_sync(dn->BM[t], rb.bm[t].get(), rb.nbm * sizeof(double), hipMemcpyHostToDevice));
  }
  f->bytes += 8 * 2 * (rb.nfw + rb.nbm);
  return SBFWI_OK;
}

void sbfwi_direct_num_free(DirectNum* dn) {
  if (!dn) return;
  for (int t = 0; t < 2; ++t) {
    sbfwi_dev_free(dn->FW[t]);
    sbfwi_dev_free(dn->BM[t]);
  }
  delete dn;
}

// ------------------------------------------------------------------ solve

namespace {

template <int NSM>
void launch_prog(int t, const DirectSym* ds, const DLaunch& L, const double* vals, int NS, int s0,
                 const double* in, double* upd, double* out, int* status, int count, hipStream_t s) {
  const size_t lds = (size_t)L.slots * NSM * sizeof(double);
  const bool sub = L.st0 < 0;
  if (t == 0 && !sub)
    hipLaunchKernelGGL((direct_prog_kernel<NSM, true, kLevelU>), dim3((unsigned)L.nblk), dim3(DT), lds, s,
                       ds->prog[0], L.blk0, L.st0, L.G, vals, NS, s0, in, upd, out, status, count);
  else if (t == 0)
    hipLaunchKernelGGL((direct_prog_kernel<NSM, true, kSubtreeU>), dim3((unsigned)L.nblk), dim3(DT), lds, s,
                       ds->prog[0], L.blk0, L.st0, L.G, vals, NS, s0, in, upd, out, status, count);
  else if (!sub)
    hipLaunchKernelGGL((direct_prog_kernel<NSM, false, kLevelU>), dim3((unsigned)L.nblk), dim3(DT), lds, s,
                       ds->prog[1], L.blk0, L.st0, L.G, vals, NS, s0, in, upd, out, status, count);
  else
    hipLaunchKernelGGL((direct_prog_kernel<NSM, false, kSubtreeU>), dim3((unsigned)L.nblk), dim3(DT), lds, s,
                       ds->prog[1], L.blk0, L.st0, L.G, vals, NS, s0, in, upd, out, status, count);
}

// Runs one direction's program for shots s0 .. s0 + nsm - 1 (nsm a power of two).
void run_prog(int t, const DirectSym* ds, int nsm, const double* vals, int NS, int s0, const double* in,
              double* upd, double* out, int* status, bool count_last, hipStream_t s) {
  const size_t nl = ds->launches[t].size();
  for (size_t k = 0; k < nl; ++k) {
    const DLaunch& L = ds->launches[t][k];
    const int count = count_last && k + 1 == nl;
    if (L.nblk == 0) continue;
    switch (nsm) {
      case 1: launch_prog<1>(t, ds, L, vals, NS, s0, in, upd, out, status, count, s); break;
      case 2: launch_prog<2>(t, ds, L, vals, NS, s0, in, upd, out, status, count, s); break;
      case 4: launch_prog<4>(t, ds, L, vals, NS, s0, in, upd, out, status, count, s); break;
      case 8: launch_prog<8>(t, ds, L, vals, NS, s0, in, upd, out, status, count, s); break;
      default: launch_prog<16>(t, ds, L, vals, NS, s0, in, upd, out, status, count, s); break;
    }
  }
}

}  // namespace

int sbfwi_direct_solve(sbfwi_factors_s* f, CoarseWork* w, int transpose, const double* b, double* x,
                       hipStream_t s) {
  const DirectSym* ds = f->m->dsym;
  const DirectNum* dn = f->dnum;
  const int t = transpose ? 1 : 0;
  const int NS = w->NS;
  ProfScope ps(PK_SOLVE, s);
  // shots per pass: the shot count rounded up to a power of two, at most 16, and
  // small enough that the largest block vector fits in 64 KiB of LDS
  int nsm = 1;
  while (nsm < NS && nsm < 16) nsm *= 2;
  while (nsm > 1 && (size_t)ds->max_slots * nsm * sizeof(double) > 65536) nsm /= 2;
  if ((size_t)ds->max_slots * sizeof(double) > 65536)
    return sbfwi_fail(SBFWI_EINVAL, "direct solve: a supernode front is too large for LDS");
  for (int s0 = 0; s0 < NS; s0 += nsm) {
    const bool last = s0 + nsm >= NS;
    // forward, leaves first: y (by position) and the update vectors from b (by node)
    run_prog(0, ds, nsm, dn->FW[t], NS, s0, b, w->dupd, w->dyb, f->d.status, false, s);
    // backward, root first: x (by position and by node) from y
    run_prog(1, ds, nsm, dn->BM[t], NS, s0, w->dyb, w->dxp, x, f->d.status, last, s);
  }
  SBFWI_HIP(hipGetLastError());
  return SBFWI_OK;
}

extern "C" int sbfwi_direct_launches(sbfwi_mesh m, int dir, int64_t* out, int cap, int* n_launches) {
  if (!m || !out || !n_launches) return sbfwi_fail(SBFWI_EINVAL, "NULL argument");
  if (dir != 0 && dir != 1) return sbfwi_fail(SBFWI_EINVAL, "dir must be 0 (forward) or 1 (backward)");
  const DirectSym* ds = m->dsym;
  if (!ds) return sbfwi_fail(SBFWI_EINVAL, "mesh has no dissection order");
  const auto& Ls = ds->launches[dir];
  *n_launches = (int)Ls.size();
  for (int k = 0; k < (int)Ls.size() && k < cap; ++k) {
    const DLaunch& L = Ls[k];
    const int64_t v[8] = {L.nblk, L.G, L.slots, L.steps, L.rows, L.vrecs, L.max_step_rows, L.st0 >= 0 ? 0 : 1};
    for (int q = 0; q < 8; ++q) out[8 * k + q] = v[q];
  }
  return SBFWI_OK;
}

extern "C" int sbfwi_direct_info(sbfwi_mesh m, int64_t* out) {
  if (!m || !out) return sbfwi_fail(SBFWI_EINVAL, "NULL argument");
  const DirectSym* ds = m->dsym;
  if (!ds) return sbfwi_fail(SBFWI_EINVAL, "mesh has no dissection order");
  out[0] = ds->nS;
  out[1] = ds->depth;
  out[2] = ds->max_nj;
  out[3] = ds->sum_j2;
  out[4] = ds->sum_jb;
  out[5] = ds->b_ptr[ds->nS];
  int64_t mx = 0;
  for (int l = 0; l <= ds->depth; ++l) mx = std::max<int64_t>(mx, ds->lvl_ptr[l + 1] - ds->lvl_ptr[l]);
  out[6] = mx;
  return SBFWI_OK;
}

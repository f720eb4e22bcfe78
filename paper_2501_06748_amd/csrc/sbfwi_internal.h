// Internal declarations of the sbfwi library (gfx950).
//
// Storage conventions (all FP64, shots innermost so that one radial level of
// one element for all shots of a launch is a contiguous, coalesced run):
//   interior state r, w and the swept sources q: ((int_off[e] + j*nb + i)*NS + s),
//       level j = 0 .. N_r-2 (the boundary level N_r-1 is the shared nodal state);
//   nodal state and coarse vectors: (node*NS + s);
//   per-slot element vectors (effective sources, boundary sweeps): ((loop_off[e] + i)*NS + s);
//   unknowns with ghosts, levels -1 .. N_r: ((x_off[e] + (j+1)*nb + i)*NS + s);
//   level fields 0 .. N_r-1 (fine grid): ((par_off[e] + j*nb + i)*NS + s).
// Cyclic tridiagonal blocks ("bands") store sub, diag, super diagonals:
//   band[t*nb + i], t = 0: M[i][i-1], t = 1: M[i][i], t = 2: M[i][i+1] (indices mod nb).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>
#include <string>
#include <vector>

#include "../../include/sbfwi.h"

#define SBFWI_MAX_NB 24

// Work item of block blockIdx.x in a sweep launch over n elements of a class and
// G groups of shots: the grid has sweep_blocks(n, G) blocks, and the G groups of
// one element sit kXcds block ids apart.  The dispatcher hands consecutive
// blocks to the XCDs in turn, so an element's groups run on one XCD at about the
// same time and share its L2 for the element's pivot blocks and for the state
// lines, whose shots are adjacent.  Returns false for the padding blocks (the
// whole block leaves).  With one group, block b takes element b.
constexpr int kXcds = 8;
__host__ __device__ inline int64_t sweep_blocks(int64_t n, int G) { return (n + kXcds - 1) / kXcds * kXcds * G; }
__device__ inline bool sweep_item(int64_t n, int G, int64_t& ei, int& g) {
  const int64_t b = blockIdx.x, tile = b / (kXcds * G);
  const int r = (int)(b % (kXcds * G));
  g = r / kXcds;
  ei = tile * kXcds + r % kXcds;
  return ei < n;
}

// acc + sum (SUB: minus) of arr[slot * NS + s] over the loop slots
// node_slot[t0 .. t1) of a node, added in that order.  The first four slots and
// their values are loaded together (an absent one reads slot entry t0, or 0 for
// an empty range, and is not added), so that a node's entries cost one chain of
// two loads rather than one per slot.
template <bool SUB>
__device__ inline double node_gather(double acc, const int64_t* __restrict__ node_slot, int64_t t0, int64_t t1,
                                     const double* __restrict__ arr, int NS, int s) {
  constexpr int C = 4;
  int64_t sl[C];
  double v[C];
#pragma unroll
  for (int c = 0; c < C; ++c) sl[c] = node_slot[t0 + c < t1 ? t0 + c : (t1 > t0 ? t0 : 0)];
#pragma unroll
  for (int c = 0; c < C; ++c) v[c] = arr[sl[c] * NS + s];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const double n = SUB ? acc - v[c] : acc + v[c];
    acc = t0 + c < t1 ? n : acc;
  }
  for (int64_t t = t0 + C; t < t1; ++t) acc = SUB ? acc - arr[node_slot[t] * NS + s] : acc + arr[node_slot[t] * NS + s];
  return acc;
}

// Sweeps form the central-difference rows from the densities (fd_bands.h).
struct FactorsDev;
inline bool sbfwi_fly_rows(const FactorsDev& f);

// The low-frequency expansion schemes (nodal time loop, K_e and M_e per element).
inline bool sbfwi_is_lfe(int scheme) {
  return scheme == SBFWI_SCHEME_LFE || scheme == SBFWI_SCHEME_LFE_CONDENSED;
}

// Plain device view of a mesh (kernel argument).
struct MeshDev {
  int64_t n_nodes = 0, n_elem = 0, n_loop = 0, nnz = 0;
  double xi0 = 1e-3;
  int32_t* nb = nullptr;
  int32_t* nr = nullptr;
  int64_t* loop_off = nullptr;
  int64_t* par_off = nullptr;
  int64_t* int_off = nullptr;
  int64_t* x_off = nullptr;
  int64_t* finv_off = nullptr;
  int64_t* dense_off = nullptr;
  int64_t* loop_nodes = nullptr;
  double* loop_xy = nullptr;     // [n_loop][2]
  double* centre = nullptr;      // [n_elem][2]
  int32_t* elem_by_cost = nullptr;  // [n_elem] elements by decreasing N_r n_b^2 (persistent sweeps)
  int64_t* node_ptr = nullptr;   // [n_nodes+1] -> node_slot
  int64_t* node_slot = nullptr;  // loop slots (loop_off[e] + i) that touch each node
  int64_t* row_ptr = nullptr;    // coarse CSR
  int32_t* col = nullptr;
  int64_t* diag_idx = nullptr;   // [n_nodes] position of (r, r)
  int64_t* tr_idx = nullptr;     // [nnz] position of (c, r) for entry (r, c)
  int64_t* contrib_ptr = nullptr;  // [nnz+1]
  int64_t* contrib_src = nullptr;  // index into S storage (dense_off[e] + i*nb + j)
  // sliced ELL copy of the coarse pattern: slices of ELL_SLICE rows, padded to
  // the widest row of the slice in chunks of ELL_LPR entries (padding: column =
  // row, value 0); chunk c holds entries c*ELL_LPR.. of every row, row-major
  int64_t n_ell = 0;
  int64_t* ell_off = nullptr;   // [n_slices + 1] offsets of the slices
  int32_t* ell_w = nullptr;     // [n_slices] chunks of ELL_LPR entries in each slice
  int32_t* ell_col = nullptr;   // [n_ell]
  int64_t* ell_pos = nullptr;   // [nnz] ELL position of every CSR entry
};
#define ELL_SLICE 256
#define ELL_LPR 4

// Direct solve programs (direct.hip).  A block of the solve kernel runs a list
// of steps; a step first assembles vectors in LDS (one DVRec per LDS slot, one
// value per shot), then evaluates dense rows against them (one DRRec per row).
struct alignas(16) DVRec {
  int64_t src;     // forward: node of the right-hand side; backward: position of y (own) or x (B set)
  int64_t g0, g1;  // forward: the children's update entries to subtract (ngl of them)
  int32_t ngl;     // forward: 0, 1 or 2; backward: 0 = read y, 1 = read x
  int32_t slot;    // LDS slot
};
struct alignas(16) DRRec {
  int64_t val;     // offset of the row's values
  int64_t out;     // forward: position of y (kind 0) or update entry (kind 1); backward: position of x
  int64_t g0;      // forward kind 1: first child update entry passed through; backward: node
  int64_t g1;      // forward kind 1: second one
  int32_t len;     // columns (LDS slots slot0 .. slot0 + len - 1)
  int32_t slot0;
  int32_t ngl;     // forward kind 1: entries passed through (0, 1 or 2)
  int32_t kind;    // forward: 0 = row of y, 1 = row of the update vector
};
struct DStep {
  int64_t v0, v1, r0, r1;   // slot records [v0, v1), row records [r0, r1)
};
struct DProgDev {
  DVRec* vrec = nullptr;
  DRRec* rrec = nullptr;
  DStep* steps = nullptr;
  int64_t* blk = nullptr;    // steps of block b: [blk[b], blk[b+1])
};
struct DLaunch {
  int64_t blk0 = 0, nblk = 0;   // blocks of the launch in the program's block list
  int64_t st0 = -1;             // >= 0: block b of the launch runs the single step st0 + b
  int G = 1, slots = 0;         // lanes per row, LDS slots per block
  int64_t steps = 0, rows = 0, vrecs = 0, max_step_rows = 0;   // totals (introspection)
};
// Nested-dissection structure of the coarse system and the solve programs.
struct DirectSym {
  int nS = 0, depth = 0;
  int64_t max_nj = 0, sum_j2 = 0, sum_jb = 0;
  std::vector<int64_t> pos, inv, sn_ptr, b_ptr, bpos, fw_off, bm_off;
  std::vector<int32_t> level, lvl_ptr, lvl_sn, snp;
  std::vector<std::vector<int32_t>> children;
  std::vector<int64_t> fr_off, gl_ptr, gl;   // front rows and the children's update entries per row
  int cut = 0, n_sub = 0;             // subtree blocks: cut level and their count
  int max_slots = 0;                  // largest LDS vector of any block (slots)
  std::vector<DLaunch> launches[2];   // forward, backward programs in launch order
  DProgDev prog[2];
  int sn_of(int64_t p) const { return snp[p]; }
};
// Row blocks of K_g (index 0) and of K_g^T (index 1), row-major per supernode:
// forward FW_J = [P_J ; C_J P_J], backward BM_J = [Q_J | -Q_J U12_J] (see direct.hip).
struct DirectNum {
  double* FW[2] = {nullptr, nullptr};
  double* BM[2] = {nullptr, nullptr};
};

struct sbfwi_mesh_s {
  int64_t n_nodes = 0, n_elem = 0, n_params = 0, n_int = 0, n_loop = 0, n_x = 0;
  int64_t nnz = 0, n_finv = 0, n_dense = 0, n_contrib = 0;
  double xi0 = 1e-3;
  // host copies
  std::vector<int32_t> h_nb, h_nr;
  std::vector<int64_t> h_loop_off, h_par_off, h_int_off, h_x_off, h_finv_off, h_dense_off;
  std::vector<int64_t> h_row_ptr, h_col64;
  std::vector<int32_t> h_class_elems[3];
  int class_nmax[3] = {0, 0, 0};   // most interior levels of an element of each class
  std::vector<int32_t> h_elem_by_cost;
  MeshDev d;
  int32_t* class_elems[3] = {nullptr, nullptr, nullptr};   // elements with nb <= 8, 16, 24
  DirectSym* dsym = nullptr;
};

// Plain device view of a factored model (kernel argument).
struct FactorsDev {
  double a0 = 0, a1 = 0, a2 = 0, c1 = 0, c2 = 0, c3 = 0, dt = 0;
  double* finv = nullptr;      // [n_finv] phi~_j^-1, j = 0 .. N_r-2, row-major
  double* th_band = nullptr;   // [3 n_params] theta_j, j = 0 .. N_r-1
  double* ps_band = nullptr;   // [3 n_params] psi_j,   j = 0 .. N_r-1
  double* pm_band = nullptr;   // [3 n_params] P_j = -xi_j^2 M0_j
  double* th_np1 = nullptr;    // [3 n_loop] theta_{n+1}
  double* phim1 = nullptr;     // [3 n_loop] phi_{-1} = E1_0^T
  double* psim1 = nullptr;     // [3 n_loop] psi_{-1}
  double* G = nullptr;         // [n_dense] psi_{n+1} psi_n^-1
  double* S = nullptr;         // [n_dense] dynamic stiffness
  double* psit0 = nullptr;     // [n_dense] psi~_0
  double* psin_inv = nullptr;  // [n_dense] psi_n^-1
  double* phit_n = nullptr;    // [n_dense] phi~_n
  double* thm1_inv = nullptr;  // [n_dense] theta_{-1}^-1
  double* gbasis = nullptr;    // [32 n_loop] d(E0,E1,E2,M0 segment block)/d(nodal density)
  // central differences only: the rows theta_j, psi_j, P_j formed on the fly by the sweeps
  double* bkap = nullptr;      // [n_loop][3][kFdKappa] kappa of every band entry (fd_bands.h)
  double* rho = nullptr;       // [n_params] the model's nodal densities
  int fly = 1;                 // the sweeps form those rows on the fly (when bkap exists)
  double* Kval = nullptr;      // [nnz] coarse matrix on the CSR pattern
  double* KTval = nullptr;     // [nnz] its transpose on the same (symmetric) pattern
  double* Kell = nullptr;      // [n_ell] K_g in the sliced ELL layout
  double* KTell = nullptr;     // [n_ell] K_g^T in the sliced ELL layout
  double* diag_inv = nullptr;  // [n_nodes] Jacobi preconditioner
  int* status = nullptr;       // device status words
  // radial Galerkin scheme: quadrature weights of every interval, by level count
  int scheme = 0;
  double* rgw = nullptr;       // [sum over level counts of (N_r - 1) * kRgW] weights
  int* rgw_off = nullptr;      // [129] offset of the table of N_r levels (in doubles)
  // low-frequency expansion: element masses and the assembled global mass
  double* Me = nullptr;        // [n_dense] M_e (S holds K_e)
  double* Mval = nullptr;      // [nnz] M_g on the CSR pattern (Kval holds K_g + a0 M_g)
};

inline bool sbfwi_fly_rows(const FactorsDev& f) { return f.bkap != nullptr && f.fly != 0; }

// Low-frequency expansion path (lfe.hip): forward run (vstore, optional, keeps
// every step's nodal velocity) and the paper-kernel gradient from the kept
// velocities; both synchronise s.
struct sbfwi_factors_s;
struct sbfwi_ckpt_s;
int sbfwi_lfe_forward(sbfwi_factors_s* f, int n_shots, int64_t n_steps, const int64_t* src_node,
                      const double* wavelet, int n_rec, const int64_t* rec_node, double* traces, double* vstore,
                      hipStream_t s);
int sbfwi_lfe_adjoint(sbfwi_factors_s* f, sbfwi_ckpt_s* ck, const double* adj_src, int per_shot, double* grad,
                      hipStream_t s);

// Weights of one radial interval [xi_j, xi_j + h] in the Galerkin scheme, for
// local levels p, q in {0, 1} (row, column) and interpolation end e in {0, 1}:
//   [0 + 4p + 2q + e]  int xi N_p' N_q' N_e          (E0)
//   [8 + 4p + 2q + e]  int N_p' N_q N_e              (E1^T)
//   [16 + 4p + 2q + e] int N_p N_q' N_e              (E1)
//   [24 + 4p + 2q + e] int N_p N_q N_e / xi          (E2)
//   [32 + 2p + e]      int xi N_p N_e                (lumped M0)
constexpr int kRgW = 36;
// Gauss-Legendre quadrature (4 points per interval) of the weights above for
// every level count present in the mesh; rgw_off[N_r] = -1 for absent counts.
void sbfwi_rg_weights(double xi0, const std::vector<int>& level_counts, std::vector<double>& w,
                      std::vector<int>& off);

// Launch plan of the sweep kernels: shots per block (1, 2, 4, 8 or 16) for each
// n_b class (n_b <= 8, <= 16, <= 24) of each sweep, or (fusedS > 0) one
// persistent launch over all classes with fusedS shots per block.  Zero
// entries take the default for the run's shot count.
enum { SW_CONDENSE = 0, SW_RECOVER = 1, SW_ADJ_CONDENSE = 2, SW_ADJ_RECOVER = 3, SW_N = 4 };
struct SweepPlan {
  int S[SW_N][3] = {};
  int fusedS[SW_N] = {};
};
inline int sbfwi_default_shots_per_block(int NS) { return NS >= 4 ? 4 : (NS >= 2 ? 2 : 1); }
int sbfwi_device_cus();

struct sbfwi_factors_s {
  sbfwi_mesh_s* m = nullptr;
  double c = 0, dt = 0, beta = 0, gamma = 0;
  double rtol = 1e-13;
  int max_iter = 500;
  int enqueued_iters = 13;       // BiCGStab iterations enqueued per solve (more run in a rescue kernel)
  int use_graphs = 0;            // forward runs replay each time step from HIP graphs
  int overlap_adjoint = 1;       // recompute the next checkpoint segment while the adjoint runs the current one
  int keep_solutions = 1;        // forward runs with checkpoints keep every step's coarse solution
  int64_t tail_kib = 0;          // forward runs with checkpoints keep the fields of the last segments (KiB)
  int joint_sweeps = 1;          // recover of step k and condense of step k + 1 in one sweep
  int scheme = 0;                // radial scheme (SBFWI_SCHEME_*)
  SweepPlan plan;
  DirectNum* dnum = nullptr;     // direct factors of K_g (coarse solver 1), else BiCGStab
  double env_r = 0;              // largest 1 / |K_g,ii|: response scale of the growth envelope
  int64_t bytes = 0;
  FactorsDev d;
};

struct sbfwi_ckpt_s {
  sbfwi_factors_s* f = nullptr;
  int n_shots = 0, n_rec = 0;
  int64_t n_steps = 0, interval = 0, n_saved = 0;
  int64_t bytes = 0;
  int64_t* src_node = nullptr;   // device copies [n_shots]
  double* wavelet = nullptr;     // [n_shots][n_steps]
  int64_t* rec_node = nullptr;   // [n_rec]
  double* states = nullptr;      // [n_saved][state size]: interior r, w then nodal U, V, A, W, corr
  bool full_store = false;       // every step's unknowns kept by the forward run
  double* xstore = nullptr;      // full storage: [n_steps][n_x*NS]
  double* fstore = nullptr;      // full storage: [n_steps][n_params*NS] accelerations a^k
  double* vstore = nullptr;      // full storage: [n_steps][n_params*NS] velocities v^k
  double* ustore = nullptr;      // optional: [n_steps][n_nodes*NS] coarse solutions (the recompute skips its solves)
  // optional tail store: steps tail_k0 + 1 .. n_steps (whole checkpoint segments at the end of
  // the run) keep the unknowns with ghosts and the accelerations, as a recompute would store
  // them, so that the exact backward pass does not recompute those segments
  int64_t tail_k0 = 0;
  double* tail_x = nullptr;      // [n_steps - tail_k0][n_x*NS], then in the same allocation
  double* tail_f = nullptr;      // [n_steps - tail_k0][n_params*NS]
  size_t tail_bytes = 0;
};

// Growth envelope of a forward run (api.cpp): the nodal displacement of shot s at
// step k may not exceed kEnvelopeSafety * 4 k r F_k(s), r = env_r of the factors and
// F_k(s) the sum of |point forces| of shot s up to step k.
constexpr double kEnvelopeSafety = 10.0;

// ---- live kernel timing (profiler.cpp) ----
#define SBFWI_PROF_KERNELS 21
enum {
  PK_CONDENSE = 0, PK_RECOVER = 1, PK_SOLVE = 2, PK_RHS = 3, PK_NODAL = 4, PK_ADJ_CONDENSE = 5,
  PK_ADJ_RECOVER = 6, PK_ADJ_RHS = 7, PK_ADJ_NODAL = 8, PK_GRAD_EXACT = 9, PK_GRAD_PAPER = 10,
  PK_FACTOR = 11, PK_SOLVE_V = 12, PK_SOLVE_T = 13, PK_SOLVE_X = 14, PK_SOLVE_INIT = 15,
  PK_RECOVER_STORE = 16, PK_FEM_STEP = 17, PK_JOINT = 18, PK_JOINT_STORE = 19, PK_ADJ_JOINT = 20
};
// Brackets the launches made during its lifetime with events on stream s when
// kernel id is enabled by sbfwi_profile.
void sbfwi_prof_suspend(int on);   // no events are recorded while suspended (graph capture)
struct ProfScope {
  ProfScope(int id, hipStream_t s);
  ~ProfScope();
  int id_;
  hipStream_t s_;
  void* a_ = nullptr;
};

// ---- error handling / allocation (api.cpp) ----
int sbfwi_fail(int code, const char* fmt, ...);
// Synchronous copy on a per-thread library stream (never the legacy null
// stream, so it is legal while other threads capture graphs).
int sbfwi_copy_sync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);
int sbfwi_zero_sync(void* dst, size_t bytes);
void* sbfwi_dev_alloc(size_t bytes);
void sbfwi_dev_free(void* p);

#define SBFWI_HIP(call)                                                        \
  do {                                                                         \
    hipError_t _e = (call);                                                    \
    if (_e != hipSuccess)                                                      \
      return sbfwi_fail(SBFWI_EHIP, "%s failed: %s (%s:%d)", #call,             \
                        hipGetErrorString(_e), __FILE__, __LINE__);             \
  } while (0)

#define SBFWI_CHECK(call)                                                      \
  do {                                                                         \
    int _r = (call);                                                           \
    if (_r != SBFWI_OK) return _r;                                             \
  } while (0)

template <typename T>
static inline int sbfwi_alloc(T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  *p = (T*)sbfwi_dev_alloc((size_t)count * sizeof(T));
  if (!*p) return sbfwi_fail(SBFWI_ENOMEM, "device allocation of %lld bytes failed",
                             (long long)((size_t)count * sizeof(T)));
  return SBFWI_OK;
}

template <typename T>
static inline int sbfwi_upload(T** p, const std::vector<T>& v) {
  SBFWI_CHECK(sbfwi_alloc(p, (int64_t)v.size()));
  if (!v.empty()) SBFWI_CHECK(sbfwi_copy_sync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return SBFWI_OK;
}

// ---- stage entry points (factor.hip, step.hip, coarse.hip, adjoint.hip) ----
int sbfwi_factor_impl(sbfwi_mesh_s* m, const double* rho, double c, double dt, double beta,
                      double gamma, int scheme, int coarse_solver, hipStream_t s, sbfwi_factors_s** out);

struct CoarseWork {
  int NS = 0;
  int64_t n = 0;
  double *r = nullptr, *rhat = nullptr, *p = nullptr, *v = nullptr, *sv = nullptr,
         *t = nullptr, *phat = nullptr, *shat = nullptr, *w = nullptr, *partial = nullptr,
         *scal = nullptr;
  unsigned* bar = nullptr;
  int nblocks = 0, nthreads = 0;
  double *dyb = nullptr, *dxp = nullptr;   // direct solve: y and x by elimination position
  double* dupd = nullptr;                  // direct solve: the supernodes' update vectors
};
int sbfwi_coarse_work_alloc(CoarseWork* w, sbfwi_mesh_s* m, int NS);
void sbfwi_coarse_work_free(CoarseWork* w);
// Solves K x = b (transpose = 0) or K^T x = b (transpose = 1) for NS right-hand
// sides; x holds the initial guess on entry.  Records failures in f->status.
int sbfwi_coarse_solve(sbfwi_factors_s* f, CoarseWork* w, int transpose, const double* b,
                       double* x, int64_t step, hipStream_t s);
// The same in parts (bit 1: start-up and enqueued iterations, bit 2: the
// cooperative rescue kernel, bit 4: final check); step_ptr (device, may be
// NULL) overrides step when failures are recorded.
int sbfwi_coarse_solve_parts(sbfwi_factors_s* f, CoarseWork* w, int transpose, const double* b,
                             double* x, int64_t step, const int64_t* step_ptr, int parts, hipStream_t s);

struct StepWork {
  int NS = 0;
  double *r = nullptr, *w = nullptr;                    // interior state: r = c1 u - c2 v - c3 a, w = a0 u + a1 v + a2 a
  double *U = nullptr, *V = nullptr, *A = nullptr;      // nodal state
  double* W = nullptr;                                  // nodal w = a0 U + a1 V + a2 A
  double* corr = nullptr;                               // predictor correction of the coarse solve
  double *q = nullptr, *yn = nullptr, *fhat = nullptr, *F = nullptr, *Unew = nullptr;
  double* ustore = nullptr;   // optional: every step's coarse solution, [n_steps][n_nodes*NS]
  double* env = nullptr;      // optional: growth envelope of the nodal displacement, [n_steps][NS] (owned)
  CoarseWork cw;
  // the swept sources (q, y_n, f_hat) of the next step are already computed (by a
  // joint sweep); reset whenever the state is replaced
  bool condensed = false;
  // graph replay of a time step: device step counter and the two captured halves
  int64_t* kdev = nullptr;
  hipGraphExec_t g_pre = nullptr, g_post = nullptr;
};
int sbfwi_step_work_alloc(StepWork* w, sbfwi_mesh_s* m, int NS);
void sbfwi_step_work_free(StepWork* w);
int64_t sbfwi_state_size(sbfwi_mesh_s* m, int NS);

// Source table of a run: n_src sources per shot; source c of shot q acts on
// node src_node[q*n_src + c] with amplitude amp[(q*n_src + c)*amp_steps + idx],
// idx = k - 1 (forward in time) or amp_steps - k (time-reversed).
struct SourceTable {
  int n_src = 1;
  const int64_t* node = nullptr;
  int node_stride = 1;           // 1: node[q*n_src + c] per shot; 0: node[c] shared by all shots
  const double* amp = nullptr;
  int64_t amp_steps = 0;
  int reversed = 0;
};

// One forward step k: condense (unless a joint sweep of step k - 1 did it), assemble,
// coarse solve, nodal update, recover; with next = true (step k + 1 follows on
// the same work buffers) the recover sweep also condenses step k + 1.
// Optional stores (nullptr = skip): unknowns with ghosts (xs) and a level field
// (fs: a^k when field_kind = 0, v^k when field_kind = 1); receiver traces.
// usol (optional): the step's coarse solution, kept by an earlier run of the
// same step; the gather and the coarse solve are then skipped.
int sbfwi_forward_step(sbfwi_factors_s* f, StepWork* w, int64_t k, const SourceTable& src,
                       int n_rec, const int64_t* rec_node, double* traces, int64_t n_steps,
                       double* xs, double* fs, int field_kind, hipStream_t s, double* vs = nullptr,
                       const double* usol = nullptr, bool next = false);
int sbfwi_state_copy(sbfwi_mesh_s* m, StepWork* w, double* dst, int to_store, hipStream_t s);
// Graph replay of forward steps (no per-step stores): the first call captures
// the step on stream s (which must not be the null stream) into two graphs
// around the coarse solve's cooperative rescue launch; every call replays one
// step, whose number is kept on the device (set by sbfwi_graph_step_reset).
int sbfwi_graph_step_reset(StepWork* w, int64_t k, hipStream_t s);
int sbfwi_forward_step_graph(sbfwi_factors_s* f, StepWork* w, const SourceTable& src, int n_rec,
                             const int64_t* rec_node, double* traces, int64_t n_steps, hipStream_t s);
int sbfwi_step_zero(sbfwi_mesh_s* m, StepWork* w, hipStream_t s);

// Autotuning of the sweep launch plans (step.hip: condense / recover,
// adjoint.hip: transposed condense / recover) for runs of NS shots: every
// candidate is timed on the factors with zero state and the fastest kept in
// f->plan.  out (host, may be NULL) receives per sweep kind: the chosen S of
// the three classes, the fused S (0 = per-class launches), and the best time
// in ms of the per-class and of the fused variants.
// Direct coarse solver (direct.hip).
int sbfwi_direct_symbolic(sbfwi_mesh_s* m, const double* host_node_xy);
// (Re)builds the solve programs with the subtree launches cut at the shallowest
// level holding at least min_subtrees supernodes (the device must be idle).
int sbfwi_direct_programs(sbfwi_mesh_s* m, int min_subtrees);
void sbfwi_direct_sym_free(DirectSym* ds);
int sbfwi_direct_factor(sbfwi_factors_s* f, hipStream_t s);
void sbfwi_direct_num_free(DirectNum* dn);
int sbfwi_direct_solve(sbfwi_factors_s* f, CoarseWork* w, int transpose, const double* b, double* x,
                       hipStream_t s);

int sbfwi_tune_step_sweeps(sbfwi_factors_s* f, int NS, hipStream_t s, double* out);
int sbfwi_tune_adj_sweeps(sbfwi_factors_s* f, int NS, hipStream_t s, double* out);

int sbfwi_adjoint_impl(sbfwi_factors_s* f, sbfwi_ckpt_s* ck, const double* adj_src, int mode,
                       double* grad, hipStream_t s);
int sbfwi_misfit_residual(const double* traces, const double* observed, int64_t count, double dt,
                          double* residual, double* misfit, hipStream_t s);

/*
 * sbfwi.h -- C ABI of the MI355X (gfx950) hot path of full-waveform inversion
 * with the scaled boundary finite element method and radial discretisation
 * (Daneshyar & Kollmannsberger, "Full-waveform inversion via the scaled
 * boundary finite element method").
 *
 * Conventions (apply to every call below)
 * ---------------------------------------
 * - Every function returns int: SBFWI_OK (0) or a negative error code; it
 *   never throws.  sbfwi_last_error() returns a thread-local message for the
 *   last failure on the calling thread.
 * - Pointers named host_* are host memory; every other array pointer is
 *   device memory owned by the caller (e.g. a torch tensor).  The library owns
 *   only the internals of the opaque handles; their device memory comes from
 *   hipMalloc, or from the allocator registered with sbfwi_set_allocator.
 * - Every device call takes a hipStream_t (0 = the null stream) and is
 *   asynchronous on that stream unless stated otherwise.  Calls that return
 *   a handle synchronise the stream before returning.
 * - FP64 throughout.  Integers: int64_t for global indices and offsets.
 *
 * Fine-grid layout (density rho and gradient): element e occupies
 * [off_e, off_e + N_r,e * n_b,e), level-major: rho[off_e + j * n_b,e + k] is
 * the density at radial level j (j = 0 at xi0 near the scaling centre,
 * j = N_r,e - 1 on the boundary) and boundary node k (position k of the
 * element's counter-clockwise loop).  Boundary-level densities are per
 * element.  off_e = sum_{e' < e} N_r,e' n_b,e'.
 */
#ifndef SBFWI_H
#define SBFWI_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbfwi_mesh_s*    sbfwi_mesh;     /* topology, element loops, coarse pattern   */
typedef struct sbfwi_factors_s* sbfwi_factors;  /* factored model for one (mesh, rho, c, dt) */
typedef struct sbfwi_ckpt_s*    sbfwi_ckpt;     /* checkpointed forward run (all shots)      */

enum {
  SBFWI_OK = 0,
  SBFWI_EINVAL = -1,      /* bad argument, or a loop that is not CCW / star-convex           */
  SBFWI_ENOMEM = -2,      /* device allocation failed                                         */
  SBFWI_ESINGULAR = -3,   /* a pivot block of the condensation sweep is singular              */
  SBFWI_ENONFINITE = -4,  /* a non-finite wavefield value was detected (step in last_error)   */
  SBFWI_EUNSTABLE = -5,   /* the wavefield grew beyond the stability envelope (step in msg)   */
  SBFWI_ENOCONV = -6,     /* the coarse Krylov solve did not converge (step in last_error)    */
  SBFWI_EHIP = -7         /* a HIP runtime call failed                                        */
};

enum { SBFWI_SCHEME_PAPER_FD = 0, SBFWI_SCHEME_RADIAL_GALERKIN = 1, SBFWI_SCHEME_LFE = 2,
       SBFWI_SCHEME_LFE_CONDENSED = 3 };
enum { SBFWI_GRAD_EXACT = 0, SBFWI_GRAD_PAPER_KERNEL = 1 };
/* Flag OR-ed into the gradient mode: one gradient (and one misfit) per shot. */
enum { SBFWI_GRAD_PER_SHOT = 16 };

/* Message of the last failure on this thread ("" if none). */
const char* sbfwi_last_error(void);

/* Optional device allocator for handle internals and work buffers (NULL, NULL
 * restores hipMalloc/hipFree).  alloc(bytes, ctx) returns device memory or NULL;
 * free(ptr, ctx) releases it.  It is called on the thread that makes the library
 * call.  Every block is released by the allocator that made it, also after the
 * registration has changed.  Thread-safe. */
int sbfwi_set_allocator(void* (*alloc_fn)(size_t bytes, void* ctx),
                        void (*free_fn)(void* ptr, void* ctx), void* ctx);

/*
 * sbfwi_build_mesh -- geometry of scaled-boundary polygons (Section "Scaled
 * boundary discretization": the scaling-centre transformation, boundary
 * interpolation by linear segments between consecutive loop nodes).
 *   host_node_xy    [n_nodes][2] node coordinates.
 *   host_elem_ptr   [n_elem + 1] offsets into host_elem_nodes.
 *   host_elem_nodes counter-clockwise loop of each element (global node ids),
 *                   3 <= n_b <= 24 nodes per element.
 *   host_centre_xy  [n_elem][2] scaling centres, or NULL for the area centroid.
 *   host_n_r        [n_elem] radial levels per element, 3 <= N_r <= 128.
 *   xi0             radial coordinate of the innermost level (the paper uses
 *                   1e-3 in place of the singular centre xi = 0).
 * Levels are xi_j = xi0 + j (1 - xi0) / (N_r - 1).  Every segment must have
 * a positive det J_b (the centre sees the loop counter-clockwise), else
 * SBFWI_EINVAL.  Builds the node -> (element, slot) map used to assemble
 * element sources by gather, and the sparsity pattern of the coarse matrix.
 * Synchronous; *out is owned by the caller (sbfwi_destroy_mesh).
 */
int sbfwi_build_mesh(const double* host_node_xy, int64_t n_nodes,
                     const int64_t* host_elem_ptr, const int64_t* host_elem_nodes,
                     int64_t n_elem, const double* host_centre_xy,
                     const int32_t* host_n_r, double xi0, sbfwi_mesh* out);

/* Sizes of a mesh: host_out[0] = n_nodes, [1] = n_elem, [2] = n_params (fine grid),
 * [3] = nnz of the coarse matrix, [4] = interior level-node count sum_e (N_r - 1) n_b. */
int sbfwi_mesh_info(sbfwi_mesh m, int64_t* host_out);

/*
 * sbfwi_factor_elements -- once per model (rho, c, dt): for every element
 * builds the coefficient matrices E0, E1, E2, M0 at each radial level from
 * the boundary Jacobian and the nodal densities (eq. Es), their radial
 * differences (central inside, one-sided at the end levels), the
 * Newmark-discretised three-point block rows theta, phi, psi and the ghost
 * rows of the flux boundary conditions (eq. system), then eliminates the
 * block system level by level as in the paper's condensation to obtain the
 * pivot blocks, the dynamic stiffness S_e and the source map; finally
 * assembles the coarse matrix K_g = sum_e L_e^T S_e L_e on the fixed pattern.
 *   rho     device [n_params] fine-grid density (layout above), > 0.
 *   c       wave speed; dt, beta, gamma the Newmark parameters (beta > 0).
 *   scheme  SBFWI_SCHEME_PAPER_FD: the paper's central differences in xi
 *           (eq. FD; not symmetric, and unstable at strong radial density
 *           contrast); SBFWI_SCHEME_RADIAL_GALERKIN: linear finite elements
 *           between the levels on the semi-weak radial equation (integrated
 *           by parts with the internal flux, natural conditions at xi0 and
 *           xi = 1), E interpolated linearly between levels, 4-point
 *           Gauss-Legendre quadrature per interval, radial mass lumped; the
 *           element system is symmetric and average-acceleration Newmark
 *           conserves its energy (a deviation from the paper, for models
 *           such as voids at a 1e-5 density floor).  Both schemes share the
 *           layout of the factors and every per-step call; the exact gradient
 *           differentiates the scheme that was factored.
 *           SBFWI_SCHEME_LFE: the conventional path of the paper's benchmark
 *           (Section "Low-frequency expansion", eq. simplified and eq. S):
 *           radially constant density (each element's boundary-level values,
 *           the other levels are ignored), element stiffness K_e and mass M_e
 *           on the boundary nodes only: K_e solves the algebraic Riccati
 *           equation (K - E1) E0^-1 (K - E1^T) = E2 (the invariant subspace of
 *           the static radial matrix for the modes bounded at the centre,
 *           obtained on the device by the scaled Newton iteration of the
 *           matrix sign function) and M_e the Lyapunov equation of the
 *           expansion (Newton iteration); the coarse matrix is K_g + a0 M_g;
 *           the time loop is nodal only.  SBFWI_ENOCONV if an iteration does
 *           not settle within 60 steps.
 *           SBFWI_SCHEME_LFE_CONDENSED: the same path with K_e the static
 *           condensation of the element's N_r radial Galerkin levels and M_e
 *           the radial mass seen through its static modes, which converge at
 *           second order in the radial spacing to the Riccati and Lyapunov
 *           solutions.
 *   coarse_solver 0 = BiCGStab with Jacobi preconditioning (K_g is not
 *           symmetric), solved every step to the tolerance of sbfwi_set_solver;
 *           1 = direct: K_g = L U factored here once, in a nested-dissection
 *           order of the nodes (supernodes of the dissection tree, fronts
 *           eliminated without pivoting), every step then solves with the
 *           factors (K_g^T = U^T L^T for the adjoint); the factorisation runs
 *           on the host and its factors are kept on the device.
 * Synchronises s.  SBFWI_ESINGULAR if a pivot block (or, for coarse_solver 1,
 * a pivot of K_g) is zero or not finite.
 * The factors keep a reference to m, which must outlive them.
 */
int sbfwi_factor_elements(sbfwi_mesh m, const double* rho, double c, double dt,
                          double beta, double gamma, int scheme, int coarse_solver,
                          hipStream_t s, sbfwi_factors* out);

/* Solver controls: relative residual tolerance (default 1e-13) and iteration cap (default 500). */
int sbfwi_set_solver(sbfwi_factors f, double rtol, int max_iter);

/* Launch-shape controls; none of them changes any result bit:
 *   param 0:  BiCGStab iterations enqueued as separate kernels per coarse solve (1 .. 1000,
 *             default 13); iterations after convergence are no-ops, and a solve that needs
 *             more continues in one cooperative kernel up to the limit of sbfwi_set_solver.
 *   param 1:  1 = forward runs without full storage replay every time step from HIP graphs
 *             captured at the first step (on a library stream of default priority, ordered
 *             after the caller's stream); 0 = ordinary launches (default).
 *   param 2:  reset the sweep launch plan to the defaults (value ignored).
 *   param 3:  1 = with the direct coarse solver and checkpoints, the backward pass
 *             recomputes the next checkpoint segment on a second library stream (default
 *             priority) while the adjoint steps of the current segment run, into a second
 *             segment store (default; skipped when that store cannot be allocated);
 *             0 = one segment after the other.
 *   param 4:  1 = forward runs with checkpoints (not full storage) also keep every step's
 *             coarse solution (n_nodes x shots x steps doubles, skipped when it does not fit)
 *             and the checkpoint recompute then skips its coarse solves (default);
 *             0 = the recompute solves again.
 *   param 5:  1 = the recover sweep of a time step and the condense sweep of the next one
 *             run as one joint sweep per element (the new w of every level kept in LDS), so
 *             that the state is read once per step, and likewise the transposed recover of
 *             an adjoint step with the transposed condense of the earlier one (default;
 *             classes whose LDS would exceed 48 KB, and plans with a persistent sweep
 *             launch, run the two sweeps in turn); 0 = separate sweeps.
 *   param 6:  (direct coarse solver) the solve programs of the mesh of f -- shared by every
 *             factors handle on that mesh -- are rebuilt with the subtree launches (one block
 *             per subtree, walking its levels) rooted at the shallowest level of the dissection
 *             tree with at least value supernodes (default 512; a value above every level's
 *             count gives one launch per level).  Waits for the device to be idle first.
 *   param 7:  (central-difference scheme) 1 = the transposed sweeps of the n_b <= 16
 *             classes form the rows theta_j, psi_j, P_j of every level from the element's
 *             nodal densities instead of reading them from the factors (default); 0 = read
 *             them.  Both give the same bits.
 *   param 8:  tail store budget in KiB (default 0): a forward run with checkpoints (not full
 *             storage) also keeps, for as many whole checkpoint segments at the end of the
 *             run as this budget holds, every step's unknowns and accelerations, as the
 *             backward pass would recompute them (skipped if the store cannot be allocated);
 *             the exact gradient then recomputes only the segments before them.  The
 *             footprint of sbfwi_plan_bytes does not include it; sbfwi_ckpt_info reports it.
 *             When the run is destroyed its tail store is kept for the next run on that
 *             device that fits in it (allocations of this size take seconds) until
 *             sbfwi_finalize.
 *   param 10 + 3 k + c: shots per block (0 = default, 1, 2, 4, 8, 16) of sweep k (0 condense,
 *             1 recover, 2 transposed condense, 3 transposed recover) for n_b class c
 *             (n_b <= 8, <= 16, <= 24).
 *   param 30 + k: > 0 = sweep k runs as one persistent launch over all classes with this
 *             many shots per block; 0 = one launch per class. */
int sbfwi_set_launch(sbfwi_factors f, int param, int value);

/*
 * Device-memory footprint, in bytes, of a run on mesh m with n_shots shots,
 * n_steps steps and n_ckpt as in sbfwi_forward (an upper bound of what the
 * library allocates): host_out[0] the factors of one model, [1] the checkpoint
 * store kept between sbfwi_forward and the end of sbfwi_adjoint, [2] the work
 * buffers of the forward run, [3] the work buffers of the backward pass (0 if
 * n_ckpt = 0; the residual of sbfwi_gradient counted with at most 64 receivers
 * per shot, and two checkpoint-segment stores, see sbfwi_set_launch param 3);
 * [1] includes the kept coarse solutions (param 4).  A forward + gradient run needs [1] + max([2], [3]) on top of the
 * factors.  For admission control by a caller that shares the device.
 */
int sbfwi_plan_bytes(sbfwi_mesh m, int n_shots, int64_t n_steps, int n_ckpt, int64_t* host_out);

/*
 * Autotuner of the sweep launch plan for runs of n_shots shots on these factors:
 * for every sweep kind and n_b class, each shots-per-block choice (1 .. 16, up to the
 * shot count rounded up to a power of two) is timed on the factors with zero state,
 * as is the single persistent launch over all classes; the fastest plan is kept for
 * later runs (sbfwi_set_launch param 2 resets it).  Synchronous; allocates and frees
 * its own work buffers.
 *   host_out (may be NULL): 24 doubles, for k = 0 .. 3: [6k .. 6k+2] the chosen shots
 *   per block of the three classes (0 = class empty), [6k+3] the persistent launch's
 *   shots per block (0 = not chosen), [6k+4] ms of the best per-class launches,
 *   [6k+5] ms of the best persistent launch.
 */
int sbfwi_autotune(sbfwi_factors f, int n_shots, double* host_out, hipStream_t s);

/*
 * Copies factor data to host memory (for inspection and tests), synchronous.
 *   which = 0: S_e of every element, element after element, row-major n_b x n_b
 *              (sum_e n_b^2 doubles);
 *   which = 1: values of K_g on the CSR pattern of sbfwi_coarse_pattern (nnz doubles);
 *   which = 2: the stored pivot inverses phi~_j^-1, j = 0 .. N_r-2, of every element,
 *              row-major (sum_e (N_r - 1) n_b^2 doubles);
 *   which = 3: G_e = psi_{n+1} psi_n^-1 of every element (sum_e n_b^2 doubles);
 *   which = 4: (expansion schemes) M_e of every element (sum_e n_b^2 doubles; which = 0
 *              then holds K_e);
 *   which = 5: (expansion schemes) values of M_g on the CSR pattern (nnz doubles; which = 1
 *              then holds K_g + a0 M_g).
 * host_dst must hold the documented count.
 */
int sbfwi_copy_factor_data(sbfwi_factors f, int which, double* host_dst);

/* CSR pattern of K_g: host_row_ptr [n_nodes + 1], host_col [nnz]. Synchronous. */
int sbfwi_coarse_pattern(sbfwi_mesh m, int64_t* host_row_ptr, int64_t* host_col);

/*
 * sbfwi_forward -- time loop of the condensed scheme for n_shots shots
 * (Section "Radial discretization": forward sweep of the Newmark residual
 * sources, effective element sources, coarse nodal solve, backward sweep of
 * the interior levels and Newmark update at every level).  Zero initial
 * conditions.  In step k (k = 1 .. n_steps) shot q applies the nodal point
 * force wavelet[q * n_steps + k - 1] at node src_node[q] and records
 * traces[(q * n_rec + r) * n_steps + k - 1] = u^k at node rec_node[r].
 *   src_node [n_shots], rec_node [n_rec]: device int64 node ids.
 *   wavelet  device [n_shots][n_steps]; traces device [n_shots][n_rec][n_steps].
 *   n_ckpt   0: no checkpoints (ckpt_out may be NULL); > 0: states kept every
 *            ceil(n_steps / n_ckpt) steps; -1: ceil(sqrt(n_steps)) of them;
 *            n_ckpt >= n_steps stores every step (full storage).
 *   ckpt_out receives the checkpoint handle (needed by sbfwi_adjoint /
 *            sbfwi_gradient), or NULL.
 * With factors of SBFWI_SCHEME_LFE (or _LFE_CONDENSED) the step is nodal only (F = M_g w + f,
 * (K_g + a0 M_g) U = F, Newmark update) and n_ckpt must be 0.
 * Growth detector (schemes 0 and 1): every step checks each new nodal
 * displacement of shot q against the envelope 10 * 4 k r F_k(q), r the largest
 * 1 / |K_g,ii| and F_k(q) the sum of |wavelet| of shot q over steps 1 .. k.  For a
 * stable system (symmetric K, M) the Newmark response to a point force obeys
 * |u^k| <= k dt (M^-1)_max sum dt |f|, and 4 r approximates dt^2 (M^-1)_max, so
 * stable runs stay below 0.15 of the envelope; the radial finite differences at
 * strong density contrast grow exponentially (the step map has eigenvalues outside
 * the unit circle) and cross it.  The run still completes every step (every kernel
 * exits normally); the call then returns SBFWI_EUNSTABLE (finite values beyond the
 * envelope) or SBFWI_ENONFINITE (a non-finite value), with the first such step in
 * sbfwi_last_error, and the traces and checkpoints are meaningless.
 * Synchronises s at the end.  SBFWI_ENOCONV if the coarse solve fails.
 */
int sbfwi_forward(sbfwi_factors f, int n_shots, int64_t n_steps,
                  const int64_t* src_node, const double* wavelet,
                  int n_rec, const int64_t* rec_node, double* traces,
                  int n_ckpt, sbfwi_ckpt* ckpt_out, hipStream_t s);

/*
 * sbfwi_adjoint -- backward pass for the shots of a checkpointed forward run:
 * forward segments are recomputed from the checkpoints in reverse order and
 * the adjoint state is stepped back in time.
 *   adj_src device [n_shots][n_rec][n_steps]: derivative of the objective with
 *           respect to each recorded trace sample (for the misfit of
 *           eq. misfit this is dt (u - d)).
 *   mode    SBFWI_GRAD_EXACT: exact derivative of the discrete objective with
 *           respect to every fine-grid density (transposed condensation,
 *           transposed coarse solve, zero-lag correlation of the adjoint rows
 *           with the forward unknowns);
 *           SBFWI_GRAD_PAPER_KERNEL: the paper's truncated Frechet kernel
 *           (time integral of the product of forward and back-propagated
 *           velocities at every fine-grid point; the back-propagated field is
 *           the forward scheme driven by the time-reversed adj_src at the
 *           receivers; sign -1 so that it points along the exact gradient).
 *           With SBFWI_GRAD_PER_SHOT or-ed in, every shot gets its own gradient.
 *           Factors of the expansion schemes accept SBFWI_GRAD_PAPER_KERNEL only
 *           (SBFWI_EINVAL otherwise): the kernel at the nodal points, written
 *           to every element's boundary-level entries (interior levels 0).
 *   grad    device [n_params], overwritten with the sum over shots; with
 *           SBFWI_GRAD_PER_SHOT: [n_shots][n_params], one gradient per shot.
 * A run without receivers has no adjoint sources: adj_src may then be NULL and
 * grad is set to zero.  Synchronises s at the end.
 */
int sbfwi_adjoint(sbfwi_factors f, sbfwi_ckpt ck, const double* adj_src, int mode,
                  double* grad, hipStream_t s);

/*
 * sbfwi_gradient -- misfit of eq. misfit, 1/2 sum_shot sum_rec sum_k dt (u - d)^2,
 * into misfit[0] (device), and its gradient via sbfwi_adjoint with
 * adj_src = dt (traces - observed).
 *   observed, traces device [n_shots][n_rec][n_steps] (traces from the run that
 *   made ck).  With SBFWI_GRAD_PER_SHOT in mode, misfit holds n_shots values
 *   (one per shot) and grad [n_shots][n_params].  A run without receivers
 *   (n_rec = 0) has no data: observed and traces may then be NULL, and misfit
 *   and grad are set to zero (synchronously).
 */
int sbfwi_gradient(sbfwi_factors f, sbfwi_ckpt ck, const double* observed,
                   const double* traces, int mode, double* misfit, double* grad,
                   hipStream_t s);

/*
 * sbfwi_misfit -- the waveform misfit of eq. misfit with the rectangle rule,
 * misfit[0] = 1/2 dt sum_i (traces[i] - observed[i])^2 over count samples (one
 * deterministic reduction), and, if residual is not NULL, its derivative with
 * respect to every trace sample, residual[i] = dt (traces[i] - observed[i]) (the
 * adjoint source of sbfwi_adjoint).  All arrays device memory; asynchronous on s.
 */
int sbfwi_misfit(const double* observed, const double* traces, int64_t count, double dt, double* residual,
                 double* misfit, hipStream_t s);

/* Checkpointed run (host values, host_out holds 6): [0] footprint in bytes, [1] checkpoint
 * interval, [2] shots, [3] receivers, [4] steps of the run -- the leading sizes of the
 * adj_src, observed and traces arrays that sbfwi_adjoint and sbfwi_gradient read, and of the
 * per-shot gradients they write (the ABI takes no sizes for those arrays: a caller
 * passing shorter arrays makes the library read and write past them) -- and [5] the steps
 * at the end of the run kept by the tail store (sbfwi_set_launch param 8). */
int sbfwi_ckpt_info(sbfwi_ckpt ck, int64_t* host_out);

/* Nested-dissection structure used by the direct coarse solver (host values):
 * host_out[0] supernodes, [1] depth of the dissection tree (levels = depth + 1),
 * [2] largest supernode, [3] sum of |J|^2, [4] sum of |J| |B_J|, [5] sum of |B_J|,
 * [6] most supernodes on one level. */
int sbfwi_direct_info(sbfwi_mesh m, int64_t* host_out);

/* Launches of the direct solve's forward (dir 0) or backward (dir 1) program,
 * in launch order: host_out[8 k + 0 .. 7] = blocks, lanes per row, LDS vector
 * slots per block, steps, row records, slot records, most rows in one step,
 * and 1 for the launch of subtree blocks (0 for a level of the dissection
 * tree).  *n_launches receives the number of launches; at most cap are
 * written.  EINVAL: NULL arguments, dir not 0 or 1, or a mesh without the
 * dissection order. */
int sbfwi_direct_launches(sbfwi_mesh m, int dir, int64_t* host_out, int cap, int* n_launches);

/* Coarse-solve statistics accumulated on these factors (synchronous):
 * host_out[0] = solves, [1] = total Krylov iterations, [2] = largest iteration count.
 * reset != 0 clears them afterwards. */
int sbfwi_solver_stats(sbfwi_factors f, int64_t* host_out, int reset);

/* Device bytes a factored model holds (host_out[0]). */
int sbfwi_factors_info(sbfwi_factors f, int64_t* host_out);

/*
 * Live kernel timing.  sbfwi_profile(mask) brackets every launch of the kernels
 * whose bit is set with HIP events on the launch stream (bit ids: 0 condense,
 * 1 recover, 2 coarse solve (all its kernels), 3 source gather, 4 nodal
 * update, 5 transposed condense, 6 transposed recover, 7 adjoint gather,
 * 8 adjoint nodal update, 9 exact-gradient contraction, 10 paper-kernel
 * correlation, 11 element factorisation kernels, 12 / 13 / 14 the three per-iteration kernels
 * of the coarse solve (v = K p, t = K s, the x / r / p update), 15 its two
 * start-up kernels, 16 the recover sweep of the checkpoint recompute, which
 * also stores the adjoint's inputs; id 1 counts the other recover sweeps), 17 the
 * time step of sbfwi_fem_forward, 18 the joint sweep (recover of a step and condense
 * of the next, sbfwi_set_launch param 5), 19 its checkpoint-recompute variant with
 * the stores, 20 the joint transposed sweep (transposed recover of an adjoint step and
 * transposed condense of the earlier one); ids 0, 1, 5, 6 and 16 then count only the
 * sweeps that run alone.  A sweep over elements of several n_b classes counts as
 * one launch.  Recorded pairs are accumulated as they complete (the oldest
 * are waited for once many are in flight).  sbfwi_profile_read waits for the
 * rest and writes, for each of the 21 ids, host_out[2 id] = launches and
 * host_out[2 id + 1] = total ms; reset != 0 clears the totals.  One host
 * thread only.
 */
int sbfwi_profile(uint32_t kernel_mask);
int sbfwi_profile_read(double* host_out, int reset);

/*
 * sbfwi_fem_forward -- observed data from a conventional finite element model
 * (Section "Numerical examples": the paper's data come from a finer bilinear
 * finite element model, so that the inversion does not commit the inverse
 * crime).  The scalar wave equation rho u_tt = div(rho c^2 grad u) + f of the
 * governing equations, on nx x ny bilinear rectangles covering [0, lx] x [0, ly]
 * with a free boundary, one density per element, lumped (row-sum) mass and
 * explicit central differences M (u_{k+1} - 2 u_k + u_{k-1}) / dt^2 + K u_k = f_k,
 * u_0 = u_1 = 0.  Time convention as in sbfwi_forward: the point force at
 * t_k = k dt is wavelet[q * n_steps + k - 1] at node src_node[q], and
 * traces[(q * n_rec + r) * n_steps + k - 1] = u(t_k) at node rec_node[r],
 * k = 1 .. n_steps.
 *   Grid nodes: node (i, j) at (i lx / nx, j ly / ny) has id j (nx + 1) + i.
 *   rho_elem  device [ny][nx]: density of element (ie, je) at je nx + ie,
 *             positive and finite (SBFWI_EINVAL otherwise).
 *   src_node  device int64 [n_shots] (1 <= n_shots <= 64); rec_node device
 *             int64 [n_rec]; ids in [0, (nx + 1)(ny + 1)), checked on the host.
 *   wavelet   device [n_shots][n_steps]; traces device [n_shots][n_rec][n_steps].
 * SBFWI_EINVAL if dt exceeds 1 / (c sqrt(1/hx^2 + 1/hy^2)) (the scheme's
 * stability bound from the row sums of M^-1 K).  Work buffers (two wavefields
 * of n_shots (nx + 1)(ny + 1) doubles and the coefficients) are allocated and
 * freed by the call.  Synchronises s.
 */
int sbfwi_fem_forward(int nx, int ny, double lx, double ly, const double* rho_elem, double c, double dt,
                      int n_shots, int64_t n_steps, const int64_t* src_node, const double* wavelet,
                      int n_rec, const int64_t* rec_node, double* traces, hipStream_t s);

/*
 * sbfwi_fem_forward_noalloc -- sbfwi_fem_forward for callers that cannot
 * allocate memory (code near HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same arguments, kernels and results, but no
 * device or host allocation by the library.  The work buffers (padded element
 * coefficients, inverse lumped mass, two wavefields, a status word) live in a
 * static device array of 48 MiB that every GPU the library runs on holds until
 * the process ends; SBFWI_EINVAL, before any launch, when
 * 8 ((nx + 2)(ny + 2) + (nx + 1)(ny + 1)(1 + 2 n_shots)) bytes plus alignment
 * exceed it (the 512 x 256 grid takes 10.6 MB with 4 shots, 35 MB with 16).
 * Node ids are checked on the device (SBFWI_EINVAL before the time loop).
 * Every call on one GPU shares the array and finds the last call's contents
 * (it clears what must start at zero): calls that overlap on one GPU race and
 * must be serialised by the caller.  Synchronises s.
 */
int sbfwi_fem_forward_noalloc(int nx, int ny, double lx, double ly, const double* rho_elem, double c, double dt,
                              int n_shots, int64_t n_steps, const int64_t* src_node, const double* wavelet,
                              int n_rec, const int64_t* rec_node, double* traces, hipStream_t s);

/*
 * sbfwi_finalize -- releases the runtime objects the library owns outside the
 * handles: the per-thread streams of its synchronous copies, the events of the
 * live kernel timing (pending timings are discarded, timing is switched off)
 * and a tail store kept from a destroyed run (sbfwi_set_launch param 8).  Waits for the device first.  Handles stay valid; later calls create
 * what they need again.  Call it after the last handle is destroyed and before
 * the process tears down the HIP runtime, so that no library-owned stream or
 * event outlives the caller's own teardown.  Not to be called while another
 * thread is inside the library.
 */
int sbfwi_finalize(void);

void sbfwi_destroy_mesh(sbfwi_mesh m);
void sbfwi_destroy_factors(sbfwi_factors f);
void sbfwi_destroy_ckpt(sbfwi_ckpt ck);

#ifdef __cplusplus
}
#endif
#endif /* SBFWI_H */

/*
 * hfmm.h -- C-ABI of libhfmm.so: a 2-D Helmholtz fast multipole method used
 * as a matrix-free preconditioner (coupled to a boundary-element correction
 * for Dirichlet boundaries) inside right-preconditioned restarted flexible
 * GMRES on the 5-point finite-difference Helmholtz system.  MI355X (gfx950).
 *
 * Paper: Ibeid, Yokota, Keyes, "A Matrix-free Preconditioner for the Helmholtz
 * Equation based on the Fast Multipole Method".
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Pointers named d_* are DEVICE pointers owned by the caller.  The library
 *   never frees them and keeps no reference to them after the call returns;
 *   the caller keeps them alive until the work queued on `stream` completes.
 * - Complex arrays are interleaved (re, im).  Multi-column arrays are
 *   column-major: column c of an n x nrhs array starts at element c * n.
 * - `stream` is a hipStream_t (NULL = the default stream).  Calls queue their
 *   kernels on it and return without synchronising unless stated otherwise.
 * - Every call returns an hfmm_status.  Invalid arguments are rejected with
 *   HFMM_ERR_ARG before any kernel is launched, except where a check needs
 *   device data (stated at the call).  HIP failures map to HFMM_ERR_HIP.
 *   hfmm_last_error() returns a thread-local message for the last non-OK
 *   status of the calling thread.  No C++ exception crosses this interface.
 * - Handles are not thread-safe; use one stream per handle at a time.
 */
#ifndef HFMM_H
#define HFMM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HFMM_OK = 0,
  HFMM_NOT_CONVERGED = 1,   /* a solve ended at maxit; x holds the last iterate */
  HFMM_ERR_ARG = -1,        /* invalid argument (message says which) */
  HFMM_ERR_HIP = -2,        /* a HIP runtime call failed */
  HFMM_ERR_OOM = -3,        /* device allocation failed */
  HFMM_ERR_STATE = -4,      /* handle used in a state that does not allow the call */
  HFMM_ERR_INTERNAL = -5,   /* internal inconsistency (a bug) */
  HFMM_ERR_NUMERIC = -6     /* NaN/Inf met in a solve, or a singular boundary matrix */
} hfmm_status;

typedef enum { HFMM_FP64 = 0, HFMM_FP32 = 1 } hfmm_precision;

typedef struct hfmm_tree_s* hfmm_tree;
typedef struct hfmm_solver_s* hfmm_solver;

typedef struct {
  int32_t iters;          /* Arnoldi steps (max over right-hand sides) */
  int32_t restarts;       /* restart cycles run (max over right-hand sides) */
  int32_t converged;      /* 1 if every right-hand side met rtol */
  int32_t nrhs;
  double rel_res_true;    /* max over columns of ||b - A x|| / ||b|| at exit */
  double rel_res_est;     /* max over columns of the Givens estimate at exit */
  double ms_precond;      /* device time in preconditioner applies (ms); 0 when not
                             measured (batched solves) */
  double ms_krylov;       /* device time of the rest of the Arnoldi steps: FD matvec,
                             CGS2, norms, Givens (ms); 0 when not measured */
  double ms_total;        /* wall time of the solve call (ms) */
  double ms_setup;        /* wall time of hfmm_solver_create for this solver (ms) */
} hfmm_solve_info;

/* Thread-local text of the last non-OK status on this thread ("" if none). */
const char* hfmm_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int32_t hfmm_version(void);

/* ------------------------------------------------------------------------
 * Hierarchical decomposition (Sec. 5.1.1): uniform quad-tree over the root
 * square [x0, x0+side] x [y0, y0+side], Morton-ordered leaves.
 *
 * d_xy      n points, (x, y) interleaved FP64, device, caller order.
 * leaf_size target mean leaf occupancy: depth L = max(2, ceil(log4(n/leaf)))
 *           (smallest L with leaf*4^L >= n); leaf_size = 0 gives a single leaf
 *           (every pair is near: the all-pairs sum).  L <= 12.
 * out       receives a library-owned handle (sorted points, permutation, leaf
 *           offsets, and a cache of per-(k, p, precision) translation plans).
 * Errors: n < 1, side <= 0, leaf_size < 0, non-finite or out-of-root
 * coordinates (checked on the device by the first kernel; the call then
 * returns HFMM_ERR_ARG and creates nothing).  Synchronises `stream`.
 * ---------------------------------------------------------------------- */
hfmm_status hfmm_build_tree(const double* d_xy, int64_t n, double x0, double y0, double side,
                            int32_t leaf_size, hipStream_t stream, hfmm_tree* out);

/* Depth and counts of a tree: any output pointer may be NULL. */
hfmm_status hfmm_tree_info(hfmm_tree t, int32_t* levels, int64_t* n_points, int64_t* n_leaves,
                           int32_t* max_leaf_count);

/* Copy the tree's sort permutation (sorted slot -> caller index, int32, n) and
 * leaf offsets (int32, n_leaves + 1, Morton order) to device buffers.  Either
 * pointer may be NULL.  Async on stream. */
hfmm_status hfmm_tree_export(hfmm_tree t, int32_t* d_perm, int32_t* d_leaf_off, hipStream_t stream);

hfmm_status hfmm_tree_destroy(hfmm_tree t);

/* Options of the plans made on this tree from now on (cached plans are
 * dropped, so the next apply rebuilds them):
 * m2l_valu   0: M2M, M2L and L2L on the matrix cores (MFMA, the default);
 *            1: the same translations on the vector units (a reference path
 *               for checking the MFMA kernels, and an ablation).
 * autotune   1: time the near-field lanes per target and the M2L target tile
 *               on this tree when a plan is made (the default); 0: use the
 *               tuning cache if it has the plan's key, else fixed defaults.
 * Errors: values other than 0 and 1. */
hfmm_status hfmm_tree_set_options(hfmm_tree t, int32_t m2l_valu, int32_t autotune);

/* Accuracy experiment for the preconditioner-accuracy study (Sec. 6.1: a
 * preconditioner need not be accurate): the operands of the matrix-core M2L
 * (the translation matrices and the multipole coefficients) are rounded to
 * FP16 (mode 1) or BF16 (mode 2), round to nearest even, before FP32
 * products accumulated in FP32, which is what a 16-bit-input matrix-core
 * product computes.  FP32 plans only (FP64 plans ignore it); levels whose
 * window runs on the VALU kernel are not rounded.  For FP16 each level's
 * table is scaled by a power of two into the format's range and the
 * products are scaled back (exact); the multipole coefficients must fit
 * FP16 as they are.  Mode 0 turns it off.  Cached plans are dropped.
 * Errors: mode outside 0..2. */
hfmm_status hfmm_tree_set_m2l_input_rounding(hfmm_tree t, int32_t mode);

/* ------------------------------------------------------------------------
 * N-body sum (Sec. 5.1, the N-body sum) with the 2-D Helmholtz kernel
 * G = (i/4) H0^(1)(k r) (Sec. 5.2), evaluated by the FMM of Sec. 5.1.2:
 *   phi[i, c] = sum_{j : |x_i - x_j| > 0} q[j, c] (i/4) H0^(1)(k |x_i - x_j|)
 * in the caller's point order.  Pairs at zero distance add nothing.
 *
 * k     wavenumber > 0.   p  leaf expansion order, 1..40; level l uses
 *       p_l = p + floor(k d_l / 2) (d_l the box diagonal), 2 p_l + 1 terms.
 * prec  HFMM_FP64: q, phi complex128, FP64 arithmetic.
 *       HFMM_FP32: q, phi complex64, FP32 arithmetic.
 * d_q   n x nrhs complex, device.   d_phi  n x nrhs complex, overwritten.
 * The first call for a (k, p, prec) builds and caches its translation plan
 * (host tables, uploaded synchronously).  Async on stream afterwards.
 * The plan holds the work arrays of the apply (expansions, the M2L's
 * class-group partial sums and counters): applies on one tree must not
 * overlap in time (different streams without ordering, or threads).
 * Errors: k <= 0, p out of range, nrhs < 1, leaves too large for k
 * (k * leaf_side / sqrt(2) above 6), FP32 tables that
 * would overflow.
 * ---------------------------------------------------------------------- */
hfmm_status hfmm_fmm_apply(hfmm_tree t, double k, int32_t p, hfmm_precision prec,
                           const void* d_q, void* d_phi, int32_t nrhs, hipStream_t stream);

/* The same apply without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments, results and errors as hfmm_fmm_apply; the
 * work arrays (expansions of every level, far field, sorted charges) come
 * from a fixed device array of hfmm_fmm_noalloc_capacity() bytes (64 MiB)
 * that each GPU the library runs on holds until the process ends.
 * - The plan of (k, p, prec) must already exist on the tree (made by
 *   hfmm_fmm_plan_info or an earlier hfmm_fmm_apply); else HFMM_ERR_STATE.
 * - An apply that needs more work memory than the array holds (about
 *   2 coefficients-per-box x nrhs + 2 N nrhs complex values) is rejected
 *   with HFMM_ERR_ARG before any launch.
 * - Every call on a GPU shares that GPU's array: calls that overlap on one
 *   GPU (other streams or threads) race.  The M2L's class-group partial
 *   sums and counters belong to the plan (allocated with it), so a call must
 *   not overlap another apply on the same tree either.  Async on stream. */
hfmm_status hfmm_fmm_apply_noalloc(hfmm_tree t, double k, int32_t p, hfmm_precision prec,
                                   const void* d_q, void* d_phi, int32_t nrhs, hipStream_t stream);

/* Bytes of the fixed work array of hfmm_fmm_apply_noalloc. */
int64_t hfmm_fmm_noalloc_capacity(void);

/* The same apply with hipEvents around its stages (tracing): ms_stages
 * (host, 9 floats) receives device times in ms.  On a tree of depth >= 2:
 * [1] P2M (which also gathers the charges into Morton order), [2] the
 * far-field chain M2M + M2L + L2L + L2P, which runs on the tree's second
 * stream beside [4] the near field (P2P) on trees of 2^18 points or more
 * (after it on smaller ones), and [3] the sum of both written in caller
 * order, including the wait for [2]; [0] and [5] are 0.  The chain's parts,
 * timed on the stream they run on: [6] the M2M levels, [7] the M2L launch,
 * [8] the L2L levels and the L2P (with the option m2l_valu the whole chain
 * counts under [8] and [6], [7] are 0).  On a single leaf: [0] the gather,
 * [4] the direct sum, [5] the scatter, the rest 0.  Synchronises `stream`. */
hfmm_status hfmm_fmm_apply_timed(hfmm_tree t, double k, int32_t p, hfmm_precision prec,
                                 const void* d_q, void* d_phi, int32_t nrhs, float* ms_stages,
                                 hipStream_t stream);

/* Plan facts for a (k, p, prec) on a tree (builds the plan if needed).
 * orders     host, levels+1 ints: p_l per level (levels < 2: only the near field).
 * near_deg   coefficients of the near-field H0 polynomial (0 when the
 *            full-range routine is used because the pair arguments exceed 12).
 * pairs      near-field source-target pairs per column, self pairs excluded.
 * Any output may be NULL. */
hfmm_status hfmm_fmm_plan_info(hfmm_tree t, double k, int32_t p, hfmm_precision prec, int32_t* orders,
                               int32_t* near_deg, int32_t* lanes_per_target, int64_t* pairs);

/* Double-layer sum (the dG/dn kernel of Sec. 5.2, 2-D form) by the same FMM:
 *   phi[i, c] = sum_{j : |x_i - x_j| > 0} q[j, c] dG/dn_j(x_i, x_j),
 *   dG/dn_j(x, y) = (i k / 4) H1^(1)(k r) (x - y).n_j / r,  r = |x - y|,
 * the derivative of G(x, y) at the source y along its unit normal n_j.  The
 * sources become dipoles in P2M (exact in the expansion order) and in the
 * near field; M2M, M2L, L2L and L2P are the single-layer ones.
 * d_normals  n x 2 FP64 (n_x, n_y) per point, caller order, device.
 * Other arguments and errors as hfmm_fmm_apply.  Async. */
hfmm_status hfmm_fmm_apply_dipole(hfmm_tree t, double k, int32_t p, hfmm_precision prec, const void* d_q,
                                  const double* d_normals, void* d_phi, int32_t nrhs, hipStream_t stream);

/* Tuning cache (process-wide): the launch shapes the autotuner chose,
 * keyed by the device architecture, precision, tree depth, mean leaf
 * occupancy, level orders, near-field polynomial and column-group width.
 * save writes it to a text file; load adds a file's entries (count in
 * *n_loaded, may be NULL), which later plans with the same key take without
 * timing.  size returns the number of entries; clear empties the cache.
 * Errors: unreadable/unwritable file, malformed line. */
hfmm_status hfmm_tune_cache_save(const char* path);
hfmm_status hfmm_tune_cache_load(const char* path, int32_t* n_loaded);
int32_t hfmm_tune_cache_size(void);
hfmm_status hfmm_tune_cache_clear(void);

/* ------------------------------------------------------------------------
 * 5-point FD Helmholtz operator (the sparse system A x = b of Sec. 2) on the
 * n x n interior grid of the unit square, zero Dirichlet ghosts:
 *   (A x)_ij = (4 x_ij - x_{i-1,j} - x_{i+1,j} - x_{i,j-1} - x_{i,j+1}) / h^2 - k2_ij x_ij
 * d_k2   n*n FP64 k^2 field (device), or NULL to use k2_const.
 * d_x    n*n x nrhs complex128, lexicographic (x index fastest).
 * d_y    n*n x nrhs complex128, overwritten.  Always FP64.  Async.
 * ---------------------------------------------------------------------- */
hfmm_status hfmm_fd_helmholtz_matvec(int32_t n, double h, const double* d_k2, double k2_const,
                                     const double* d_x, double* d_y, int32_t nrhs, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Solver for A u = f on the n x n grid, h = 1/(n+1), with the FMM-BEM
 * preconditioner of Sec. 5.2-5.3 at the constant wavenumber k0:
 *   z = M^{-1} r:  pass 1  V = FMM(sources h^2 r at the interior nodes)
 *                  boundary  q = -S^{-1} V_Gamma (Dirichlet boundary equation)
 *                  pass 2  z = V_Omega + S_vol r + FMM(sources w q at the
 *                          boundary element midpoints), interior equation.
 * Boundary: 4(n+1) constant elements of width w = h, midpoint collocation, no
 * corner nodes (Sec. 5.3); S diagonal from the analytic formula of Sec. 5.3.
 * S is assembled and inverted in FP64 on the device at creation.
 *
 * d_k2/k2_const  the operator's k^2 field (copied), as in the matvec.
 * k0             preconditioner wavenumber (> 0).
 * p, leaf_size   FMM order and leaf occupancy; leaf_size = 0 times one
 *                preconditioner apply on the trees of leaf sizes 16, 32 and 64
 *                and keeps the fastest (hfmm_solver_info reports the choice).
 * precond_prec   HFMM_FP32: the whole preconditioner runs in complex64 (the
 *                Krylov part stays FP64); HFMM_FP64: all FP64.
 * nrhs           columns solved together (independent Krylov spaces, one
 *                batched preconditioner apply).
 * Synchronises `stream`.
 * ---------------------------------------------------------------------- */
hfmm_status hfmm_solver_create(int32_t n, double h, const double* d_k2, double k2_const, double k0,
                               int32_t p, int32_t leaf_size, hfmm_precision precond_prec,
                               int32_t nrhs, hipStream_t stream, hfmm_solver* out);

/* Preconditioner wavenumber matched to the 5-point stencil's dispersion: the
 * mean of the discrete wavenumbers of a plane wave at k along a grid axis,
 * (2/h) asin(k h/2), and along a diagonal, (2 sqrt2/h) asin(k h/(2 sqrt2)).
 * The continuous Green's function of the preconditioner (Sec. 5.2) then keeps
 * the phase of the discrete operator's waves; k0 = k is the paper's choice.
 * Host only; ERR_ARG when k h >= 2 or an argument is not positive. */
hfmm_status hfmm_matched_wavenumber(double k, double h, double* k0);

/* Replace the operator's k^2 field (preconditioner unchanged).  Async. */
hfmm_status hfmm_solver_set_k2(hfmm_solver s, const double* d_k2, double k2_const, hipStream_t stream);

/* Replace the operator's k^2 field by one constant on nb x nb square blocks
 * of (n/nb)^2 nodes each: d_kb is nb*nb FP64, row-major, block row index
 * following y (node (i, j) takes d_kb[(j / (n/nb)) nb + i / (n/nb)]).  The
 * library expands it on the device.  Errors: nb < 1 or nb not dividing n.
 * Async. */
hfmm_status hfmm_solver_set_k2_blocks(hfmm_solver s, const double* d_kb, int32_t nb, hipStream_t stream);

/* Gradient product of the adjoint method: with u the solution of A u = f and
 * mu the solution of A^H mu = dJ/du (both n*n complex128, device), dA/dk^2_x
 * = -e_x e_x^T gives dJ/dk^2_x = Re(conj(mu_x) u_x) = -Re(lambda_x u_x) for
 * lambda = -conj(mu).  d_grad (nb*nb FP64, device) receives the sums over the
 * nb x nb blocks of set_k2_blocks (nb = n: one value per node).  Blocks are
 * summed row by row in a fixed order (deterministic).  Async. */
hfmm_status hfmm_k2_gradient(int32_t n, const double* d_u, const double* d_mu, int32_t nb, double* d_grad,
                             hipStream_t stream);

/* z = M^{-1} r for nrhs columns (complex128 n*n x nrhs in and out).  Async. */
hfmm_status hfmm_precond_apply(hfmm_solver s, const double* d_r, double* d_z, int32_t nrhs,
                               hipStream_t stream);

/* Right-preconditioned FGMRES(restart) (Sec. 3-4): x0 from d_x (zeros for the
 * paper's setting), stop when ||b - A x|| / ||b|| <= rtol for every column
 * (true residual, checked at the end of each cycle), at most maxit Arnoldi
 * steps.  CGS2 orthogonalisation, complex Givens rotations, all FP64.
 * d_b, d_x   n*n x nrhs complex128 (nrhs as created).
 * transpose  1 solves A^T x = b with the same preconditioner.  For this FD
 *            operator with a real k^2 field A^T = A, and M^{-1} is complex
 *            symmetric, so both settings run the same iteration.
 * info       host struct, filled on return (may be NULL).
 * Returns HFMM_OK, HFMM_NOT_CONVERGED, or an error.  Synchronises `stream`. */
hfmm_status hfmm_fgmres_solve(hfmm_solver s, const double* d_b, double* d_x, int32_t restart,
                              int32_t maxit, double rtol, int32_t transpose, hfmm_solve_info* info,
                              hipStream_t stream);

/* The same solve for nprob solvers at once: d_b[i], d_x[i] belong to s[i].
 * Restart cycles run in lockstep.  With several problems each runs its
 * Arnoldi steps on a stream of its own (forked from and joined to `stream`),
 * so that their kernels overlap on the device.
 * use_graph = 1 captures one Arnoldi step of each problem once per call into
 * a hipGraph of its own (the step reads its index and flags from device
 * memory) and replays it: 4 replays per problem between two reads of the
 * flags, a finished column or problem making every later kernel of it
 * return at once (device-side early exit).  use_graph = 0 launches the same
 * kernels eagerly, one step at a time, with the flags read after every
 * step.  info has nprob entries.  Synchronises `stream`. */
hfmm_status hfmm_fgmres_solve_batched(hfmm_solver* s, int32_t nprob, const double* const* d_b,
                                      double* const* d_x, int32_t restart, int32_t maxit, double rtol,
                                      int32_t use_graph, hfmm_solve_info* info, hipStream_t stream);

/* The boundary-element solution with inhomogeneous Dirichlet data (Sec. 5.2,
 * the boundary equation with its 1/2 delta and double-layer terms, then the
 * interior equation; constant elements and the analytic diagonal of Sec. 5.3):
 *   boundary  S q = g/2 + D[g] - V     at the element midpoints,
 *   interior  u = V + S_vol f + sum_b w G q_b - D[g]   at the interior nodes,
 * with V the volume potential of f (h^2 weights), D[g] the double layer
 * sum_b w g_b dG/dn_b, w = h, all sums by the solver's FMM (wavenumber k0,
 * precision as created).  With g = 0 this is hfmm_precond_apply.
 * d_f  n*n x nrhs complex128 source.  d_g  4(n+1) x nrhs complex128 values
 * at the element midpoints in the order of hfmm_solver_boundary_nodes.
 * d_u  n*n x nrhs complex128, overwritten.  nrhs as created.  Async. */
hfmm_status hfmm_dirichlet_apply(hfmm_solver s, const double* d_f, const double* d_g, double* d_u, int32_t nrhs,
                                 hipStream_t stream);

/* The 4(n+1) boundary element midpoints, (x, y) interleaved FP64 into d_xy
 * (device): bottom side (y = 0), right (x = 1), top (y = 1), left (x = 0),
 * each with the free coordinate (m + 1/2) h, m = 0..n.  Async. */
hfmm_status hfmm_solver_boundary_nodes(hfmm_solver s, double* d_xy, hipStream_t stream);

/* Right-preconditioned BiCGSTAB (van der Vorst's method, the short-recurrence
 * alternative of Sec. 3) with the solver's operator and FMM-BEM
 * preconditioner: two preconditioner applies and two matvecs per iteration,
 * FP64 vectors and scalars on the device, conj(a).b inner products.  Stops
 * when ||b - A x|| / ||b|| <= rtol for every column (recursive residual,
 * the true residual is computed at exit and decides info->converged), or
 * after maxit iterations, or on breakdown of a column (a zero denominator).
 * d_b, d_x as hfmm_fgmres_solve (x0 read from d_x).  info->iters counts
 * BiCGSTAB iterations.  Returns HFMM_OK, HFMM_NOT_CONVERGED or an error.
 * Synchronises `stream`. */
hfmm_status hfmm_bicgstab_solve(hfmm_solver s, const double* d_b, double* d_x, int32_t maxit, double rtol,
                                hfmm_solve_info* info, hipStream_t stream);

/* Diagnostics of a solver: N_Gamma, the 1-norm condition estimate
 * ||S||_1 ||S^{-1}||_1 of the boundary matrix, the tree depth and the leaf
 * size in use (host outputs, each may be NULL). */
hfmm_status hfmm_solver_info(hfmm_solver s, int32_t* n_gamma, double* cond_S, int32_t* levels, int32_t* leaf_size);

/* hfmm_tree_set_m2l_input_rounding for the solver's FMM passes; the plan is
 * rebuilt before returning (so a later captured solve allocates nothing).
 * Synchronises the device.  Errors: NULL solver, mode outside 0..2. */
hfmm_status hfmm_solver_set_m2l_input_rounding(hfmm_solver s, int32_t mode);

hfmm_status hfmm_solver_destroy(hfmm_solver s);

/* ------------------------------------------------------------------------
 * 3-D FMM on an oct-tree (the 3-D decomposition of Sec. 5.1.1, the 3-D
 * Green's function G = exp(i k r) / (4 pi r) of Sec. 5.2, the calculation
 * flow of Sec. 5.1.2).
 *
 * hfmm3_build_tree: uniform oct-tree over the cube [x0, x0+side] x
 * [y0, y0+side] x [z0, z0+side].
 *   d_xyz      n x 3 FP64 (x, y, z) per point, device, caller-owned, read
 *              during the call only.
 *   leaf_size  >= 1; depth L = max(2, smallest L with leaf_size 8^L >= n),
 *              at most 7.
 * Errors: n < 1 or >= 2^30, side <= 0, a point outside the cube or
 * non-finite (checked on the device, HFMM_ERR_ARG, nothing created), depth
 * above 7.  Synchronises `stream`. */
typedef struct hfmm3_tree_s* hfmm3_tree;
hfmm_status hfmm3_build_tree(const double* d_xyz, int64_t n, double x0, double y0, double z0, double side,
                             int32_t leaf_size, hipStream_t stream, hfmm3_tree* out);
/* levels, points, leaves (8^L) and the largest leaf; each output may be NULL. */
hfmm_status hfmm3_tree_info(hfmm3_tree t, int32_t* levels, int64_t* n_points, int64_t* n_leaves,
                            int32_t* max_leaf_count);
hfmm_status hfmm3_tree_destroy(hfmm3_tree t);

/* phi[i] = sum_{j : |x_i - x_j| > 0} G(|x_i - x_j|) q[j], caller order.
 * k     wavenumber > 0.   p  leaf expansion order, 1..20; level l uses
 *       p_l = p + floor(k d_l / 2) (d_l the box diameter sqrt(3) side / 2^l),
 *       (p_l + 1)^2 coefficients, each at most 20.
 * prec  HFMM_FP64: q, phi complex128.  HFMM_FP32: complex64, FP32 arithmetic.
 * d_q   n complex, device.   d_phi  n complex, device, overwritten.
 * The first call for a (k, p, prec) builds and caches the plan: the
 * translation tables (M2L for the 316 offsets of each level, M2M and L2L for
 * the 8 child positions), built on the host and uploaded synchronously, and
 * the expansion arrays.  Async on stream afterwards: the far-field chain
 * (P2M, M2M, M2L, L2L) runs on a second stream owned by the tree, forked from
 * and joined back to `stream` by events, beside the near field (P2P).
 * Applies on one tree must not overlap in time.
 * Errors: k <= 0, p out of range, an order above 20, leaves too large for k
 * (k times the leaf half-diagonal above 6), FP32 tables that would overflow,
 * a tree of depth < 2. */
hfmm_status hfmm3_fmm_apply(hfmm3_tree t, double k, int32_t p, hfmm_precision prec, const void* d_q,
                            void* d_phi, hipStream_t stream);

/* The same apply with hipEvents between its stages, which then run one
 * after another on `stream` (no overlap): ms_stages (host, 6 floats) receives [0] the upward pass (charge gather, P2M, M2M), [1] the
 * M2L of every level, [2] the L2L levels, [3] the P2P, [4] the L2P (which
 * adds the near field and writes caller order) and [5] the total, in ms.
 * Synchronises `stream`. */
hfmm_status hfmm3_fmm_apply_timed(hfmm3_tree t, double k, int32_t p, hfmm_precision prec, const void* d_q,
                                  void* d_phi, float* ms_stages, hipStream_t stream);

/* Expansion order of each level (host, levels + 1 ints). */
hfmm_status hfmm3_fmm_orders(hfmm3_tree t, double k, int32_t p, int32_t* orders);

/* ------------------------------------------------------------------------
 * The 3-D model problem (Sec. 7, eq. helm3, with kappa = k > 0): the 7-point
 * finite-difference system A u = b, A = -Laplace_h - k^2 on the n^3 interior
 * nodes (i h, j h, l h) of the unit cube, h = 1/(n+1), x fastest, zero
 * Dirichlet data.  Vectors are complex128, interleaved, device, n^3 values.
 *
 * hfmm3_fd_matvec: y = A x.  Errors: n outside [1, 1024], aliasing.  Async. */
hfmm_status hfmm3_fd_matvec(int32_t n, double k2, const double* d_x, double* d_y, hipStream_t stream);

/* A solver of that system whose right preconditioner is the volume
 * potential of the residual by the oct-tree FMM (the 3-D counterpart of the
 * preconditioner's first pass, Sec. 4-5; no boundary-element correction for
 * the cube's faces):
 *   z_i = h^3 sum_{j != i} G(|x_i - x_j|) r_j + c_self r_i,  G = exp(i k r)/(4 pi r),
 * c_self = the integral of G over the node's cell.  The tree is built over
 * the nodes with leaf_size; the FMM runs at order p in precond_prec (the
 * Krylov vectors stay FP64).  Creation builds the tree and the FMM plan
 * (synchronises `stream`).  Errors: n outside [2, 512], k <= 0, p outside
 * [1, 20], the FMM plan's own errors. */
typedef struct hfmm3_solver_s* hfmm3_solver;
hfmm_status hfmm3_solver_create(int32_t n, double k, int32_t p, int32_t leaf_size, hfmm_precision precond_prec,
                                hipStream_t stream, hfmm3_solver* out);
/* z = M^{-1} r (r, z: n^3 complex128, device, not aliased).  Async. */
hfmm_status hfmm3_precond_apply(hfmm3_solver s, const double* d_r, double* d_z, hipStream_t stream);
/* Right-preconditioned FGMRES(restart), CGS2, from x0 = d_x; stops when
 * ||b - A x|| / ||b|| <= rtol (true residual at each cycle start) or after
 * maxit steps.  restart in [1, 200].  info (host, may be NULL) as for the
 * 2-D solve (nrhs 1).  Returns HFMM_OK, HFMM_NOT_CONVERGED, HFMM_ERR_NUMERIC
 * or an argument error.  Synchronises `stream`. */
hfmm_status hfmm3_fgmres_solve(hfmm3_solver s, const double* d_b, double* d_x, int32_t restart, int32_t maxit,
                               double rtol, hfmm_solve_info* info, hipStream_t stream);
/* c_self (host, 2 doubles: re, im), the tree depth and the set-up time (ms);
 * each output may be NULL. */
hfmm_status hfmm3_solver_info(hfmm3_solver s, double* self_term, int32_t* levels, double* ms_setup);
hfmm_status hfmm3_solver_destroy(hfmm3_solver s);

#ifdef __cplusplus
}
#endif

#endif /* HFMM_H */

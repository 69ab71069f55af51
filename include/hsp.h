/*
 * hsp.h - C ABI of the MI355X two-grid sweeping preconditioner library.
 *
 * Method: C. C. Stolk, "An improved sweeping domain decomposition
 * preconditioner for the Helmholtz equation" (arXiv 1412.0464).
 *
 * Problem (Sec. 1, Sec. 2.1): -Laplace u - k^2 u = f with k = omega / c on a
 * rectangle, truncated by PML layers (d/dx -> alpha d/dx, alpha = 1/(1 +
 * i sigma/omega), sigma = C dist^2, C = S c_pml / d^3) and homogeneous
 * Dirichlet values outside.  Time factor exp(-i omega t): outgoing waves
 * behave like exp(+i k r).
 *
 * Mesh (Sec. 2.2): N = n + 1 + 2 w cells per axis (n interior nodes, w
 * outer-PML cells on each side), spacing h, unknowns at nodes 1..N-1.
 * Vectors are dense arrays over the unknown nodes with the x axis (the
 * sweep axis) slowest: index (i-1)*(N2-1) + (k-1) for node (i, k); in 3-D
 * (hsp_grid.dim = 3, Sec. 6.2) index ((i-1)*(N2-1) + (j-1))*(N3-1) + (k-1)
 * for node (i, j, k), z fastest.
 * Complex vectors are interleaved (re, im) pairs of double ("complex128").
 *
 * Memory and streams.  Every pointer named *_dev is a device pointer on the
 * current HIP device.  The caller owns all of them, including the workspace
 * passed to hsp_setup; the library never allocates device memory (the
 * allocation-free batched entry point uses a fixed device array of the
 * library instead).  All work
 * is enqueued on the HIP stream passed in (NULL = the default stream); a call
 * blocks the host only where it must read a result (setup status, solve
 * iterations).  A handle may be used from one host thread at a time.
 *
 * Errors.  Every function returns an hsp_status; 0 is success.  Nothing is
 * thrown across the ABI.  hsp_last_error() returns a message for the last
 * failure on the calling thread.
 */
#ifndef HSP_H
#define HSP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HSP_OK = 0,
  HSP_EINVAL = -1,     /* invalid argument: nothing was enqueued            */
  HSP_ENOMEM = -2,     /* workspace smaller than hsp_workspace_size        */
  HSP_ESINGULAR = -3,  /* zero or non-finite pivot in a slab factorization,
                          or Schur-complement growth beyond the limit      */
  HSP_ENOCONV = -4,    /* maxit reached; the last iterate is returned      */
  HSP_EDEVICE = -5     /* a HIP runtime call failed                        */
} hsp_status;

enum { HSP_SWEEP_X = 0, HSP_SWEEP_UD = 1, HSP_SWEEP_NX = 2 };
enum { HSP_FP64 = 0, HSP_MIXED = 1 };
enum { HSP_SLAB_AUTO = 0, HSP_SLAB_BLOCK = 1, HSP_SLAB_ND = 2 };

typedef struct hsp_ctx* hsp_handle;

/* Geometry of the fine mesh. */
typedef struct hsp_grid {
  int dim;          /* 2 or 3 (other values: HSP_EINVAL)                      */
  int n[3];         /* interior nodes per axis, x first                       */
  double h;         /* mesh spacing                                            */
  int pml[3];       /* outer PML cells per side, per axis (>= 0)               */
  double S_outer;   /* outer PML strength S; <= 0 selects 5 * pml[0]           */
  double c_pml;     /* PML reference speed c_pml; <= 0 selects mean(c)        */
  int sponge;       /* 0: the pml[a] outer cells are PML layers.  1 (2-D,
                       fine_stencil 5): they are sponge layers instead
                       (Sec. 2.1): no PML, k replaced by k (1 + i beta) with
                       beta = beta_max (dist/d)^2 per axis (summed in the
                       corners), beta_max = S_outer, or for S_outer <= 0 the
                       value that damps a crossing wave by 1e-2 at c_pml
                       (3 ln 100 / (k d), d the layer width).  With two_grid
                       the coarse mesh then coarsens every cell (the two-grid
                       method in absence of PML layers, Sec. 4: full
                       weighting and linear interpolation), and the slab
                       partition spreads over all layers.                   */
} hsp_grid;

/* Method parameters (Sec. 4, Sec. 6.1). */
typedef struct hsp_options {
  int fine_stencil; /* 5: the 5-point PML finite differences of eq.
                       define_pml_fd (the paper's fine level); 9: the
                       finite-element 9-point form (App. A) with Table (a)
                       coefficients at the fine 1/G                           */
  int two_grid;     /* 0: the sweep acts on the fine operator itself;
                       1: two-grid sweeping preconditioner (TGSP, Sec. 4): the
                       sweep acts on the optimized 9-point FE operator of the
                       PML-aware coarse mesh (App. A)                         */
  int w_dd;         /* DD-PML layers added to each slab side (>= 1)           */
  double S_dd;      /* DD-PML strength; <= 0 selects 5 * w_dd                  */
  int nu;           /* omega-Jacobi pre- and post-smoothing steps             */
  double omega_jac; /* Jacobi weight                                           */
  int sweep;        /* HSP_SWEEP_X (SweepingPrecX), HSP_SWEEP_UD
                       (SweepingPrecUD) or HSP_SWEEP_NX (SweepingPrecNX:
                       partial X-sweeps over ncell groups of slabs coupled
                       through the boundary slabs between them; the groups'
                       sweeps share every stage launch)                       */
  int precision;    /* HSP_FP64: everything complex128.  HSP_MIXED: smoother,
                       slab factors and sweeps complex64; the FGMRES Arnoldi
                       orthogonalisation, its residual, the coarse-grid
                       correction and the solution complex128 (the batched
                       solvers store the preconditioned vectors in complex64,
                       exact for a complex64 preconditioner)                  */
  int restart;      /* FGMRES restart length (sizes the workspace)            */
  int chunk;        /* blocks per chunk of the parallel slab substitutions
                       (1..64); 0 selects about sqrt(n_t) for n_t tangential
                       nodes.  Changes the evaluation order only.             */
  int krylov_fp32;  /* HSP_MIXED only (1 with HSP_FP64: HSP_EINVAL), opt-in
                       (default 0): the batched solvers
                       store the Arnoldi basis in complex64 as well (products
                       and sums still in complex128; a right-hand side whose
                       true residual misses tol gets another restart cycle).
                       Halves the orthogonalisation traffic; the basis is then
                       orthogonal to complex64 accuracy only.                 */
  int ncell;        /* HSP_SWEEP_NX: number of groups N_cell (1..16; 1 is the
                       X-sweep).  Boundary slabs j_cell,m = round(m (J+1) /
                       N_cell), 0 < m < N_cell, group centres j_mid,m =
                       floor((j_cell,m-1 + j_cell,m + 1) / 2) with j_cell,0 =
                       0 and j_cell,N_cell = J + 1; every group needs a slab
                       (HSP_EINVAL otherwise).  Ignored by the other sweeps. */
  int slab_factor;  /* factorization of the 3-D slabs (the paper uses a
                       sparse multifrontal solver, Sec. 5):
                       HSP_SLAB_BLOCK  block tridiagonal along y with dense
                                       (n_l m3)^2 blocks, inverted on the
                                       matrix cores; the substitutions take
                                       one step per y-plane;
                       HSP_SLAB_ND     nested dissection of the (y, z) plane
                                       of the slab (multifrontal; dense fronts
                                       eliminated on the matrix cores); the
                                       substitutions take one step per level
                                       of the dissection and about a third of
                                       the factor bytes at 79^2 planes;
                       HSP_SLAB_AUTO   nested dissection in 3-D.
                       2-D slabs are always block tridiagonal (HSP_SLAB_ND:
                       HSP_EINVAL).                                          */
} hsp_options;

/* Fills *opt with: fine_stencil 5, two_grid 0, w_dd 4, S_dd 0 (= 5 w_dd),
 * nu 3, omega_jac 0.8 (Sec. 6.1, 2-D experiments), sweep X, precision FP64, restart 40,
 * chunk 0 (automatic), krylov_fp32 0, ncell 2, slab_factor HSP_SLAB_AUTO. */
hsp_status hsp_default_options(hsp_options* opt);

/* Bytes of device workspace that hsp_setup needs for this geometry, slab
 * count J and options (depends on sizes only, not on the medium).
 * Errors: HSP_EINVAL for an invalid geometry / J / options (the same checks
 * as hsp_setup except those that need the medium). */
hsp_status hsp_workspace_size(const hsp_grid* grid, int J, const hsp_options* opt,
                              size_t* bytes);

/* Build the preconditioner for one medium and frequency (Sec. 2-4):
 * PML profiles, coarse mesh and coarse optimized-FE coefficients (App. A),
 * slab partition beta_j (outer-PML layers join the first and last cores, the
 * interior layers are split evenly), slab operators with DD-PML and k
 * continuation (Sec. 2.1 "subdomains"), and the LU factorization of all J
 * slabs on the device.
 *   c_dev      wave speed at all (N1-1)*(N2-1) unknown nodes, PML nodes
 *              included, x slowest; read during the call only.
 *   omega      angular frequency (> 0).
 *   J          number of slabs (>= 1); every core must have >= 3 layers.
 *   ws_dev     caller-owned device workspace of at least
 *              hsp_workspace_size bytes, 256-byte aligned; it must stay
 *              valid and untouched until hsp_destroy.
 *   stream     hipStream_t or NULL.
 *   out        receives the handle.
 * Errors: HSP_EINVAL (bad geometry, options, non-positive or non-finite c or
 * omega, cores thinner than 3 layers, DD-PML leaving the domain, odd interior
 * cell count with two_grid), HSP_ENOMEM (workspace too small),
 * HSP_ESINGULAR (a zero or non-finite pivot, or Schur-complement growth
 * beyond the limit of hsp_debug_set), HSP_EDEVICE.  Synchronises
 * the stream (it reads the medium statistics and the pivot status). */
hsp_status hsp_setup(const double* c_dev, double omega, const hsp_grid* grid, int J,
                     const hsp_options* opt, void* ws_dev, size_t ws_bytes, void* stream,
                     hsp_handle* out);

/* Right-hand side of the discrete system (right side of eq. define_pml_fd,
 * FE scaled): b = h^2 f / (alpha_1(x_i) alpha_2(y_k)).  f_dev, b_dev:
 * complex128 vectors of the fine unknowns (may alias). */
hsp_status hsp_rhs(hsp_handle hd, const void* f_dev, void* b_dev, void* stream);

/* y = A x with the fine operator (eq. define_pml_fd times h^2, or the FE
 * 9-point form), complex128.  x_dev and y_dev must not alias. */
hsp_status hsp_apply_operator(hsp_handle hd, const void* x_dev, void* y_dev, void* stream);

/* z = M r: one application of the preconditioner - the X (or UD) sweep of
 * Table 3 on the fine level (two_grid = 0) or the two-grid cycle of Sec. 4
 * with that sweep as coarse solver (two_grid = 1).  complex128 in and out,
 * no aliasing.  M is a fixed linear map. */
hsp_status hsp_apply_precond(hsp_handle hd, const void* r_dev, void* z_dev, void* stream);

/* Solve A u = b for the FE-scaled right-hand side b (see hsp_rhs) with
 * right-preconditioned FGMRES (x0 = 0, restart from options; the paper uses
 * the two-grid cycle as a preconditioner for GMRES, Sec. 4), stopping when
 * ||b - A u||_2 <= tol ||b||_2 (Arnoldi estimate, then checked on the true
 * residual).  conj_transpose = 1 solves A^H u = b instead (A is complex
 * symmetric, so this is conj(A^{-1} conj(b))).  iters and relres (may be
 * NULL) receive the iteration count and the true relative residual.
 * Errors: HSP_ENOCONV when maxit is reached (u holds the last iterate). */
hsp_status hsp_solve(hsp_handle hd, const void* b_dev, void* u_dev, double tol, int maxit,
                     int conj_transpose, int* iters, double* relres, void* stream);

/* Release the handle (host memory only; the caller frees the workspace). */
hsp_status hsp_destroy(hsp_handle hd);

/* Message for the last error on this thread (never NULL). */
const char* hsp_last_error(void);

/* ---- Component entry points, used to check each step against the
 *      reference implementation.  Vectors are complex128. ---------------- */

/* Sizes of the handle: fine unknowns per axis n_fine[2], coarse unknowns
 * n_coarse[2] (zeros without two-grid), J, the largest slab thickness. */
typedef struct hsp_info {
  int n_fine[2];
  int n_coarse[2];
  int J;
  int max_slab_layers;
  int precision;
  int two_grid;
  double pivot_growth;  /* largest growth factor max_t |S_t| / max_t |B_t|
                           of the slab Schur complements (Sec. 5: block LU
                           with pivoting inside each block only)           */
  int dim;              /* 2 or 3                                          */
  int n_fine_z;         /* 3-D: fine unknowns along z (0 in 2-D)            */
  int n_coarse_z;       /* 3-D with two-grid: coarse unknowns along z       */
  int slab_factor;      /* HSP_SLAB_BLOCK or HSP_SLAB_ND (the one in use)   */
} hsp_info;
hsp_status hsp_get_info(hsp_handle hd, hsp_info* info);

/* Debugging knobs (process-wide; they affect later hsp_setup calls), for
 * testing the failure paths of the setup:
 *   HSP_DEBUG_SINGULAR_SLAB  value = slab index j (0-based): the first block
 *                            of slab j is replaced by zero, so hsp_setup
 *                            returns HSP_ESINGULAR; -1 switches it off.
 *   HSP_DEBUG_GROWTH_LIMIT   value > 0 replaces the growth limit of the slab
 *                            factorization (default 0.01 / eps of the factor
 *                            precision: hsp_setup returns HSP_ESINGULAR when
 *                            the Schur complements grow beyond it); <= 0
 *                            restores the default.
 * Errors: HSP_EINVAL for an unknown knob. */
enum { HSP_DEBUG_SINGULAR_SLAB = 0, HSP_DEBUG_GROWTH_LIMIT = 1 };
hsp_status hsp_debug_set(int knob, double value);

/* Partition (host arrays supplied by the caller): beta[0..J] (Sec. 2.2) and
 * the first / last global layer x0[j], x1[j] of slab j = 0..J-1. */
hsp_status hsp_get_partition(hsp_handle hd, int* beta, int* x0, int* x1);

/* y = A_level x for level 0 (fine) or 1 (coarse optimized FE operator,
 * App. A, eq. define_H_FE), complex128, computed in the precision of that
 * level's use inside the preconditioner converted to complex128. */
hsp_status hsp_apply_level_operator(hsp_handle hd, int level, const void* x_dev,
                                    void* y_dev, void* stream);

/* r_c = P^T r_f (restriction, Sec. 4 "Using PML layers in the two-grid
 * method"); e_f += P e_c (prolongation and correction).  complex128. */
hsp_status hsp_restrict(hsp_handle hd, const void* rf_dev, void* rc_dev, void* stream);
hsp_status hsp_prolong_add(hsp_handle hd, const void* ec_dev, void* xf_dev, void* stream);

/* x = S^steps(0; r): omega-Jacobi smoothing on the fine operator from a zero
 * start, x <- x + omega_jac D^{-1} (r - A x).  complex128. */
hsp_status hsp_smooth(hsp_handle hd, const void* r_dev, void* x_dev, int steps, void* stream);

/* u = P_X f (or P_UD f) on the level that carries the slabs (the coarse
 * level with two-grid, the fine level otherwise), Table 3.  complex128. */
hsp_status hsp_sweep(hsp_handle hd, const void* f_dev, void* u_dev, void* stream);

/* x = (A^(j))^{-1} b for slab j (0-based) alone: b and x are complex128
 * arrays over the slab's unknowns, layer-major (layer x0[j] first).  Uses
 * the stored factors. */
hsp_status hsp_slab_solve(hsp_handle hd, int j, const void* b_dev, void* x_dev, void* stream);

/* Adjoint-state gradient of a data misfit with respect to the squared
 * slowness m = 1/c^2 at the fine unknown nodes.  With A u = b, A^H lam = r
 * (r = R^T of the misfit gradient, solved with hsp_solve(conj_transpose=1))
 * and the FE-scaled 5-point operator, whose only m-dependence is the
 * diagonal term -h^2 omega^2 m / (alpha_1 alpha_2) of eq. define_pml_fd:
 *   g_dev[i] += h^2 omega^2 Re( conj(lam_i) u_i / (alpha_1 alpha_2)_i ).
 * u_dev, lam_dev: complex128 fine vectors; g_dev: double fine array,
 * accumulated in place.  Requires fine_stencil = 5 and an explicit c_pml in
 * the grid (with c_pml = mean(c) the PML itself would depend on m).
 * Errors: HSP_EINVAL otherwise. */
hsp_status hsp_gradient_accumulate(hsp_handle hd, const void* u_dev, const void* lam_dev, double* g_dev,
                                   void* stream);

/* ---- Batched right-hand sides.  Many sources (or adjoint sources) of one
 *      medium and frequency share the setup: the slab factors serve every
 *      right-hand side, which is the multi-RHS pipelining of Sec. 5.  A
 *      batch is nrhs contiguous complex128 fine vectors, right-hand side j
 *      at offset j * (N1-1)(N2-1).  These calls need a second caller-owned
 *      device workspace, 256-byte aligned, which holds the per-right-hand-
 *      side vectors, the FGMRES bases and the slab scratch, and may be
 *      reused between calls.  tile selects the number of right-hand sides
 *      per work item of the stage launches (1, 2, 4 or 8; 0 = the tile found
 *      by hsp_tune_batch for this batch size, else a size heuristic); it
 *      changes the evaluation order only. ------------------------------- */

/* Bytes of batch workspace for up to nrhs right-hand sides (>= 1) and FGMRES
 * restart length restart (>= 1). */
hsp_status hsp_batch_workspace_size(hsp_handle hd, int nrhs, int restart, size_t* bytes);

/* z_j = M r_j for j < nrhs (the preconditioner of hsp_apply_precond applied
 * to every column).  r_dev, z_dev: nrhs complex128 fine vectors, no aliasing;
 * nrhs = 0 does nothing.  ws sized for (nrhs, restart >= 1).
 * Errors: HSP_EINVAL (bad tile, null or aliased pointers), HSP_ENOMEM. */
hsp_status hsp_apply_precond_batch(hsp_handle hd, int nrhs, const void* r_dev, void* z_dev, int tile,
                                   void* ws_dev, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * map as hsp_apply_precond_batch (same kernels, same evaluation order for
 * the same tile, so bitwise the same z), with the batch workspace taken from
 * a fixed device array inside the library instead of a caller workspace.
 * Calls no allocating routine.  The array holds 256 MiB per GPU (written to
 * *scratch_bytes if not NULL); it is reserved on every GPU the library runs
 * on until the process ends, and it is shared by all calls on that GPU:
 * calls that overlap on one GPU (other streams or host threads) race and must
 * be serialised by the caller.  Every call clears what must start at zero.
 * Errors: HSP_EINVAL (bad tile, null or aliased vectors), HSP_ENOMEM (the
 * batch needs more than the fixed scratch: hsp_batch_workspace_size(hd,
 * nrhs, 1) must not exceed it), HSP_EDEVICE. */
hsp_status hsp_apply_precond_batch_noalloc(hsp_handle hd, int nrhs, const void* r_dev, void* z_dev, int tile,
                                           size_t* scratch_bytes, void* stream);

/* Autotuner of the batched solvers' evaluation order (the map computed does
 * not depend on it): for every chunk length of the candidate list 16, 20,
 * 24, 28, 34, 40, 48, 64 (those that give distinct chunk counts for the
 * tangential length of the slabs) the problem is set up with that chunk
 * length and one batched preconditioner application of nrhs right-hand
 * sides is timed for every tile (hsp_tune_batch); the fastest (chunk, tile)
 * is returned, and the caller sets its solver up with that chunk (the tile
 * is passed to the batched calls).  2-D only.
 *   ws / bws  device workspaces of at least the sizes
 *             hsp_autotune_workspace_size gives (setup and batch workspaces,
 *             the largest over the candidates); overwritten.
 *   chunk_out, tile_out, ms_out  the choice and its time per application;
 *   table (optional, 3 doubles per candidate chunk: chunk, best tile, ms)
 *   and *ntable (entries written; at most 8).
 * Errors: those of hsp_setup and hsp_tune_batch. */
hsp_status hsp_autotune_workspace_size(const hsp_grid* grid, int J, const hsp_options* opt, int nrhs, int restart,
                                       size_t* ws_bytes, size_t* bws_bytes);
hsp_status hsp_autotune(const double* c_dev, double omega, const hsp_grid* grid, int J, const hsp_options* opt,
                        int nrhs, int restart, void* ws_dev, size_t ws_bytes, void* bws_dev, size_t bws_bytes,
                        int* chunk_out, int* tile_out, double* ms_out, double* table, int* ntable, void* stream);

/* Times one batched preconditioner application for every tile and keeps the
 * fastest for batches of nrhs right-hand sides (used when tile = 0).  Writes
 * into the batch workspace (sized for nrhs, restart).  tile_out and ms_out
 * (may be NULL) receive the tile and its time per application.
 * Synchronises the stream. */
hsp_status hsp_tune_batch(hsp_handle hd, int nrhs, int restart, void* ws_dev, size_t ws_bytes, int* tile_out,
                          double* ms_out, void* stream);

/* Solve A u_j = b_j (or A^H u_j = b_j) for j < nrhs with one right-
 * preconditioned FGMRES process per right-hand side (x0 = 0, restart
 * length restart), all advanced together; each stops at its own test
 * ||b_j - A u_j||_2 <= tol ||b_j||_2 and leaves the batch, so later
 * iterations work on the remaining ones only.  The Arnoldi vectors are
 * orthogonalised by classical Gram-Schmidt with one reorthogonalisation,
 * the reorthogonalisation of each vector being carried out with the
 * projection of the next one (one pass over the basis for both).  With
 * HSP_MIXED the preconditioned vectors are stored in complex64 and the
 * Arnoldi basis, products, Hessenberg matrix, residuals and u_j in
 * complex128; krylov_fp32 = 1 stores the Arnoldi basis in complex64 too.
 * A right-hand side whose true residual misses tol after its estimate met
 * it gets another restart cycle.  b_j = 0 gives u_j = 0 with 0 iterations.
 * iters[nrhs] and relres[nrhs] (host arrays, may be NULL) receive the
 * iteration counts and true relative residuals.  One host synchronisation
 * per iteration.
 * Errors: HSP_EINVAL, HSP_ENOMEM, HSP_ENOCONV (some right-hand side's true
 * residual misses tol at maxit; all u_j hold their last iterates). */
hsp_status hsp_solve_batch(hsp_handle hd, int nrhs, const void* b_dev, void* u_dev, double tol, int maxit,
                           int restart, int conj_transpose, int tile, void* ws_dev, size_t ws_bytes,
                           int* iters, double* relres, void* stream);

/* ---- Groups: the right-hand sides of several problems (media, frequencies,
 *      grid sizes; each set up with its own handle and workspace) solved
 *      together.  The sweep stages of all problems are aligned on the
 *      coarse residual of the sweep (Table 3) and each step of the aligned
 *      schedule is one pair of launches over the work items of every
 *      problem.  All handles must share the precision; a handle may appear
 *      once.  Vectors: b_dev[p], u_dev[p] (or r_dev[p], z_dev[p]) hold
 *      nrhs[p] contiguous complex128 fine vectors of problem p (nrhs[p] = 0
 *      allowed).  Group workspace: caller-owned, 256-byte aligned.
 *      flags: HSP_GROUP_GRAPH captures one preconditioner application in a
 *      HIP graph (re-captured when the set of active right-hand sides
 *      changes) and replays it. ------------------------------------------ */
enum { HSP_GROUP_GRAPH = 1 };

hsp_status hsp_group_workspace_size(int nprob, const hsp_handle* hds, const int* nrhs, int restart, size_t* bytes);

hsp_status hsp_apply_precond_group(int nprob, const hsp_handle* hds, const int* nrhs, const void* const* r_dev,
                                   void* const* z_dev, int tile, int flags, void* ws_dev, size_t ws_bytes,
                                   void* stream);

/* As hsp_solve_batch for every right-hand side of every problem; iters and
 * relres hold sum(nrhs) entries, problem by problem. */
hsp_status hsp_solve_group(int nprob, const hsp_handle* hds, const int* nrhs, const void* const* b_dev,
                           void* const* u_dev, double tol, int maxit, int restart, int conj_transpose, int tile,
                           int flags, void* ws_dev, size_t ws_bytes, int* iters, double* relres, void* stream);

/* ---- Timing (tracing aid).  When enabled, every kernel launch of the
 *      classes below is bracketed by a pair of HIP events on the stream it
 *      is launched on; hsp_profile_read synchronises on the last event and
 *      returns the summed event time, the launch count and the algorithmic
 *      bytes of those launches (what the method must move: factors, the
 *      gathered right-hand side, the scattered solution and transmission
 *      layers for a sweep stage; the vectors and coefficients read and the
 *      vector written for a stencil or transfer), then resets the class. */
enum {
  HSP_PROF_STAGE = 0,     /* fused slab-solve stage kernels (sweeps)        */
  HSP_PROF_SMOOTH = 1,    /* fine-level Jacobi / residual kernels (two-grid) */
  HSP_PROF_COARSE = 2,    /* residual inside the sweep (DD level)           */
  HSP_PROF_TRANSFER = 3,  /* restriction and prolongation                   */
  HSP_PROF_KRYLOV = 4,    /* FGMRES matvec and Gram-Schmidt kernels (the     */
                          /* batched projection and update passes excepted) */
  HSP_PROF_PROJECT = 5,   /* batched FGMRES projection pass (k_bmultidot2)   */
  HSP_PROF_UPDATE = 6,    /* batched FGMRES update pass (k_bdcgs_update)     */
  HSP_PROF_NCLASS = 7
};
hsp_status hsp_profile_enable(hsp_handle hd, int on);
hsp_status hsp_profile_read(hsp_handle hd, int cls, double* total_ms, long long* launches,
                            double* alg_bytes);

#ifdef __cplusplus
}
#endif

#endif /* HSP_H */

/* fsi.h - C ABI of the MI355X block-preconditioned FSI Jacobian solver.
 *
 * The library solves one linearised monolithic ALE fluid-structure system
 *
 *     A_h x = b,   A_h = [ M     C_ms  0    ]
 *                        [ C_sm  S     C_sf ]
 *                        [ C_fm  C_fs  F    ]
 *
 * (Jodlbauer, Langer, Wick, Section 3.4: unknowns ordered mesh motion, solid,
 * fluid) by flexible GMRES, right-preconditioned with the approximate block
 * LDU factorisation of Section 4.1 ("Evaluation of P^{-1} r"): C_sm dropped,
 * fluid Schur complement approximated by F, every inverse replaced by one
 * smoothed-aggregation AMG V-cycle (Sections 4.2-4.4; damped-Jacobi or
 * Chebyshev smoothing per hierarchy, see fsi_precond_opts), or, for the
 * hierarchies so selected, by Chebyshev steps alone.
 *
 * Conventions shared by every call
 *   - Status: every call returns fsi_status.  A negative value is an error;
 *     the context is left unchanged by a failing call and fsi_last_error()
 *     returns a message.  FSI_NOT_CONVERGED (> 0) is a warning: the output is
 *     valid and holds the best iterate.
 *   - Memory: CSR arrays passed to setup calls are HOST memory, read during
 *     the call only (the library copies what it keeps).  Vectors passed to
 *     fsi_solve / fsi_spmv / fsi_apply_precond / fsi_vcycle are DEVICE
 *     pointers (FP64, contiguous) on the context's device, borrowed for the
 *     duration of the call.  The context owns every allocation it makes and
 *     frees it in fsi_destroy.
 *   - Streams: all device work is enqueued on the stream given to fsi_create
 *     (NULL = the default stream).  Calls that return device results do not
 *     synchronise except fsi_solve, which synchronises before filling info.
 *   - Sizes: row pointers are int64, column indices int32 (N < 2^31).
 *   - Threading: a context must not be used from two threads at once.
 *   - Logging: with FSI_LOG set in the environment (to anything but "0") the
 *     library writes one stderr line per setup phase (A_h upload, operators
 *     and SA setup per hierarchy, device upload per hierarchy) and per solve
 *     (iterations, true residual per block, time, bytes per phase).
 */
#ifndef FSI_H
#define FSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FSI_OK = 0,
  FSI_NOT_CONVERGED = 1, /* warning: x holds the best iterate                     */
  FSI_ERR_ARG = -1,      /* NULL pointer, bad size or option                       */
  FSI_ERR_CSR = -2,      /* malformed CSR (row pointers, column range or order)    */
  FSI_ERR_STRUCT = -3,   /* block identity violated (S_uv != -dt*theta*S_uu, ...)  */
  FSI_ERR_HIP = -4,      /* a HIP runtime call failed                              */
  FSI_ERR_OOM = -5,      /* device or host allocation failed                       */
  FSI_ERR_NUMERIC = -6,  /* NaN/Inf input, zero diagonal or pivot, stalled setup   */
  FSI_ERR_STATE = -7     /* call order (e.g. solve before build)                   */
} fsi_status;

typedef struct fsi_ctx fsi_ctx;

/* Host CSR matrix: rowptr[nrows+1] (rowptr[0] = 0, rowptr[nrows] = nnz,
 * non-decreasing), col[nnz] in [0, ncols) strictly increasing within a row,
 * val[nnz] FP64. */
typedef struct {
  int64_t nrows, ncols, nnz;
  const int64_t* rowptr;
  const int32_t* col;
  const double* val;
} fsi_csr;

/* The eight stored blocks of A_h (Section 3.4), in this order. */
enum { FSI_M = 0, FSI_CMS, FSI_CSM, FSI_S, FSI_CSF, FSI_CFM, FSI_CFS, FSI_F, FSI_NBLK };

/* The five AMG hierarchies of the preconditioner:
 *   FSI_H_M   scalar mesh Laplacian L, M = L (x) I_d        (Section 4.2)
 *   FSI_H_SIG solid Schur matrix Sigma_s = S_vv + dt*theta*S_vu (Section 4.3)
 *   FSI_H_MS  solid mass block S_uu                         (Section 4.3)
 *   FSI_H_A   fluid velocity block A_f                      (Section 4.4)
 *   FSI_H_P   pressure Schur approximation -D diag(A_f)^{-1} G (Section 4.4) */
enum { FSI_H_M = 0, FSI_H_SIG, FSI_H_MS, FSI_H_A, FSI_H_P, FSI_NHIER };

/* Block layout.  Dofs inside each block are node-major with the d vector
 * components interleaved.  S is ordered [v_s | u_s] with n_s = 2 n_vs (equal
 * order velocity and displacement, Section 4.3); F is ordered [v_f | p] with
 * n_f = n_vf + n_p (Section 4.4). */
typedef struct {
  int32_t dim;               /* d = 2 or 3                                       */
  int32_t pad;
  int64_t n_m, n_s, n_f;     /* block sizes of A_h                               */
  int64_t n_vs;              /* solid velocity dofs (= solid displacement dofs)  */
  int64_t n_vf;              /* fluid velocity dofs                              */
  double dt_theta;           /* dt * theta of the solid Schur step (Section 4.3) */
  int64_t n_nodes;           /* number of lattice nodes                          */
  const double* coords;      /* n_nodes * dim node coordinates (rigid modes)     */
  const int32_t* dof_node;   /* N = n_m + n_s + n_f: node of every dof           */
  const int32_t* node_ijk;   /* n_nodes * dim lattice indices (the learned
                                smoother's 3^d stencils); may be NULL            */
} fsi_layout;

enum { FSI_P_F64 = 0, FSI_P_F32 = 1, FSI_P_F32_BF16DIAG = 2 };

typedef struct {
  int32_t precision;   /* FSI_P_F64 (default) or FSI_P_F32: precision of the
                          preconditioner's V-cycles and coupling products; the
                          Krylov loop, A_h products and coarsest solves stay FP64.
                          FSI_P_F32_BF16DIAG: FSI_P_F32 with the smoothers'
                          inverse diagonals D^{-1} stored in BF16 (rounded to
                          nearest even through FP32; the setup products A D^{-1}
                          and R (I - omega A D^{-1}) use the same rounded values,
                          so each sweep is the Jacobi or Chebyshev sweep of the
                          hierarchy with that diagonal).  The learned smoother
                          is not available with it.                              */
  int32_t max_coarse;  /* AMG: coarsest level size bound (default 500)          */
  int32_t max_levels;  /* AMG: level bound (default 10)                         */
  int32_t cheb_degree; /* 0 (default): one damped-Jacobi sweep before and after
                          the coarse correction; k in 1..8: k Chebyshev steps for
                          D^{-1} A on [lam/30, lam], lam = 1.1 x the power
                          estimate of its spectral radius, on the hierarchies
                          in cheb_mask                                           */
  double strength0;    /* AMG: strength threshold on the finest level (0.08)    */
  int32_t cheb_mask;   /* bit FSI_H_*: hierarchies with Chebyshev sweeps
                          (default H_MS | H_SIG | H_P; H_A is rejected: its
                          operator is nonsymmetric)                             */
  int32_t poly_mask;   /* bit FSI_H_*: inverses taken as poly_degree Chebyshev
                          steps alone on the finest matrix, no coarse grid
                          (default none; meant for the solid mass matrix M_s,
                          whose D^{-1} M_s has a bounded spectrum), on
                          [lam/poly_ratio, lam]; H_A is rejected               */
  int32_t poly_degree; /* 2..16 (default 3); k - 1 launches per inverse        */
  int32_t schur;       /* pressure Schur approximation S_p = -D W^{-1} G of the
                          fluid step (Section 4.4): FSI_SCHUR_SIMPLE (default),
                          W = diag(A_f); FSI_SCHUR_SIMPLEC, W = the absolute
                          row sums of A_f                                      */
  double poly_ratio;   /* > 1 (default 8)                                       */
  int32_t fluid_inner; /* 0 (default): F^{-1} is the Uzawa-like step alone;
                          k in 1..16: k steps of flexible GMRES on the fluid
                          block F from zero, right-preconditioned by that step
                          (the fluid sub-problem solved by AMG-preconditioned
                          GMRES, Section 4.4), classical Gram-Schmidt with one
                          reorthogonalisation, stopping early only at an exact
                          solve; the outer FGMRES absorbs the nonlinearity.
                          Stores F once more and 2k + 1 fluid vectors        */
  int32_t fluid_inner_pc; /* preconditioner of those steps: FSI_INNER_UZAWA
                          (default; the Uzawa-like step, two A_f V-cycles and
                          one S_p V-cycle) or FSI_INNER_TRIANGULAR (the block
                          upper-triangular step x_p = S_p^{-1} r_p,
                          x_v = A_f^{-1}(r_v - G x_p): one V-cycle of each)  */
  int32_t reuse;       /* 0 (default): run the SA setup.  1: keep the five
                          hierarchies the context holds (those of the previous
                          fsi_build_precond of the same system, or imported by
                          fsi_set_hierarchy) and rebuild only what depends on
                          the other options (precision, smoothers, fluid
                          solve); strength0, max_coarse, max_levels and schur
                          must equal the previous build's.  FSI_ERR_STATE
                          without such a build since fsi_setup_blocks.  After
                          fsi_update_values the kept hierarchies are those of
                          the earlier values                                  */
  int32_t x_approx;    /* the fluid operator inverted in place of the Schur
                          complement X = F - C~_fs S^{-1} C_sf of Section 4.1
                          (C~_fs = C_fs - C_fm M^{-1} C_ms): FSI_X_F (default,
                          the perturbation dropped, as in the paper's
                          algorithm) or FSI_X_BLOCKDIAG (S and M replaced by
                          their node-block diagonals, d x d blocks per field
                          and node: X ~ F - C~ D_S^{-1} C_sf, the
                          block-diagonal approximation the paper cites; the
                          pressure Schur approximation then includes the
                          resulting pressure block)                           */
  int32_t uzawa_inner; /* 0 (default): each inverse of the Uzawa-like fluid
                          step is one V-cycle.  k in 1..16: Section 4.4 as
                          written, each occurring inverse (A_f^{-1} twice,
                          S_p^{-1} once) approximated by k steps of GMRES on
                          A_f or on S_p from zero, right-preconditioned by its
                          V-cycle (classical Gram-Schmidt with one
                          reorthogonalisation, stopping early only at an exact
                          solve).  Not combined with fluid_inner > 0.  Stores
                          A_f and S_p once more                               */
  int32_t order;       /* block order of the LDU factorisation (Section 4.1
                          remarks that it decides the preconditioner), one of
                          FSI_ORDER_*: FSI_ORDER_MSF (default; mesh, solid,
                          fluid: the paper's algorithm).  Another order
                          (a, b, c), its pivot and multiplier perturbations
                          dropped as the paper drops its own (C_sm dropped,
                          S, M, F as pivots), is a block symmetric
                          Gauss-Seidel sweep in that order: forward
                          x_i = A_ii^{-1}(r_i - sum_{j before i} A_ij x_j),
                          then x_b, x_a -= A_ii^{-1} sum_{j after i} A_ij x_j
                          (e.g. FSI_ORDER_FSM: x_f = F^{-1} r_f,
                          x_s = S^{-1}(r_s - C_sf x_f),
                          x_m = M^{-1}(r_m - C_ms x_s),
                          x_f -= F^{-1}(C_fm x_m + C_fs x_s)).  Each stores
                          one more fluid vector; the orders with the fluid in
                          the middle store C_fm and C_fs once more          */
} fsi_precond_opts;

enum { FSI_INNER_UZAWA = 0, FSI_INNER_TRIANGULAR = 1 };
enum { FSI_X_F = 0, FSI_X_BLOCKDIAG = 1 };
enum {
  FSI_ORDER_MSF = 0, /* mesh, solid, fluid: the paper's order */
  FSI_ORDER_FSM = 1, /* the reverse order */
  FSI_ORDER_MFS = 2,
  FSI_ORDER_SMF = 3,
  FSI_ORDER_SFM = 4,
  FSI_ORDER_FMS = 5
};

enum { FSI_SCHUR_SIMPLE = 0, FSI_SCHUR_SIMPLEC = 1 };

typedef struct {
  double tol;       /* stop when ||b - A_h x||_2 <= tol ||b||_2 (default 1e-8)  */
  int32_t restart;  /* GMRES restart length m (default 50, at most 200)         */
  int32_t maxit;    /* total iteration bound (default 2000)                     */
  int32_t timing;   /* 1: time every Arnoldi step's phases with HIP events    */
  int32_t pad;
} fsi_solve_opts;

typedef struct {
  int32_t iters, restarts, converged, pad;
  double true_rel_resid;   /* recomputed FP64 ||b - A_h x|| / ||b||             */
  double t_total_ms;       /* wall time of the solve, stream-synchronised        */
  /* with opts.timing: summed device time of each phase over the timed Arnoldi
   * steps (n_timed of them): P^{-1} v, the A_h product, Gram-Schmidt */
  double t_precond_ms, t_spmv_ms, t_gs_ms;
  int32_t n_timed;
  int32_t mlp_fallbacks;   /* learned pre-smoothing sweeps replaced by Jacobi     */
  double resid_block[3];   /* ||(b - A_h x)_B|| / ||b|| of the final FP64 true
                              residual restricted to B = mesh, solid, fluid      */
  /* bytes the solve moved as the library stores its operands (values, column
   * lists and row pointers once per product, every vector read or written
   * once): all A_h products (the Arnoldi steps and the true residuals), all
   * applications of P^{-1} (Section 4.1's algorithm with its sub-inverses),
   * and the Krylov vector work (Gram-Schmidt passes and normalisations, the
   * norms of b and of the residuals, the solution update); launched-ahead
   * Arnoldi steps that the stopping test then discarded are included */
  double bytes_spmv, bytes_precond, bytes_gs;
} fsi_solve_info;

/* Defaults for the option structs (tol 1e-8, m 50, maxit 2000, no timing;
 * AMG as above). */
void fsi_default_precond_opts(fsi_precond_opts* o);
void fsi_default_solve_opts(fsi_solve_opts* o);

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t, or NULL for the default stream). */
fsi_status fsi_create(fsi_ctx** ctx, int device, void* hip_stream);
fsi_status fsi_destroy(fsi_ctx* ctx);
/* Message of the last failing call on ctx ("" if none); valid until the next
 * call on ctx.  With ctx == NULL: the last fsi_create failure. */
const char* fsi_last_error(const fsi_ctx* ctx);

/* Copy the eight blocks of A_h (host CSR, Section 3.4) and the layout into the
 * context and validate them: CSR well-formedness, block shapes against the
 * layout, S_uv = -dt_theta S_uu within 1e-12 relative (Section 4.3),
 * M = L (x) I_d (frozen Jacobian-scaled mesh Laplacian), empty pressure block
 * of F.  `mem` must be 0 (host arrays).  Replaces any earlier system and
 * invalidates the preconditioner. */
fsi_status fsi_setup_blocks(fsi_ctx* ctx, const fsi_layout* layout, const fsi_csr blk[FSI_NBLK],
                            int mem);

/* New values for the eight blocks of the system in the context, with the
 * same sparsity patterns (equal row pointers and column indices, checked) and
 * the same structural identities (checked as by fsi_setup_blocks): the device
 * copy of A_h is rewritten in place, in its stored layout.  The preconditioner
 * (if built) is kept as it was built from the earlier values, so fsi_solve
 * then runs FGMRES on the new A_h with the earlier P^{-1}: the reuse of a
 * quasi-Newton step (the scheme of Section 6 reassembles the Jacobian only
 * when the last Newton step cut the residual's max-norm by less than a factor
 * of ten; a caller can keep the preconditioner by the same test).
 * fsi_build_precond rebuilds it from the new values; with `reuse` it keeps
 * the SA hierarchies of the earlier values and takes everything else from the
 * new ones.  On error nothing changes. */
fsi_status fsi_update_values(fsi_ctx* ctx, const fsi_csr blk[FSI_NBLK]);

/* Build the preconditioner of Section 4: Sigma_s, the pressure Schur
 * approximation and the five SA-AMG hierarchies (host setup, then upload).
 * opts may be NULL (defaults). */
fsi_status fsi_build_precond(fsi_ctx* ctx, const fsi_precond_opts* opts);

/* Solve A_h x = b by FGMRES(m), right-preconditioned by the block LDU
 * algorithm, FP64 Arnoldi (classical Gram-Schmidt with reorthogonalisation),
 * FP64 Givens least squares, acceptance on the recomputed true residual.
 * b, x: device FP64 vectors of length N; x holds the initial guess on entry
 * and the solution on return.  opts/info may be NULL. */
fsi_status fsi_solve(fsi_ctx* ctx, const double* b, double* x, const fsi_solve_opts* opts,
                     fsi_solve_info* info);

/* y = A_h x (all eight blocks, C_sm included).  Device vectors of length N. */
fsi_status fsi_spmv(fsi_ctx* ctx, const double* x, double* y);

/* Bytes one y = A_h x moves as the library stores A_h (Section 3.4's block
 * matrix): values, column indices and row (or row-group) pointers once, x
 * once and y written.  The fluid-velocity rows are stored in groups of d
 * rows sharing one column list, so this is below the plain CSR figure
 * 12 nnz + 8 (N + 1) + 16 N.  Used to report achieved bandwidth.
 * FSI_ERR_STATE before fsi_setup_blocks. */
fsi_status fsi_spmv_bytes(fsi_ctx* ctx, double* bytes);

/* z = P^{-1} r, the block LDU algorithm of Section 4.1 with the AMG
 * sub-inverses.  Device vectors of length N. */
fsi_status fsi_apply_precond(fsi_ctx* ctx, const double* r, double* z);

/* x = one V(1,1) cycle of hierarchy `which` applied to b.  Length is the
 * finest level size (for FSI_H_M: n_m, the cycle acting on each of the d
 * interleaved components with the scalar L).  Device vectors. */
fsi_status fsi_vcycle(fsi_ctx* ctx, int which, const double* b, double* x);

/* Replace hierarchy `which` by caller-provided levels (host CSR): A[0..nlev-1]
 * level matrices, P[0..nlev-2] prolongators, R[0..nlev-2] restrictions,
 * omega[0..nlev-2] Jacobi weights.  The coarsest A[nlev-1] is inverted by the
 * library.  Requires a built preconditioner; A[0] must have the size of the
 * hierarchy's finest level. */
fsi_status fsi_set_hierarchy(fsi_ctx* ctx, int which, int nlev, const fsi_csr* A, const fsi_csr* P,
                             const fsi_csr* R, const double* omega);

/* Sizes of hierarchy `which`: *nlev levels; n[l], nnz[l] of each level matrix
 * (arrays of at least 16 entries), omega[l] (0 on the coarsest level). */
fsi_status fsi_hierarchy_info(fsi_ctx* ctx, int which, int32_t* nlev, int64_t* n, int64_t* nnz,
                              double* omega);

/* Bytes one z = P^{-1} r (fsi_apply_precond, one Arnoldi step's
 * preconditioner) moves as the library stores its operands: the eleven
 * sub-inverse applications of Section 4.1's algorithm as executed (each as
 * fsi_vcycle_bytes counts it, or the inner GMRES steps of the fluid inverse
 * with their products and vector passes), the coupling products with their
 * vectors, the vector updates, and in the FP32 precisions the casts of r and
 * z.  FSI_ERR_STATE before fsi_build_precond. */
fsi_status fsi_precond_bytes(fsi_ctx* ctx, double* bytes);

/* Bytes one V(1,1) cycle of hierarchy `which` moves as executed: per level
 * the down-sweep matrices (A D^{-1}, Q = R (I - omega A D^{-1})), the
 * up-sweep matrices (P, A P), the diagonal and the level vectors, plus the
 * dense coarsest inverse.  Used to report achieved bandwidth. */
fsi_status fsi_vcycle_bytes(fsi_ctx* ctx, int which, double* bytes);

/* Copy level `level` of hierarchy `which` to host buffers: what = 0 the level
 * matrix A_l, 1 the prolongator P_l.  Pass NULL buffers to query only the
 * sizes (*nrows, *ncols, *nnz). */
fsi_status fsi_get_level(fsi_ctx* ctx, int which, int level, int what, int64_t* nrows,
                         int64_t* ncols, int64_t* nnz, int64_t* rowptr, int32_t* col, double* val);

/* Aggregate id of every node of level `level` (< nlev-1) of hierarchy `which`
 * (host int32 buffer of n_l / block_l entries; *count receives that number). */
fsi_status fsi_get_aggregates(fsi_ctx* ctx, int which, int level, int32_t* agg, int64_t* count);

/* ---- learned smoother ------------------------------------------------------
 * A per-node MLP may replace the first damped-Jacobi sweep on the finest level
 * of FSI_H_M (mesh motion) and FSI_H_SIG (solid Schur matrix).  For node i,
 * z_i = (D^{-1} b) at the 3^d lattice nodes around i (d components each, 0 for
 * absent neighbours, offsets in lexicographic order of (di, dj[, dk]) in
 * {-1,0,1}^d), K = 3^d d inputs; delta_i = W3^T relu(W2^T relu(W1^T z_i)),
 * W1: K x 64, W2: 64 x 64, W3: 64 x d, row-major FP32 at the ABI, stored and
 * applied in BF16 with FP32 accumulation (matrix cores).  If the network's
 * correction x gives ||b - A x|| > ||b|| the Jacobi sweep is used instead
 * (counted in fsi_solve_info.mlp_fallbacks); after 8 consecutive such cycles
 * the network is not tried again until the next fsi_solve, new weights or
 * training (those cycles count as fallbacks too).  Requires layout.node_ijk.
 * `which` is FSI_H_M or FSI_H_SIG. */
/* Training losses.  FSI_MLP_LOSS_L2: (1/n) sum_i w_i ||delta_i - e_i||^2
 * against the exact corrections e = A^{-1} b (w_i: node's diagonal relative
 * to the mean).  FSI_MLP_LOSS_ENERGY: the A-norm error left after delta and an
 * exact coarse-grid correction, L = ||(I - P A_1^{-1} R A)(e - delta)||_A^2 - e.b,
 * evaluated as -delta.b - delta.r - rc.c with r = b - A delta, rc = R r,
 * c = A_1^{-1} rc; gradient -2 (r - A P c) (A taken as symmetric, R = P^T).
 * Each recorded residual is scaled to ||b||_{D^{-1}} = 1 first. */
enum { FSI_MLP_LOSS_L2 = 0, FSI_MLP_LOSS_ENERGY = 1 };

typedef struct {
  int32_t steps;        /* Adam steps (default 400)                               */
  int32_t batch;        /* samples (nodes) per step (default 16384)               */
  double lr;            /* Adam step size (default 1e-3)                          */
  double exact_tol;     /* L2 loss: relative residual of the exact corrections    */
  int32_t exact_maxit;  /* L2 loss: V-cycle iterations allowed for them (300)     */
  uint32_t seed;        /* sample shuffling                                       */
  int32_t loss;         /* FSI_MLP_LOSS_* (default ENERGY)                        */
  int32_t coarse_cycles;/* energy loss: V-cycles for A_1^{-1} when level 1 is not
                           the coarsest (default 4; exact dense solve otherwise)  */
} fsi_mlp_train_opts;

typedef struct {
  int32_t vectors[2];   /* recorded residuals used (H_M, H_SIG)                   */
  int64_t samples[2];   /* node samples                                           */
  double loss_first[2], loss_last[2];  /* mean loss before / after training      */
} fsi_mlp_train_info;

void fsi_default_mlp_train_opts(fsi_mlp_train_opts* o);
/* Set the network weights (host FP32, shapes above); resets the optimiser
 * state; does not enable the network. */
fsi_status fsi_mlp_set_weights(fsi_ctx* ctx, int which, const float* W1, const float* W2, const float* W3);
/* Current (FP32 master) weights into host buffers of the shapes above. */
fsi_status fsi_mlp_get_weights(fsi_ctx* ctx, int which, float* W1, float* W2, float* W3);
/* Use (1) or stop using (0) the network in the V-cycles. */
fsi_status fsi_mlp_enable(fsi_ctx* ctx, int which, int enable);
/* x = network correction for the residual b of hierarchy `which`'s finest
 * level (device FP64 vectors of that level's size). */
fsi_status fsi_mlp_forward(fsi_ctx* ctx, int which, const double* b, double* x);
/* The same correction for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no allocation and no synchronisation.  In the FP32 precisions
 * b and x are staged through a library-owned FP32 array of 2 x 4,194,304
 * entries (32 MiB per GPU, held until the process ends) instead of buffers
 * allocated per call; FSI_ERR_ARG when the level has more than 4,194,304
 * entries.  Every call on one GPU uses that GPU's one array: calls that
 * overlap on one GPU (different streams or threads) race.  b, x as in
 * fsi_mlp_forward; the result is the same. */
fsi_status fsi_mlp_forward_noalloc(fsi_ctx* ctx, int which, const double* b, double* x);
/* One pass of the training kernels over m samples (host FP32: Z m x K, E m x d,
 * w m): loss = (1/m) sum w ||delta - e||^2 and its gradients G1, G2, G3 (host,
 * shapes of W1, W2, W3). */
fsi_status fsi_mlp_loss_grad(fsi_ctx* ctx, int which, int64_t m, const float* Z, const float* E, const float* w,
                             float* G1, float* G2, float* G3, double* loss);
/* Energy loss (FSI_MLP_LOSS_ENERGY, as is: b not rescaled) of the network's
 * correction for one residual b (device FP64, level-0 size of `which`) and its
 * gradients (host, shapes of W1, W2, W3); A_1^{-1} as in the training. */
fsi_status fsi_mlp_energy_grad(fsi_ctx* ctx, int which, const double* b, int coarse_cycles, float* G1, float* G2,
                               float* G3, double* loss);
/* Record the finest-level inputs of the FSI_H_M and FSI_H_SIG V-cycles during
 * the following solves (every `every`-th cycle, at most max_vectors each);
 * max_vectors = 0 stops recording and drops the records. */
fsi_status fsi_mlp_collect(fsi_ctx* ctx, int max_vectors, int every);
/* Train both networks on the recorded residuals: exact corrections by
 * V-cycle iteration to opts.exact_tol, then Adam on the node samples (on the
 * device); enables the trained networks.  Needs weights set first (the
 * initial weights are an input).  opts/info may be NULL. */
fsi_status fsi_mlp_train(fsi_ctx* ctx, const fsi_mlp_train_opts* opts, fsi_mlp_train_info* info);

/* ------------------------------------------------------------------------
 * Finite-element assembly and the quasi-Newton loop.
 *
 * Section 3: the discrete residual R(U) = A(U)(Phi) - F(Phi) of the monolithic
 * ALE-FSI problem (the sum of the variational equations, equation fsi:all,
 * one step of the one-step-theta scheme of Section 3.2) on the structured
 * channel of Q2 velocity / displacement and Q1 pressure quads (d = 2) or hexes
 * (d = 3), every integral by the tensor 3-point Gauss rule, the outflow term
 * on the face x_0 = extent[0]; and its Jacobian A'(U), the matrix of the
 * Newton step (Algorithm newton of Section 3.3).  The unknowns are numbered as
 * the system of fsi_setup_blocks (mesh | solid v, u | fluid v | p); a state is
 * the given node fields plus an offset dU on the free dofs (constrained dofs
 * hold the given values).  The advecting velocity w of the convective term,
 * v_old, u_old and the displacement u_fz whose det(I + grad u_fz) scales the
 * mesh stiffness are given fields (with newton_mesh the stiffness uses the
 * current J instead).  Mesh-equation test functions vanish on nodes of solid
 * cells (the interface), velocity test functions on Dirichlet nodes.
 * With theta < 1 the convection, viscous stress, outflow correction and solid
 * stress carry dt theta at the new level and dt (1 - theta) at the previous
 * one (v_old, u_old; v_old advecting itself), the fluid mass term uses
 * theta J + (1 - theta) J_old and the kinematics dt (theta v + (1 - theta)
 * v_old); pressure, mesh velocity, incompressibility and mesh motion stay
 * implicit (theta = 1/2: Crank-Nicolson, 1/2 + dt: its shifted variant).
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t dim;                 /* 2 or 3: the system's d                                   */
  int32_t cells[3];            /* cells per axis (1..65535, at most 2^31 - 1 in all;
                                  unused axes ignored)                                    */
  double extent[3];            /* channel lengths                                          */
  int32_t solid_lo[3];         /* solid cells: solid_lo[a] <= C[a] < solid_hi[a], all a    */
  int32_t solid_hi[3];
  double rho_f, nu_f, rho_s, mu_s, lambda_s;  /* fluid density, viscosity; solid density, Lame */
  double dt, theta;            /* theta in (0, 1]; dt * theta must equal the layout's       */
  int32_t newton_mesh;         /* 1: 1/J of the mesh equation from the current state       */
  int32_t pad;
  int64_t n_nodes;             /* prod_a (2 cells[a] + 1): the Q2 lattice, row-major,
                                  axis 0 slowest                                           */
  /* host arrays of n_nodes entries: first velocity dof, first displacement dof
   * (components follow) and pressure dof of each node, -1 where none (Dirichlet
   * node, or no such field there); every free dof must appear exactly once */
  const int64_t* vdof;
  const int64_t* udof;
  const int64_t* pdof;
  /* host node fields, d values per node (component-interleaved), p: one */
  const double* v;
  const double* u;
  const double* p;
  const double* v_old;
  const double* u_old;
  const double* w;
  const double* u_fz;
} fsi_fe_mesh;

#define FSI_NEWTON_MAX 64
enum {
  FSI_NEWTON_PC_REBUILD = 0, /* on reassembly: a new preconditioner (new SA hierarchies)   */
  FSI_NEWTON_PC_REUSE = 1,   /* on reassembly: new preconditioner, SA hierarchies kept      */
  FSI_NEWTON_PC_KEEP = 2     /* the preconditioner of the last fsi_build_precond throughout */
};

typedef struct {
  double rtol;              /* stop once ||r_k||_inf < rtol ||r_0||_inf (1e-6, Section 6)   */
  double reassemble_ratio;  /* reassemble when ||r_k||_inf > ratio ||r_{k-1}||_inf (0.1)     */
  int32_t max_steps;        /* Newton steps, at most FSI_NEWTON_MAX (25)                     */
  int32_t precond;          /* FSI_NEWTON_PC_* (REBUILD)                                     */
  double lin_tol;           /* FGMRES relative residual per step (1e-3, Section 6)          */
  int32_t restart, maxit;   /* FGMRES(restart), at most maxit iterations per step (50, 2000) */
} fsi_newton_opts;

typedef struct {
  int32_t converged, steps, reassemblies, lin_iters_total;
  double resid[FSI_NEWTON_MAX + 1];      /* ||r_k||_inf, k = 0 .. steps                     */
  int32_t reassembled[FSI_NEWTON_MAX];   /* step k assembled A'(U_k)                         */
  int32_t lin_iters[FSI_NEWTON_MAX];     /* FGMRES iterations of step k                      */
  double t_assemble_ms, t_precond_ms, t_solve_ms, t_total_ms;
} fsi_newton_info;

void fsi_default_newton_opts(fsi_newton_opts* o);

/* Upload the finite-element description of the system in the context (after
 * fsi_setup_blocks; a new system drops it).  Checks the sizes (FSI_ERR_ARG
 * before any array is read), the dof maps against N and the fields for
 * NaN/Inf.  Host arrays; copied. */
fsi_status fsi_fe_setup(fsi_ctx* ctx, const fsi_fe_mesh* mesh);

/* R = R(U) of Section 3 at U = given fields + dU.  dU: device, length N, or
 * NULL (dU = 0); R: device, length N.  FSI_ERR_NUMERIC when J <= 0 at a
 * quadrature point of a fluid cell or a value is not finite. */
fsi_status fsi_fe_residual(fsi_ctx* ctx, const double* dU, double* R);

/* A'(U) assembled into the context's A_h in place (its stored layout; the
 * sparsity pattern of fsi_setup_blocks must hold every cell matrix entry,
 * else FSI_ERR_STRUCT): fsi_spmv and fsi_solve use it at once.  With
 * host_blocks the host copies of the eight blocks take the new values too
 * (checked as by fsi_setup_blocks), so that fsi_build_precond builds from
 * them; else the preconditioner's blocks keep their values.  dU as above.
 * On error (J <= 0, a non-finite value, an entry outside the pattern, a block
 * identity violated) A_h and the blocks keep their previous values; the call
 * holds a device copy of A_h's values (its stored bytes) while it runs.  The
 * context keeps, from the first call on, a device buffer of the integrand
 * values and derivatives at the quadrature points of one parity class of
 * cells (d = 3: 650 doubles per point, 36 points per cell; 3.1 GB for
 * 128 x 32 x 32 cells). */
fsi_status fsi_fe_jacobian(fsi_ctx* ctx, const double* dU, int host_blocks);

/* Algorithm newton with Section 6's quasi-Newton scheme: r_k = R(U_k) on the
 * device; stop once ||r_k||_inf < rtol ||r_0||_inf; at k = 0, and whenever
 * ||r_k||_inf > ratio ||r_{k-1}||_inf, assemble A'(U_k) (and, unless
 * FSI_NEWTON_PC_KEEP, rebuild the preconditioner with the options of the last
 * fsi_build_precond, or the defaults); solve A' delta = r_k by FGMRES to
 * lin_tol; U_{k+1} = U_k - delta.  dU: device, length N: the initial offset
 * on entry, the last iterate's on return (also on an error, which ends the
 * loop at the step that failed; A_h then holds the last assembled Jacobian).
 * FSI_NOT_CONVERGED after max_steps steps.  opts/info may be NULL. */
fsi_status fsi_newton(fsi_ctx* ctx, const fsi_newton_opts* opts, double* dU, fsi_newton_info* info);

/* End a time step (Section 3.2): the state U = fields + dU (dU: device,
 * length N) becomes the fields of the next step and its previous level
 * (v_old, u_old), the advecting velocity w and the mesh-stiffness
 * displacement u_fz; constrained dofs keep their values. */
fsi_status fsi_fe_advance(fsi_ctx* ctx, const double* dU);

/* One time step: fsi_newton from dU = 0, then, once it converged,
 * fsi_fe_advance with its iterate (not on FSI_NOT_CONVERGED: the fields are
 * then unchanged).  The system's pattern and dt * theta carry over; the
 * preconditioner follows opts.precond.  opts/info may be NULL. */
fsi_status fsi_time_step(fsi_ctx* ctx, const fsi_newton_opts* opts, fsi_newton_info* info);

/* Copy the current state fields to host arrays: v and u (n_nodes * d,
 * component-interleaved), p (n_nodes). */
fsi_status fsi_fe_get_fields(fsi_ctx* ctx, double* v, double* u, double* p);

#ifdef __cplusplus
}
#endif

#endif /* FSI_H */

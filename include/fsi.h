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
 * fluid Schur complement approximated by F, every inverse replaced by
 * smoothed-aggregation AMG V(1,1) cycles (Sections 4.2-4.4).
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
} fsi_layout;

enum { FSI_P_F64 = 0, FSI_P_F32 = 1 };

typedef struct {
  int32_t precision;   /* FSI_P_F64 (default) or FSI_P_F32: precision of the
                          preconditioner's V-cycles and coupling products; the
                          Krylov loop, A_h products and coarsest solves stay FP64 */
  int32_t max_coarse;  /* AMG: coarsest level size bound (default 500)          */
  int32_t max_levels;  /* AMG: level bound (default 10)                         */
  int32_t pad;
  double strength0;    /* AMG: strength threshold on the finest level (0.08)    */
} fsi_precond_opts;

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
  int32_t n_timed, pad2;
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

#ifdef __cplusplus
}
#endif

#endif /* FSI_H */

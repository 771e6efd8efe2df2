/*
 * libfem — HEX8 finite-element hot path on one AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Every function returns an int status (FEM_OK = 0, negative codes
 * below); no C++ exception or abort crosses this boundary.  The message of the
 * last failure on the calling thread is available from fem_last_error().
 *
 * Problem solved (paper, Sec. 2.1): find u with u = u_D on the Dirichlet set and
 *     C(u; theta) = R_int(u; theta) - F_ext = 0            (Eq. (weak), discretised)
 * where R_int[(a,i)] = sum_e int_{Omega_e} f(grad u_h) : grad phi_(a,i) over HEX8
 * elements with 2x2x2 Gauss quadrature, and f is one of
 *   FEM_POISSON         f = m * grad u                         (scalar, ndpn = 1)
 *   FEM_LINEAR_ELASTIC  f = lambda tr(eps) I + 2 mu eps, E = m  (Sec. 2.3, Eq. (linear_elasticity))
 *   FEM_NEO_HOOKEAN     f = P = dW/dF, G = m, kappa = bulk_ratio * m  (Sec. 2.3, Eq. (neo-hookean))
 *   FEM_J2_PLASTIC      f = sigma^k of perfect J2 plasticity, E = m, nu, yield_stress (Sec. 2.3,
 *                       plasticity paragraph): sigma_trial = sigma^{k-1} + lambda tr(d eps) I
 *                       + 2 mu d eps with d eps = sym(grad u^k) - eps^{k-1}, radial return to
 *                       the von Mises surface; (eps, sigma) at every Gauss point are the
 *                       handle's history, committed after each converged load step
 * with a per-element modulus m(theta_e): theta_e itself (FEM_THETA_IDENTITY) or the
 * SIMP map emin + theta_e^p (e0 - emin) (FEM_THETA_SIMP, Sec. 3.2, Eq. (top_weak)).
 *
 * Conventions shared with callers:
 *   - HEX8 local node order 0:(0,0,0) 1:(1,0,0) 2:(1,1,0) 3:(0,1,0) 4:(0,0,1)
 *     5:(1,0,1) 6:(1,1,1) 7:(0,1,1) in the reference cube;
 *   - dof = ndpn * node + component (node-major, interleaved components);
 *   - the global matrix is CSR over ALL dofs (Dirichlet dofs included), row i
 *     holding every dof j that shares an element with i, columns ascending;
 *   - Dirichlet dofs are eliminated symmetrically: residual entry 0, matrix row
 *     and column replaced by the unit vector (so K stays symmetric for every
 *     model here and the adjoint solve uses the same matrix).
 *
 * Memory ownership: all arrays passed to calls other than fem_build_pattern are
 * DEVICE pointers owned by the caller (e.g. torch tensors on the same GPU) and
 * must stay valid until the call's work on `stream` has finished.  The handle
 * owns its own device copies of the mesh and the sparsity structure (allocated
 * in fem_build_pattern, released by fem_destroy): node graph, row pointers, the
 * element-to-block maps and small reduction buffers, about 1.4 GB for a
 * 1M-element mesh.  They are built on the host from the mesh, live as long as the
 * handle, and are not exposed as caller buffers (a caller-allocated form would add
 * a size query and a fill call per array for no gain in reuse).  Only three setup
 * calls allocate device memory: fem_build_pattern, fem_amg_setup and
 * fem_filter_setup.  Every other call allocates nothing: scratch memory for
 * assembly and solves is a caller-provided device `workspace` of
 * fem_workspace_bytes(), 256-byte aligned (FEM_EINVAL otherwise; torch
 * allocations are).  `stream` is a hipStream_t passed as void* (NULL = the
 * default stream).
 */
#ifndef FEM_H
#define FEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status codes */
#define FEM_OK 0
#define FEM_EINVAL (-1)     /* bad argument (null pointer, size, enum value, mesh index) */
#define FEM_ERANGE (-2)     /* pattern too large for 32-bit column indices / slots */
#define FEM_EHIP (-3)       /* HIP runtime error */
#define FEM_EMESH (-4)      /* det(dx/dxi) <= 0 at a Gauss point */
#define FEM_EINVERTED (-5)  /* det(F) <= 0 at a Gauss point (neo-Hookean) */
#define FEM_ENAN (-6)       /* NaN or Inf in a residual, tangent or Krylov scalar */
#define FEM_EBREAKDOWN (-7) /* Krylov breakdown (rho or omega or p.Ap vanished) */
#define FEM_EMAXITER (-8)   /* Newton or Krylov iteration limit reached */
#define FEM_EDIVERGED (-9)  /* Newton residual grew beyond the divergence limit */
#define FEM_ENOMEM (-10)    /* device allocation failed or workspace too small */

/* ---------------------------------------------------------------- enumerations */
enum { FEM_POISSON = 0, FEM_LINEAR_ELASTIC = 1, FEM_NEO_HOOKEAN = 2, FEM_J2_PLASTIC = 3 };
enum { FEM_THETA_IDENTITY = 0, FEM_THETA_SIMP = 1 };
enum { FEM_F32 = 0, FEM_F64 = 1 };
/* Storage of tangent values.
 * FEM_LAYOUT_CSR: CSR over all dofs (row_ptr / col_idx of fem_pattern_export).
 * FEM_LAYOUT_SYM_BLOCK: the matrix is symmetric (all models here, with the symmetric
 *   Dirichlet elimination), so only the ndpn x ndpn blocks (n, m) with m >= n are
 *   stored: in CSR order of the node graph (node n ascending, then neighbour m
 *   ascending), each block row-major; block (m, n) with m > n is read as the
 *   transpose of block (n, m).  About half the values of the CSR layout. */
enum { FEM_LAYOUT_CSR = 0, FEM_LAYOUT_SYM_BLOCK = 1 };
/* FEM_PREC_FP64: tangent, SpMV and Krylov vectors in FP64.
 * FEM_PREC_MIXED: tangent values, SpMV and Krylov vectors in FP32 with FP32
 * accumulation; the Newton/refinement residual, the adjoint refinement residual
 * and all Krylov inner products stay FP64.
 * FEM_PREC_MIXED_V64: the tangent is assembled and stored in FP32 (the SpMV streams
 * FP32 values, the bulk of its bytes), while the Krylov vectors, the SpMV's products
 * and sums and every vector update are FP64: the Krylov method runs in FP64 on the
 * fixed FP32 operator.  Residuals and refinement as in FEM_PREC_MIXED.  Jacobi and
 * node-block Jacobi only (FEM_EINVAL with FEM_PRECOND_AMG). */
enum { FEM_PREC_FP64 = 0, FEM_PREC_MIXED = 1, FEM_PREC_MIXED_V64 = 2 };
enum { FEM_KRYLOV_CG = 0, FEM_KRYLOV_BICGSTAB = 1 };
/* Krylov preconditioner.  FEM_PRECOND_JACOBI: the inverse diagonal of the tangent
 * (the paper's Jacobi preconditioner, Sec. 5).  FEM_PRECOND_BLOCK_JACOBI: the
 * inverse of each node's ndpn x ndpn diagonal block (equal to Jacobi when ndpn = 1).
 * FEM_PRECOND_AMG (CG only): a two-level aggregation preconditioner, one symmetric
 * V-cycle per application -- Chebyshev smoothing of the Jacobi-scaled tangent, a
 * Galerkin coarse operator on a rigid-body-mode coarse space of node aggregates (6
 * columns per aggregate; 1, the constant, when ndpn = 1) and Chebyshev steps on it.
 * The paper names the Jacobi-preconditioned solver as the bottleneck (Sec. 5, item 2);
 * this is the stronger preconditioner built on that remark.  fem_amg_setup builds the
 * aggregates and prolongator once per handle (solves with FEM_PRECOND_AMG refuse to run
 * before it); the handle keeps them with the coarse operator of the latest tangent; see
 * fem_amg_setup / fem_amg_export / fem_amg_apply below.  With FEM_PRECOND_JACOBI,
 * BiCGSTAB runs on K D^{-1} (the scaling is folded into the solver's copy of the
 * tangent), CG applies D^{-1} to its residual. */
enum { FEM_PRECOND_JACOBI = 0, FEM_PRECOND_BLOCK_JACOBI = 1, FEM_PRECOND_AMG = 2 };

typedef struct fem_handle fem_handle;

/* Mesh, material and loads.  HOST pointers; copied by fem_build_pattern. */
typedef struct {
    int64_t n_nodes;
    int64_t n_elems;
    int32_t ndpn;              /* 1 for FEM_POISSON, 3 otherwise */
    int32_t model;             /* FEM_POISSON / FEM_LINEAR_ELASTIC / FEM_NEO_HOOKEAN / FEM_J2_PLASTIC */
    int32_t pmap;              /* FEM_THETA_IDENTITY / FEM_THETA_SIMP */
    int32_t reserved;
    double nu;                 /* Poisson ratio (linear elasticity, J2 plasticity) */
    double bulk_ratio;         /* kappa / G (neo-Hookean) */
    double simp_p, simp_emin, simp_e0;
    const double *coords;      /* [n_nodes * 3] */
    const int32_t *conn;       /* [n_elems * 8], HEX8 local order above */
    const uint8_t *dirichlet_mask; /* [n_nodes * ndpn], 1 = Dirichlet dof; may be NULL */
    const double *f_nodal;     /* [n_nodes * ndpn] nodal point loads; may be NULL */
    const double *source_nodal;/* [n_nodes * ndpn] body source b given at the nodes and
                                  interpolated with the shape functions; may be NULL */
    int64_t n_traction_faces;
    const int32_t *traction_faces; /* [n_traction_faces * 2]: (element, local face);
                                      local face = 2*axis + side, the face where the
                                      reference coordinate xi_axis = -1 (side 0) or +1 */
    const double *traction;        /* [n_traction_faces * ndpn] constant traction per face */
    double yield_stress;           /* sigma_yield of FEM_J2_PLASTIC (> 0); ignored otherwise */
} fem_mesh_desc;

typedef struct {
    int32_t precision;      /* FEM_PREC_FP64, FEM_PREC_MIXED or FEM_PREC_MIXED_V64 */
    int32_t krylov;         /* FEM_KRYLOV_CG (SPD tangents) or FEM_KRYLOV_BICGSTAB */
    int32_t n_load_steps;   /* >= 1 */
    int32_t newton_max_it;  /* per load step */
    double newton_rtol;     /* relative Newton tolerance (see fem_newton_solve) */
    double newton_atol;
    double krylov_rtol;     /* inner tolerance of each correction solve (recursive residual) */
    int32_t krylov_max_it;
    int32_t check_every;    /* Krylov convergence is read back every this many iterations */
    double adjoint_rtol;    /* adjoint stops when ||b - K lambda|| <= adjoint_rtol ||b|| (FP64) */
    int32_t adjoint_max_refine; /* outer refinement sweeps of the adjoint solve (mixed) */
    int32_t profile_spmv;   /* 1: time the SpMV launches of the middle Krylov iteration of every
                               check_every block with HIP events (a sample of the solve) */
    int32_t newton_fixed_its; /* > 0: run exactly this many Newton iterations per load step
                                 (the first one being the lifted step), without a convergence test */
    int32_t precond;        /* FEM_PRECOND_JACOBI, FEM_PRECOND_BLOCK_JACOBI or FEM_PRECOND_AMG (CG only) */
    int32_t amg_smooth_degree; /* FEM_PRECOND_AMG: Chebyshev steps of each fine smoothing (1..64) */
    int32_t amg_coarse_degree; /* FEM_PRECOND_AMG: Chebyshev steps on the coarse operator (1..64) */
    int32_t max_bisections; /* load-step recovery of fem_newton_solve (0 = off, at most 30): when a
                               load step fails with FEM_EBREAKDOWN, FEM_EMAXITER, FEM_EDIVERGED,
                               FEM_EINVERTED or FEM_ENAN, u is restored to the start of the step
                               and the remaining increment is halved, at most this many times per
                               load step */
    int32_t reserved_opts;
    double refine_rtol;     /* FEM_PREC_MIXED Newton corrections (0 = off): the correction K du = b is
                               solved to ||b - K du|| <= krylov_rtol ||b|| measured in FP64 with the
                               matrix-free tangent, by FP32 Krylov sweeps that each reduce the FP64
                               residual by at most this factor (each restarts from the FP64 residual;
                               at most adjoint_max_refine sweeps).  Off: one FP32 solve to krylov_rtol on
                               its recursive residual.  The mixed adjoint's sweeps likewise ask for at
                               most this reduction each (instead of krylov_rtol). */
} fem_solve_opts;

#define FEM_MAX_HIST 64
typedef struct {
    int32_t newton_its;       /* total over load steps */
    int32_t load_steps;
    int32_t krylov_its_total;
    int32_t n_hist;           /* entries used in krylov_its[] / residual_hist[] */
    double initial_residual;  /* ||r_free|| at the start of the last load step */
    double final_residual;    /* ||r_free|| (Newton) or ||b - K lambda|| (adjoint) at exit */
    double ms_residual, ms_assemble, ms_krylov, ms_vjp, ms_total;
    int32_t spmv_calls;       /* SpMV launches timed (sampled) when profile_spmv = 1 */
    int32_t krylov_unconverged; /* correction solves that stopped before reaching krylov_rtol */
    double spmv_ms_total;     /* their summed event durations */
    int32_t krylov_its[FEM_MAX_HIST];     /* Krylov iterations of each correction solve */
    double residual_hist[FEM_MAX_HIST];   /* ||r_free|| before each correction */
    double krylov_relres[FEM_MAX_HIST];   /* final recursive ||r||/||b|| of each correction solve */
    int32_t bisections;       /* load-step halvings taken by the recovery (opts.max_bisections) */
    int32_t reserved_stats;
    double iter_ms[FEM_MAX_HIST];         /* fem_newton_solve: wall time of each Newton iteration, from
                                             its right-hand side to the residual norm after the update
                                             (the first iteration of a load step includes the lifting) */
} fem_solve_stats;

/* Message of the last failure on this thread ("" if none).  Never NULL. */
const char *fem_last_error(void);

/* Fills *opts with defaults: FP64, BiCGSTAB, 1 load step, newton_max_it 30,
 * newton_rtol 1e-10, atol 0, krylov_rtol 1e-6, krylov_max_it 20000,
 * check_every 16, adjoint_rtol 1e-10, adjoint_max_refine 20, profile off,
 * newton_fixed_its 0, Jacobi, amg degrees 1 / 16, max_bisections 0. */
int fem_default_opts(fem_solve_opts *opts);

/* Builds the handle: uploads the mesh, computes the external load vector
 * (nodal + traction + interpolated source, Sec. 2.1 Eq. (weak)), and builds the
 * CSR pattern of the dof graph and the element-to-CSR slot map that implements
 * "Add K_e to K" of Sec. 2.2 Alg. 1 without atomics.  Synchronous; uses the
 * current HIP device.  Writes the number of dofs N = n_nodes*ndpn and of stored
 * entries.  Errors: FEM_EINVAL (bad sizes, node index out of range, model/ndpn
 * mismatch), FEM_ERANGE (nnz >= 2^31), FEM_ENOMEM, FEM_EHIP. */
int fem_build_pattern(const fem_mesh_desc *desc, fem_handle **out, int64_t *n_dofs, int64_t *nnz);

/* The host half of fem_build_pattern, with no device and no handle: checks the mesh
 * the same way, builds the node graph and the CSR pattern of the dof graph (Sec. 2.2,
 * Alg. 1: the entries "Add K_e to K" touches) and the external load vector (Eq. (weak)
 * with the nodal, traction and interpolated source terms).  Writes N and nnz; then,
 * into caller HOST buffers that may each be NULL, row_ptr [N+1] int64, col_idx [nnz]
 * int32 (ascending per row) and f_ext [N] FP64 (Dirichlet entries included).  A call
 * with NULL arrays returns the sizes.  Synchronous; errors as fem_build_pattern. */
int fem_pattern_host(const fem_mesh_desc *desc, int64_t *n_dofs, int64_t *nnz, int64_t *row_ptr, int32_t *col_idx,
                     double *f_ext);

/* Releases the handle and its device memory (NULL is accepted). */
void fem_destroy(fem_handle *h);

/* Copies the pattern into caller DEVICE buffers (any may be NULL):
 *   row_ptr [N+1] int64, col_idx [nnz] int32 (ascending per row),
 *   slot_map [n_elems * Nd * Nd] int32 with Nd = 8*ndpn: slot_map[(e*Nd + p)*Nd + q] is the
 *     CSR position of (dof(e,p), dof(e,q)), p = ndpn*a + i;
 *   diag_slot [N] int64: CSR position of (d, d);
 *   transpose_perm [nnz] int32: CSR position of the transposed entry.
 * Asynchronous on `stream`. */
int fem_pattern_export(fem_handle *h, int64_t *row_ptr, int32_t *col_idx, int32_t *slot_map, int64_t *diag_slot,
                       int32_t *transpose_perm, void *stream);

/* Number of stored tangent values in `layout` (nnz for FEM_LAYOUT_CSR). */
int fem_values_count(fem_handle *h, int32_t layout, int64_t *count);

/* Copies the external load vector F_ext [N] (FP64) into a caller device buffer. */
int fem_load_vector(fem_handle *h, double *f_ext, void *stream);

/* Workspace size in bytes for fem_newton_solve / fem_adjoint_vjp with `opts`, or,
 * with opts == NULL, for fem_assemble with FP64 values (the largest assembly case). */
int fem_workspace_bytes(fem_handle *h, const fem_solve_opts *opts, size_t *bytes);

/* Residual and tangent at u (Sec. 2.2: R_e and K_e = dr_e/dU_e, Alg. 1 assembly):
 *   residual [N] FP64 (may be NULL): r = R_int(u; theta) - F_ext, Dirichlet entries 0;
 *   values [fem_values_count(layout)] (may be NULL): K(u) in `values_layout`,
 *   FEM_F32 or FEM_F64, with the symmetric Dirichlet elimination.
 *   u [N] FP64, theta [n_elems] FP64; workspace of fem_workspace_bytes(h, NULL).
 * Asynchronous on `stream`: the call checks its arguments (errors returned at once),
 * clears the handle's status word and enqueues the kernels.  Conditions the kernels
 * detect (det J <= 0, det F <= 0, NaN) raise bits in that word; fem_check reports
 * them after the work has finished. */
int fem_assemble(fem_handle *h, const double *u, const double *theta, double *residual, void *values,
                 int32_t values_dtype, int32_t values_layout, void *workspace, size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): the residual of fem_assemble
 * (residual [N] FP64 = R_int(u; theta) - F_ext, Dirichlet entries 0; u [N] FP64,
 * theta [n_elems] FP64, device pointers owned by the caller) computed with the
 * library's static device scratch array instead of a workspace, so the call allocates
 * nothing.  Limit: n_elems * 8 * ndpn doubles of element terms must fit the 64 MiB
 * array (up to 349,525 elements with 3 dofs per node, 1,048,576 with 1); larger meshes
 * get FEM_ENOMEM before any work is enqueued.  Each GPU holds its own copy of the
 * array until the process ends; every call on one GPU shares it, so calls that
 * overlap on one GPU (different streams or threads) race.  Enqueue-only like
 * fem_assemble: fem_check reports what the kernels found. */
int fem_residual_noalloc(fem_handle *h, const double *u, const double *theta, double *residual, void *stream);

/* Waits for `stream` and reports what the kernels of the enqueue-only calls
 * (fem_assemble, fem_residual_noalloc) found since they cleared the status word: FEM_EMESH (det J <= 0 at a
 * Gauss point), FEM_EINVERTED (det F <= 0), FEM_ENAN, or FEM_OK.  A reported condition
 * is cleared.  Blocks. */
int fem_check(fem_handle *h, void *stream);

/* The matrix-vector product inside the Jacobi-preconditioned Krylov solver (Sec. 5,
 * item 2, which names that solver as the cost of the forward problem; the transposed
 * form is the operator of the adjoint equation, Sec. 3, Eq. (adjoint_PDE)):
 * y = alpha * op(K) x + beta * y with op(K) = K or K^T (transpose != 0; for
 * FEM_LAYOUT_SYM_BLOCK both are K).  values [fem_values_count(layout)] in `layout`
 * (as written by fem_assemble), x and y [N], all of `dtype` (FEM_F32 or FEM_F64) on the
 * device; products and sums in that dtype.  With beta == 0, y is not read.  x and y
 * must not overlap.  Asynchronous on `stream`; FEM_EINVAL for bad enums or NULL
 * pointers. */
int fem_spmv(fem_handle *h, const void *values, int32_t dtype, int32_t layout, int32_t transpose, const void *x,
             void *y, double alpha, double beta, void *stream);

/* Tangent-vector product y = K(u) v, matrix-free in FP64, with the same Dirichlet
 * elimination as the assembled matrix (y_d = v_d on Dirichlet dofs, Dirichlet
 * entries of v ignored elsewhere).  Asynchronous. */
int fem_apply_tangent(fem_handle *h, const double *u, const double *theta, const double *v, double *y,
                      void *workspace, size_t workspace_bytes, void *stream);

/* Newton's method (Sec. 2.1, Eq. (newton)) with incremental loading: load step k of
 * n scales F_ext by k/n and moves the Dirichlet values from those found in u on
 * entry to `dirichlet_values` [N] (read on Dirichlet dofs only).  The first iteration
 * of a step carries the Dirichlet increment D through the tangent at the previous
 * state (du_D = D, K_ff du_f = -r_f - K_fD D); every later iteration evaluates the
 * FP64 residual, assembles K(u), solves K du = -r with the Jacobi-preconditioned
 * Krylov method of opts (Sec. 5, item 2) and updates u.  A step stops when
 * ||r_free|| <= max(newton_rtol * max(||first right-hand side||, ||F_k||), atol).  In
 * FEM_PREC_MIXED the correction solve runs in FP32 (in FEM_PREC_MIXED_V64 with FP64
 * vectors on the FP32 tangent) and the FP64 residual of the next iteration performs
 * the refinement.  u [N] FP64 is in/out.  Blocks; returns
 * FEM_EMAXITER / FEM_EDIVERGED / FEM_EBREAKDOWN / FEM_EMESH / FEM_EINVERTED / FEM_ENAN
 * on failure (u then holds the last iterate).  `stats` may be NULL. */
int fem_newton_solve(fem_handle *h, double *u, const double *theta, const double *dirichlet_values,
                     const fem_solve_opts *opts, fem_solve_stats *stats, void *workspace, size_t workspace_bytes,
                     void *stream);

/* Adjoint gradient (Sec. 3, Eq. (adjoint_PDE) and Eq. (adjoint_chain_simp)):
 * solves (dC/du)^T lambda = dJdu with Dirichlet entries of the right-hand side set
 * to 0, then writes vjp_theta[e] = -lambda^T dC/dtheta_e [n_elems] FP64.  u is the
 * converged state.  lambda_out [N] may be NULL.  In FEM_PREC_MIXED the transposed
 * solve runs in FP32 (FEM_PREC_MIXED_V64: FP64 vectors on the FP32 tangent) inside
 * FP64 iterative refinement whose residual uses the matrix-free FP64 tangent.
 * Blocks. */
int fem_adjoint_vjp(fem_handle *h, const double *u, const double *theta, const double *dJdu, double *vjp_theta,
                    double *lambda_out, const fem_solve_opts *opts, fem_solve_stats *stats, void *workspace,
                    size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------------
 * Path-dependent state of FEM_J2_PLASTIC.  The history holds, for every element e and
 * Gauss point q, 12 FP64 values at [(e*8 + q)*12]: the total strain of the last
 * committed load step, then its stress, each symmetric tensor as (xx, yy, zz, yz, xz,
 * xy).  It starts at zero and fem_newton_solve commits it after every converged load
 * step.  fem_adjoint_vjp / fem_param_vjp are not defined for this law (FEM_EINVAL).
 * ---------------------------------------------------------------------------- */

/* Copies the history between the handle and a caller device buffer buf of
 * n_elems * 96 doubles: into_handle = 0 reads it out (history -> buf), 1 replaces it
 * (buf -> history; e.g. to restart a path or to reset it with zeros).  Asynchronous
 * on stream.  FEM_EINVAL for other laws. */
int fem_history_copy(fem_handle *h, double *buf, int32_t into_handle, void *stream);

/* Volume average of the committed stress, sum_e sum_q detJ sigma_q / sum_e sum_q detJ,
 * as (xx, yy, zz, yz, xz, xy) to the host array out[6] (the quantity the paper plots
 * for its loading-unloading path; zeros for an empty mesh).  Blocks.  FEM_EINVAL for
 * other laws. */
int fem_average_stress(fem_handle *h, double *out, void *stream);

/* ------------------------------------------------------------------------------
 * Two-level preconditioner (FEM_PRECOND_AMG): its parts, for inspection and tests.
 * ---------------------------------------------------------------------------- */

/* Setup of the two-level preconditioner (a setup call, like fem_build_pattern): builds
 * the node aggregates and the rigid-body-mode prolongator on the host and allocates
 * the handle's device arrays for them, the coarse operator and its vectors.  Once per
 * handle (later calls return at once); needed before any call with FEM_PRECOND_AMG
 * (FEM_EINVAL otherwise).  Synchronous. */
int fem_amg_setup(fem_handle *h);

/* The number of aggregates and of coarse ncoarse x ncoarse blocks (ncoarse = 6, or 1
 * when ndpn = 1), to the host.  FEM_EINVAL before fem_amg_setup. */
int fem_amg_sizes(fem_handle *h, int64_t *n_aggregates, int64_t *n_coarse_blocks);

/* Copies to caller DEVICE buffers (any may be NULL): the aggregate of every node
 * agg [n_nodes] int32; the prolongator P [n_nodes * ndpn * ncoarse] FP64, row-major
 * ndpn x ncoarse per node (rows of Dirichlet dofs and dropped columns are zero); the
 * coarse block pattern coarse_ptr [n_aggregates + 1] int64 and coarse_col
 * [n_coarse_blocks] int32 (aggregates ascending per row).  Synchronous. */
int fem_amg_export(fem_handle *h, int32_t *agg, double *P, int64_t *coarse_ptr, int32_t *coarse_col);

/* Assembles the tangent at (u, theta) in opts->precision, builds the coarse operator
 * and the Chebyshev intervals, and applies the preconditioner once: z = M r (r, z
 * [N] FP64 device, distinct).  lmax_out (host, may be NULL) receives the fine and
 * coarse largest-eigenvalue bounds; coarse_values (device, may be NULL) receives the
 * coarse operator, FP64 [n_coarse_blocks * ncoarse^2] block-major row-major.  Uses the
 * solve workspace of fem_workspace_bytes(opts).  Synchronous. */
int fem_amg_apply(fem_handle *h, const double *u, const double *theta, const double *r, double *z,
                  const fem_solve_opts *opts, double *lmax_out, double *coarse_values, void *workspace,
                  size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------------
 * SIMP compliance optimisation (Sec. 3.2): the pieces around the gradient.  The
 * loop is: solve, compliance C = F_ext . u, dC/dtheta by the adjoint (lambda = u
 * for this self-adjoint objective) through fem_param_vjp, the sensitivity filter,
 * and one MMA step (Svanberg 1987) under the material-fraction constraint.
 * ---------------------------------------------------------------------------- */

/* Per-element parameter VJP for a given adjoint state (no solve):
 * vjp_theta[e] = -lambda^T dC/dtheta_e (Sec. 3, Eq. (adjoint_chain_simp)); entries
 * of lambda on Dirichlet dofs are ignored.  u, lambda [N]; theta, vjp_theta
 * [n_elems]; FP64 device pointers.  Asynchronous on `stream`. */
int fem_param_vjp(fem_handle *h, const double *u, const double *theta, const double *lambda, double *vjp_theta,
                  void *stream);

/* Element volumes v_e = sum_q det J_q (2x2x2 Gauss, weights 1) [n_elems] FP64 into
 * a caller device buffer; with normalized != 0 the fractions v_e / sum_f v_f (the
 * gradient of the material fraction).  Blocks when normalized, else asynchronous. */
int fem_element_volumes(fem_handle *h, double *volumes, int32_t normalized, void *stream);

/* Builds the convolution filter of radius rmin > 0 over the element centroids (mean
 * of the 8 node coordinates): weights H_ef = max(0, rmin - |c_e - c_f|).  The filter
 * lives in the handle (a later call replaces it).  Synchronous.  FEM_EINVAL for
 * rmin <= 0. */
int fem_filter_setup(fem_handle *h, double rmin);

/* FEM_FILTER_DENSITY:     out_e = sum_f H_ef x_f / sum_f H_ef
 * FEM_FILTER_SENSITIVITY: out_e = sum_f H_ef theta_f x_f / (max(1e-3, theta_e) sum_f H_ef)
 * (the sensitivity filter that blurs dC/dtheta against checkerboards).  x, out
 * [n_elems] FP64 device (distinct buffers); theta is read only by the sensitivity
 * filter.  FEM_EINVAL when fem_filter_setup was not called.  Asynchronous. */
enum { FEM_FILTER_DENSITY = 0, FEM_FILTER_SENSITIVITY = 1 };
int fem_filter_apply(fem_handle *h, int32_t mode, const double *theta, const double *x, double *out, void *stream);

/* Scratch bytes of fem_dot and fem_mma_update for vectors of length n. */
size_t fem_vector_workspace_bytes(int64_t n);

/* Deterministic FP64 dot product sum_i a_i b_i of two device vectors of length n on
 * the current device (fixed blocking, fixed summation order); the result goes to
 * the host pointer `result`.  Blocks. */
int fem_dot(const double *a, const double *b, int64_t n, double *result, void *workspace, size_t workspace_bytes,
            void *stream);

/* Method of moving asymptotes (Svanberg 1987), one constraint, box [xmin, xmax]:
 * asymptotes at asy_init * box for the first two iterations, then moved by
 * asy_decr (oscillating coordinate) or asy_incr (monotone) and kept between 0.01
 * and 10 box widths from x; move limits albefa of the distance to the asymptote and
 * `move` * box; convex approximations with the 0.001 / 1.001 split and raa0 / box
 * regularisation; the dual in the multiplier solved by doubling then
 * `bisect_iters` bisection steps.  When the approximated constraint cannot be met
 * inside the move limits (the doubling reaches 2^200), the step takes that
 * multiplier, i.e. the point of the move box that minimises the approximation. */
typedef struct {
    double xmin, xmax, move, asy_init, asy_decr, asy_incr, albefa, raa0;
    int32_t bisect_iters;
    int32_t reserved;
} fem_mma_opts;
int fem_mma_default_opts(fem_mma_opts *opts);

/* One MMA iteration for min f0 s.t. f1 <= 0: x, xold1, xold2 (iterates k, k-1, k-2),
 * df0, df1 (gradients at x) [n] FP64 device; f1 the constraint value at x (host);
 * low, upp [n] device in/out (asymptotes; read only from iteration 2 on); xnew [n]
 * device out; *lambda_out (host, may be NULL) the constraint multiplier.  `iter` is
 * the 0-based iteration count.  Current device; blocks. */
int fem_mma_update(int64_t n, int32_t iter, const double *x, const double *xold1, const double *xold2,
                   const double *df0, double f1, const double *df1, double *low, double *upp, double *xnew,
                   double *lambda_out, const fem_mma_opts *opts, void *workspace, size_t workspace_bytes,
                   void *stream);

/* ------------------------------------------------------------------------------
 * Full-field inference (Sec. 3.1): the source of a Poisson problem as the parameter.
 * F(theta) = M theta with M the consistent mass of the nodal source; the adjoint of
 * Eq. (full_field_inverse) gives dJ/dtheta = M lambda.
 * ---------------------------------------------------------------------------- */

/* y = M x: the load of the nodal field x [N] (values at the nodes, ndpn components,
 * interpolated with the shape functions and integrated by the 2x2x2 Gauss rule, the
 * body-source term of Eq. (weak)), on every dof including Dirichlet dofs.  x, y [N]
 * FP64 device, distinct.  Uses the assembly workspace (fem_workspace_bytes with
 * opts NULL).  Asynchronous. */
int fem_mass_apply(fem_handle *h, const double *x, double *y, void *workspace, size_t workspace_bytes, void *stream);

/* Replaces the external load vector F_ext [N] (FP64 device) used by the residual and
 * the Newton tolerance of later calls (entries on Dirichlet dofs are ignored).
 * Blocks. */
int fem_set_load(fem_handle *h, const double *f_ext, void *stream);

/* y = a x + b y on n FP64 device entries (with b == 0, y is not read).  Current
 * device; asynchronous. */
int fem_axpby(int64_t n, double a, const double *x, double b, double *y, void *stream);

/* Observation misfit J = sum_k (u[idx_k] - obs_k)^2 (Eq. (full_field_inverse)) to the
 * host pointer J, and dJdu [n] (device) = 0 except 2 (u[idx_k] - obs_k) at idx_k.
 * idx [n_obs] int64 device (distinct, < n), obs [n_obs] and u [n] FP64 device.
 * Workspace fem_vector_workspace_bytes(n_obs).  Current device; blocks. */
int fem_obs_misfit(int64_t n, int64_t n_obs, const int64_t *idx, const double *obs, const double *u, double *dJdu,
                   double *J, void *workspace, size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FEM_H */

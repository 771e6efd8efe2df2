// Internal declarations of libfem (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "fem.h"

namespace fem {

// Error carried from deep inside the library up to the ABI wrapper.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

// Runs f, translating a thrown Error (or any other exception) into its status code
// and the thread's last-error message; FEM_OK clears the message.  Every ABI entry
// point runs its body through this.
int run_guarded(const std::function<void()> &f);

#define FEM_HIP(call)                                                                                        \
    do {                                                                                                     \
        hipError_t e_ = (call);                                                                              \
        if (e_ != hipSuccess)                                                                                \
            throw ::fem::Error(e_ == hipErrorOutOfMemory ? FEM_ENOMEM : FEM_EHIP,                            \
                               std::string(#call " failed: ") + hipGetErrorString(e_));                      \
    } while (0)

// Blocks of the grid-stride reduction kernels (one FP64 partial per block).
constexpr int kRedGrid = 1024;

// Bits of the device status word raised by kernels.
enum : int { ST_MESH = 1, ST_INVERTED = 2, ST_NAN = 4, ST_BREAKDOWN = 8 };

// Storage of tangent values: full CSR, or only the blocks (n, m) with m >= n.
enum Layout { LAYOUT_CSR = 0, LAYOUT_SYM = 1 };

// Material description passed by value to kernels.
struct Material {
    int model, pmap;
    double nu, bulk_ratio, simp_p, simp_emin, simp_e0;
    double yield_stress;  // J2 plasticity
};

// Device-side Krylov scalars (FP64), one instance per solve in the workspace.
struct KrylovScalars {
    double rho, rho_old, alpha, omega, beta;
    double bnorm2, rnorm2, tol2;
    double rh2;      // |rhat|^2 (BiCGSTAB shadow residual)
    double rmin2;    // smallest |r|^2 reached so far
    int its, converged, breakdown;
    int restart_at;  // BiCGSTAB restarts (rhat = p = r) at the iteration with this index
    // CG: rho of iteration k lives in rho_pp[k & 1], so a kernel that publishes the
    // next rho never overwrites the value its other blocks are still reading
    double rho_pp[2];
    // BiCGSTAB (fused form): the scalars of iteration k in slot k & 1 -- alpha and omega,
    // |rhat|^2 and the smallest |r|^2 so far -- written by one kernel of iteration k and
    // read by kernels of iteration k + 1, never by blocks of the kernel writing them
    double alpha_pp[2], omega_pp[2], rh2_pp[2], rmin2_pp[2];
};
constexpr size_t kScalarsHostBytes = sizeof(KrylovScalars);

// Sparsity structure on the device.  A "block" is the ndpn x ndpn coupling of a
// node pair (n, m); blocks are numbered in CSR order of the node graph.
struct Graph {
    int64_t Nn = 0, Ne = 0, N = 0, nnz = 0, nnzb = 0;
    int nd = 1;
    int64_t *node_ptr = nullptr;  // [Nn+1] first block of node n
    int32_t *node_nb = nullptr;   // [nnzb] neighbour node of each block, ascending per node
    int16_t *node_dnb = nullptr;  // [nnzb] node_nb - row node, when every offset fits 16 bits (else null)
    uint8_t *nb_bits = nullptr;   // [nnzb] Dirichlet bits of the neighbour's dofs (bit c: dof c)
    int32_t *blk_row = nullptr;   // [nnzb] owning node of each block
    int32_t *mirror = nullptr;    // [nnzb] block (m, n) for block (n, m)
    int32_t *bdiag = nullptr;     // [Nn] block (n, n)
    int64_t *blk_ptr = nullptr;   // [nnzb+1] contributions of element-pair blocks
    int32_t *blk_src = nullptr;   // [64*Ne] contribution kpos[e*8+a]*8 + b, element ascending
    int64_t *ne_ptr = nullptr;    // [Nn+1] node -> (element, local node) incidence
    int32_t *kpos = nullptr;      // [8*Ne] slot of (e, a) in node-major incidence order
                                  //        (node n owns slots ne_ptr[n] .. ne_ptr[n+1]-1,
                                  //        element ascending)
    int32_t *bslot = nullptr;     // [Ne*64] block of local pair (a, b) of element e
    uint8_t *tgt = nullptr;       // [Ne*64] for slot k and column block b: the block's position
                                  //         in the row node's neighbour list (max_deg <= 255)
    int max_deg = 0;              // largest node degree of the node graph
    int64_t *row_ptr = nullptr;   // [N+1] scalar CSR row starts
    // Symmetric block layout: only blocks (n, m) with m >= n are stored, block-major
    // (nd x nd, row-major), in CSR order of the node graph.
    int64_t nnzb_up = 0;
    int64_t *up_base = nullptr;   // [Nn+1] first stored block of node n
    int32_t *lo_val = nullptr;    // [nnzb] for a block (n, m) with m < n: stored block (m, n)
};

// Problem mesh on the device.
struct DeviceMesh {
    double *coords = nullptr;  // [Nn*3]
    int32_t *conn = nullptr;   // [Ne*8]
    uint8_t *mask = nullptr;   // [N]
    double *fext = nullptr;    // [N]
    double fext_norm = 0.0;
    std::vector<uint8_t> host_mask;
};

// Convolution filter over element centroids (CSR over elements).
struct Filter {
    int64_t *ptr = nullptr;   // [Ne+1]
    int32_t *idx = nullptr;   // neighbour elements, ascending
    double *w = nullptr;      // weights rmin - distance
    double *wsum = nullptr;   // [Ne] row sums
    int64_t nnz = 0;
    bool ready = false;
    std::vector<void *> allocations;
};

// Two-level aggregation preconditioner (amg.hip).  Built once per handle (first use);
// the coarse operator and the Chebyshev bounds are refreshed for every tangent.
struct Amg {
    int64_t na = 0, nbc = 0;       // aggregates, coarse blocks
    int nc = 0;                    // coarse dofs per aggregate (6, or 1 when ndpn = 1)
    int32_t *agg = nullptr;        // [Nn] aggregate of each node
    int64_t *agg_ptr = nullptr;    // [na+1] members of each aggregate in agg_nodes
    int32_t *agg_nodes = nullptr;  // [Nn] nodes ascending per aggregate
    double *P64 = nullptr;         // [Nn*nd*nc] prolongator, row-major nd x nc per node
    float *P32 = nullptr;          // the same in FP32
    int64_t *cptr = nullptr;       // [na+1] coarse block rows
    int32_t *ccol = nullptr;       // [nbc] column aggregate of each coarse block
    int32_t *crow = nullptr;       // [nbc] row aggregate of each coarse block
    int64_t *cdiag = nullptr;      // [na] diagonal block of each row
    int64_t *cbp = nullptr;        // [nbc+1] fine blocks feeding each coarse block in cbk
    int32_t *cbk = nullptr;        // [nnzb] fine block indices, ascending per coarse block
    uint8_t *dropped = nullptr;    // [na] bit k set: coarse column k of the aggregate is empty
    void *cvals = nullptr;         // [nbc*nc*nc] coarse operator in the solve precision
    void *cdinv = nullptr;         // [na*nc] its inverse diagonal
    void *fine_tmp = nullptr;      // 3 fine vectors [N] (SpMV output, Chebyshev residual, direction)
    void *coarse_tmp = nullptr;    // 5 coarse vectors [na*nc]
    double *red = nullptr;         // reduction partials
    double *host_red = nullptr;    // pinned read-back of the partials
    double lmax = 0.0, lmax_c = 0.0;
    int precision = -1;            // precision of the current coarse operator
    int sdeg = 2, cdeg = 16;       // Chebyshev degrees of the smoother and of the coarse solve
};

}  // namespace fem

struct fem_handle {
    int device = 0;
    fem::Material mat{};
    fem::Graph g;
    fem::DeviceMesh m;
    int *status = nullptr;                    // device status word (ST_* bits)
    int *host_status = nullptr;               // pinned read-back slots
    double *host_scalar = nullptr;
    fem::KrylovScalars *host_kry = nullptr;
    std::vector<hipEvent_t> events;           // SpMV timing events (profile_spmv)
    int spmv_group = 16;                      // SpMV tuning knob (nodes in flight per lane group)
    int num_cus = 256;                        // compute units of the device
    std::vector<void *> allocations;          // device allocations owned by the handle
    fem::Filter filter;                       // fem_filter_setup (owns its allocations)
    double *red_partials = nullptr;           // [kRedGrid] reduction partials (fem_element_volumes, fem_set_load)
    double *hist = nullptr;                   // J2 history [Ne*8*12] (eps, sigma per Gauss point)
    double *hist_partials = nullptr;          // per-block partials of fem_average_stress (J2)
    fem::Amg *amg = nullptr;                  // two-level preconditioner (fem_amg_setup)
};

namespace fem {

// ------------------------------------------------------------------ setup (host)
// The sparsity structure built on the host (host_graph, no device work); build_graph
// uploads it into the handle's Graph (same array meanings).
struct HostGraph {
    int64_t Nn = 0, Ne = 0, N = 0, nnz = 0, nnzb = 0, nnzb_up = 0;
    int nd = 1, max_deg = 0;
    std::vector<int64_t> ne_ptr, node_ptr, blk_ptr, row_ptr, up_base;
    std::vector<int32_t> kpos, node_nb, blk_row, mirror, bdiag, bslot, blk_src, lo_val;
    std::vector<int16_t> dnb;  // empty when some neighbour offset needs more than 16 bits
    std::vector<uint8_t> tgt, nb_bits;
};
HostGraph host_graph(const fem_mesh_desc *d, const std::vector<uint8_t> &mask);
std::vector<double> host_load_vector(const fem_mesh_desc *d);
void build_graph(fem_handle *h, const fem_mesh_desc *d);
void build_load_vector(fem_handle *h, const fem_mesh_desc *d);
void *dev_alloc(fem_handle *h, size_t bytes);

// ------------------------------------------------------------------ element kernels
// r_scratch: [Ne*8*nd] FP64 per (element, local node, component).
void launch_residual(const fem_handle *h, const double *u, const double *theta, double load_factor,
                     double *r_scratch, double *r_out, hipStream_t s);
void launch_apply_tangent(const fem_handle *h, const double *u, const double *theta, const double *v,
                          double *y_scratch, double *y_out, hipStream_t s);
// ke_scratch: [Ne*64*nd*nd] of the value type; values [nnz] (or the symmetric block
// layout); when dinv is not null it receives the preconditioner: the inverse diagonal
// [N] (FEM_PRECOND_JACOBI) or the inverse node blocks [Nn*nd*nd], row-major
// (FEM_PRECOND_BLOCK_JACOBI).
template <typename T>
void launch_tangent(const fem_handle *h, const double *u, const double *theta, T *ke_scratch, T *values, T *dinv,
                    hipStream_t s, int layout = LAYOUT_CSR, int precond = FEM_PRECOND_JACOBI);
// y = (K(u) v) on free dofs with v used on every dof (Dirichlet lifting), 0 on Dirichlet dofs.
void launch_lift(const fem_handle *h, const double *u, const double *theta, const double *v, double *scratch,
                 double *y, hipStream_t s);
// y = M x (consistent mass of a nodal field, all dofs), scratch [Ne*8*nd] FP64.
void launch_mass(const fem_handle *h, const double *x, double *scratch, double *y, hipStream_t s);
void launch_vjp(const fem_handle *h, const double *u, const double *theta, const double *lam, double *g,
                hipStream_t s);
// J2: commit the history at u (after a converged load step); volume-averaged stress.
void launch_j2_commit(const fem_handle *h, const double *u, const double *theta, hipStream_t s);
void j2_average_stress(fem_handle *h, double out[6], hipStream_t s);
// Doubles of the per-block partials of j2_average_stress (allocated with the history).
size_t j2_partials_count(int64_t n_elems);
template <typename T>
void launch_extract_dinv(const fem_handle *h, const T *values, T *dinv, hipStream_t s, int layout = LAYOUT_CSR);

// ------------------------------------------------------------------ sparse / vector kernels
template <typename T>
void launch_spmv(const fem_handle *h, const T *values, int transpose, const T *x, T *y, T alpha, T beta,
                 hipStream_t s);
template <typename T>
void launch_spmv_sym(const fem_handle *h, const T *values, const T *x, T *y, T alpha, T beta, hipStream_t s);
void launch_export(const fem_handle *h, int64_t *row_ptr, int32_t *col_idx, int32_t *slot, int64_t *diag,
                   int32_t *tperm, hipStream_t s);

// Fused Krylov kernels (grid-stride, FP64 reductions finished by the last block).
int krylov_grid(const fem_handle *h);
size_t krylov_partials_bytes(const fem_handle *h);

template <typename T>
struct KrylovVecs {
    const T *A;  // values of the operator
    int layout;  // LAYOUT_CSR or LAYOUT_SYM
    T *x, *r, *rh, *p, *v, *s, *t, *ph, *sh;
    T *dinv;     // preconditioner: inverse diagonal [N] or inverse node blocks [Nn*nd*nd]
    int bj;      // 1: dinv holds node blocks (block Jacobi)
    double *partials;   // per-block partial sums written by one kernel ...
    double *partials2;  // ... and by the next one (the two alternate)
    KrylovScalars *sc;
    const float *A32 = nullptr;  // FP32 values under FP64 vectors (A unused then)
    int fold = 0;  // 1: point Jacobi folded into the values (BiCGSTAB on K D^{-1}; its iterate y, x = D^{-1} y)
};

template <typename T>
void kry_bicg_init(const fem_handle *h, const KrylovVecs<T> &k, const T *b, double rtol, hipStream_t s);
// BiCGSTAB iteration number `it` (0-based within this solve).  With the point Jacobi
// preconditioner the scalar updates are folded into the vector kernels, and
// kry_bicg_check brings the convergence flag up to date after iteration it - 1.
template <typename T>
void kry_bicg_iter(const fem_handle *h, const KrylovVecs<T> &k, int it, hipStream_t s, hipEvent_t *ev);
template <typename T>
void kry_bicg_check(const fem_handle *h, const KrylovVecs<T> &k, int it, hipStream_t s);
template <typename T>
void kry_cg_init(const fem_handle *h, const KrylovVecs<T> &k, const T *b, double rtol, hipStream_t s);
// Two-level preconditioned CG (amg.hip): init (z = M b) and iteration `it`.
template <typename T>
void kry_cg_amg_init(fem_handle *h, const KrylovVecs<T> &k, const T *b, double rtol, hipStream_t s);
template <typename T>
void kry_cg_amg_iter(fem_handle *h, const KrylovVecs<T> &k, int it, hipStream_t s, hipEvent_t *ev);
// Builds the aggregation (once) and the coarse operator and bounds for `values`.
void amg_setup(fem_handle *h);
template <typename T>
void amg_refresh(fem_handle *h, const T *values, const T *dinv, int precision, int smooth_degree, int coarse_degree,
                 hipStream_t s);
// z = M r in the solve precision (no convergence flag).
template <typename T>
void amg_apply(fem_handle *h, const T *values, const T *dinv, const T *r, T *z, const KrylovScalars *sc,
               hipStream_t s);
void amg_destroy(fem_handle *h);
void amg_coarse_values_f64(const fem_handle *h, double *out, hipStream_t s);
// CG kernels shared with the preconditioned iteration (linalg.hip).
int krylov_vec_grid_of(const fem_handle *h);
template <typename T>
int kry_spmv_q(const fem_handle *h, const KrylovVecs<T> &k, hipStream_t s);  // q = K p, (p, q) partials
template <typename T>
void kry_cg_p_update(const fem_handle *h, const KrylovVecs<T> &k, int it, hipStream_t s);
template <typename T>
void launch_spmv_sc(const fem_handle *h, const T *values, const T *x, T *y, T alpha, T beta, const KrylovScalars *sc,
                    hipStream_t s);
// CG iteration number `it` (0-based within this solve).
template <typename T>
void kry_cg_iter(const fem_handle *h, const KrylovVecs<T> &k, int it, hipStream_t s, hipEvent_t *ev);

// SIMP optimisation pieces (topopt.hip).
size_t vector_workspace_bytes(int64_t n);
void element_volumes(fem_handle *h, double *vol, bool normalized, hipStream_t s);
void filter_setup(fem_handle *h, double rmin);
void filter_apply(const fem_handle *h, int mode, const double *theta, const double *x, double *out, hipStream_t s);
double dot(const double *a, const double *b, int64_t n, void *ws, hipStream_t s);
void axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s);
double obs_misfit(int64_t n, int64_t n_obs, const int64_t *idx, const double *obs, const double *u, double *dJdu,
                  void *ws, hipStream_t s);
void set_load(fem_handle *h, const double *f, hipStream_t s);
double mma_update(int64_t n, int iter, const double *x, const double *xold1, const double *xold2, const double *df0,
                  double f1, const double *df1, double *low, double *upp, double *xnew, const fem_mma_opts &o,
                  void *ws, hipStream_t s);

// Vector helpers.
void launch_norm2_free(const fem_handle *h, const double *r, double *partials, double *out, hipStream_t s);
template <typename TO, typename TI>
void launch_scale_cast(const TI *in, TO *out, double alpha, int64_t n, hipStream_t s);
template <typename TI>
void launch_axpy_to_f64(const TI *x, double *y, int64_t n, hipStream_t s);
// values of column dof j *= dinv[j] (CSR layout of the node graph)
template <typename T>
void launch_scale_columns(const fem_handle *h, T *values, const T *dinv, hipStream_t s);
template <typename T>
void launch_mul_inplace(T *x, const T *d, int64_t n, hipStream_t s);
void launch_set_dirichlet(const fem_handle *h, double *u, const double *u0, const double *g, double lam,
                          hipStream_t s);
// delta = (u0 + lam (g - u0) - u) on Dirichlet dofs, 0 elsewhere
void launch_dirichlet_increment(const fem_handle *h, const double *u, const double *u0, const double *g, double lam,
                                double *delta, hipStream_t s);
// out = -(a + b)
void launch_neg_sum(const double *a, const double *b, double *out, int64_t n, hipStream_t s);
void launch_mask_copy(const fem_handle *h, const double *in, double *out, hipStream_t s);
void launch_sub(const double *a, const double *b, double *out, int64_t n, hipStream_t s);

}  // namespace fem

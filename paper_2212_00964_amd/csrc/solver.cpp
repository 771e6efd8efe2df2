// Host drivers of the hot path: Newton's method with incremental loading, the
// Jacobi-preconditioned Krylov solves inside it, and the adjoint gradient.  Every
// arithmetic step runs in device kernels; the host only sequences launches and
// reads a few scalars back (the Newton residual norm once per iteration, the
// Krylov convergence flags every `check_every` iterations).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "solver.h"

namespace fem {

namespace {

constexpr size_t kAlign = 256;

// Layout of the tangent inside the solvers.  The symmetric block layout stores half
// the values, but the transposed reads of its lower blocks miss L2 at these sizes
// (measured at 1M elements: 282 us and 1.83 GB fetched beyond L2 per SpMV, against
// ~245 us for the full CSR layout), so the solvers use CSR.
constexpr int kSolverLayout = LAYOUT_CSR;

// Point-Jacobi BiCGSTAB folds D^{-1} into the stored tangent (right preconditioning
// applied to the values once per assembly), which removes the D^{-1} p and D^{-1} s
// vectors from every iteration.
bool fold_jacobi(const fem_solve_opts &o) {
    return o.krylov == FEM_KRYLOV_BICGSTAB && o.precond == FEM_PRECOND_JACOBI;
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Bump allocator over the caller's workspace.
struct Carver {
    char *base;
    size_t used = 0, cap;
    bool dry;
    Carver(void *b, size_t c, bool d) : base(static_cast<char *>(b)), cap(c), dry(d) {}
    template <typename T>
    T *take(int64_t n) {
        size_t off = used;
        used = align_up(used + size_t(std::max<int64_t>(n, 1)) * sizeof(T));
        if (dry) return nullptr;
        if (used > cap) throw Error(FEM_ENOMEM, "workspace smaller than fem_workspace_bytes()");
        return reinterpret_cast<T *>(base + off);
    }
};

}  // namespace

void check_status(fem_handle *h, hipStream_t s) {
    FEM_HIP(hipMemcpyAsync(h->host_status, h->status, sizeof(int), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    int st = *h->host_status;
    if (st & ST_MESH) throw Error(FEM_EMESH, "non-positive Jacobian determinant at a Gauss point (invalid element)");
    if (st & ST_INVERTED) throw Error(FEM_EINVERTED, "det(F) <= 0 at a Gauss point (inverted material)");
    if (st & ST_NAN) throw Error(FEM_ENAN, "NaN or Inf in a residual, tangent or diagonal");
}

void reset_status(fem_handle *h, hipStream_t s) { FEM_HIP(hipMemsetAsync(h->status, 0, sizeof(int), s)); }

static std::string sci(double v) {
    char buf[32];
    std::snprintf(buf, sizeof buf, "%.3e", v);
    return buf;
}

// v32 (FEM_PREC_MIXED_V64, T = double): element blocks and values in FP32.
template <typename T>
static void carve_solve(Carver &c, const fem_handle *h, SolveWork &w, bool need_ke, bool v32 = false) {
    const Graph &g = h->g;
    const int64_t N = g.N;
    const int64_t nvals = kSolverLayout == LAYOUT_SYM ? g.nnzb_up * g.nd * g.nd : g.nnz;
    w.r64 = c.take<double>(N);
    w.u0 = c.take<double>(N);
    w.res64 = c.take<double>(N);
    w.lam64 = c.take<double>(N);
    w.ustep = c.take<double>(N);
    w.tmp64 = c.take<double>(N);
    w.rscr = c.take<double>(g.Ne * 8 * g.nd);
    w.v32 = v32;
    if (v32) {
        w.ke = need_ke ? static_cast<void *>(c.take<float>(g.Ne * 64 * g.nd * g.nd)) : nullptr;
        w.values = c.take<float>(nvals);
        w.dinv32 = c.take<float>(g.Nn * g.nd * g.nd);
    } else {
        w.ke = need_ke ? static_cast<void *>(c.take<T>(g.Ne * 64 * g.nd * g.nd)) : nullptr;
        w.values = c.take<T>(nvals);
    }
    w.b = c.take<T>(N);
    T *v[10];
    for (int i = 0; i < 9; ++i) v[i] = c.take<T>(N);
    v[9] = c.take<T>(g.Nn * g.nd * g.nd);  // preconditioner: diagonal or node blocks
    w.x = v[0];
    w.r = v[1];
    w.rh = v[2];
    w.p = v[3];
    w.v = v[4];
    w.s = v[5];
    w.t = v[6];
    w.ph = v[7];
    w.sh = v[8];
    w.dinv = v[9];
    w.partials = c.take<double>(3 * int64_t(krylov_grid(h)));  // up to 3 sums per block
    w.partials2 = c.take<double>(3 * int64_t(krylov_grid(h)));
    w.norm_partials = c.take<double>(krylov_grid(h));
    w.sc = c.take<KrylovScalars>(1);
    w.norm_out = c.take<double>(1);
}

size_t solve_workspace_bytes(const fem_handle *h, const fem_solve_opts *o) {
    Carver c(nullptr, 0, true);
    SolveWork w;
    if (o == nullptr) {
        c.take<double>(h->g.Ne * 64 * h->g.nd * h->g.nd);  // FP64 element blocks
        c.take<double>(h->g.Ne * 8 * h->g.nd);            // element vectors
        return c.used;
    }
    if (o->precision == FEM_PREC_MIXED) carve_solve<float>(c, h, w, true);
    else carve_solve<double>(c, h, w, true, o->precision == FEM_PREC_MIXED_V64);
    return c.used;
}

void carve_assemble(const fem_handle *h, void *ws, size_t bytes, void **ke, double **rscr, int dtype) {
    Carver c(ws, bytes, false);
    if (dtype == FEM_F32) *ke = c.take<float>(h->g.Ne * 64 * h->g.nd * h->g.nd);
    else *ke = c.take<double>(h->g.Ne * 64 * h->g.nd * h->g.nd);
    *rscr = c.take<double>(h->g.Ne * 8 * h->g.nd);
}

double norm2(fem_handle *h, const double *r, SolveWork &w, hipStream_t s) {
    launch_norm2_free(h, r, w.norm_partials, w.norm_out, s);
    FEM_HIP(hipMemcpyAsync(h->host_scalar, w.norm_out, sizeof(double), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    return std::sqrt(*h->host_scalar);
}

// Jacobi-preconditioned Krylov solve K x = b (x0 = 0) to ||b - K x|| <= rtol ||b||
// (recursive residual).  Returns the iteration count; throws on breakdown before
// any progress.
template <typename T>
int krylov_solve(fem_handle *h, SolveWork &w, const T *A, const fem_solve_opts &o, double rtol,
                 fem_solve_stats *st, hipStream_t s) {
    KrylovVecs<T> k{A,
                    kSolverLayout,
                    static_cast<T *>(w.x),
                    static_cast<T *>(w.r),
                    static_cast<T *>(w.rh),
                    static_cast<T *>(w.p),
                    static_cast<T *>(w.v),
                    static_cast<T *>(w.s),
                    static_cast<T *>(w.t),
                    static_cast<T *>(w.ph),
                    static_cast<T *>(w.sh),
                    static_cast<T *>(w.dinv),
                    o.precond == FEM_PRECOND_BLOCK_JACOBI,
                    w.partials,
                    w.partials2,
                    w.sc};
    k.fold = fold_jacobi(o) ? 1 : 0;
    if constexpr (sizeof(T) == 8)
        if (w.v32) {  // the FP32 tangent under FP64 vectors
            k.A = nullptr;
            k.A32 = static_cast<const float *>(w.values);
        }
    const bool cg = o.krylov == FEM_KRYLOV_CG;
    const bool amg = o.precond == FEM_PRECOND_AMG;  // CG only (checked at the ABI)
    const T *b = static_cast<const T *>(w.b);
    if (amg) kry_cg_amg_init<T>(h, k, b, rtol, s);
    else if (cg) kry_cg_init<T>(h, k, b, rtol, s);
    else kry_bicg_init<T>(h, k, b, rtol, s);
    // a two-level iteration costs several SpMVs: read convergence back more often
    const int every = amg ? std::max(1, std::min(o.check_every, 4)) : std::max(1, o.check_every);
    const int spmv_per_it = cg ? 1 : 2;
    std::vector<hipEvent_t> &ev = h->events;
    const bool prof = o.profile_spmv != 0;
    if (prof && ev.size() < 4) {
        size_t old = ev.size();
        ev.resize(4);
        for (size_t i = old; i < ev.size(); ++i) FEM_HIP(hipEventCreate(&ev[i]));
    }
    int its_done = 0;
    KrylovScalars hs{};
    for (int it = 0;; it += every) {
        for (int j = 0; j < every; ++j) {
            // timing samples the middle iteration of each check interval (away from the
            // host read-back at its end): an event pair around every SpMV would itself
            // cost about 4% of the iteration time
            hipEvent_t *e = (prof && j == every / 2) ? &ev[0] : nullptr;
            if (amg) kry_cg_amg_iter<T>(h, k, it + j, s, e);
            else if (cg) kry_cg_iter<T>(h, k, it + j, s, e);
            else kry_bicg_iter<T>(h, k, it + j, s, e);
        }
        if (!cg && !amg) kry_bicg_check<T>(h, k, it + every, s);
        FEM_HIP(hipMemcpyAsync(h->host_kry, w.sc, kScalarsHostBytes, hipMemcpyDeviceToHost, s));
        FEM_HIP(hipStreamSynchronize(s));
        std::memcpy(&hs, h->host_kry, kScalarsHostBytes);
        if (prof && st && hs.its > its_done + every / 2) {  // the sampled iteration did an update
            for (int q = 0; q < spmv_per_it; ++q) {
                float ms = 0.f;
                FEM_HIP(hipEventElapsedTime(&ms, ev[2 * q], ev[2 * q + 1]));
                st->spmv_ms_total += ms;
                st->spmv_calls += 1;
            }
        }
        its_done = hs.its;
        if (hs.converged) break;
        if (hs.breakdown) {
            if (hs.breakdown == 2) throw Error(FEM_ENAN, "NaN/Inf in a Krylov inner product");
            // CG's breakdown is a direction with p.Kp <= 0: the tangent is not positive
            // definite, so no CG iterate can be trusted
            if (cg)
                throw Error(FEM_EBREAKDOWN, "CG met non-positive curvature p.Kp <= 0 at iteration " +
                                                std::to_string(hs.its) + " (the tangent is not positive definite)");
            if (hs.its == 0) throw Error(FEM_EBREAKDOWN, "Krylov breakdown before the first update");
            break;  // keep the last iterate; the outer loop measures its true residual
        }
        if (it + every >= o.krylov_max_it) break;
    }
    if (k.fold) launch_mul_inplace<T>(k.x, k.dinv, h->g.N, s);  // x = D^{-1} y
    const double relres = hs.bnorm2 > 0.0 ? std::sqrt(hs.rnorm2 / hs.bnorm2) : 0.0;
    if (st) {
        st->krylov_its_total += hs.its;
        if (!hs.converged) st->krylov_unconverged++;
        if (st->n_hist < FEM_MAX_HIST) st->krylov_relres[st->n_hist] = relres;
    }
    // An unconverged solve is still a usable inexact correction as long as it reduced
    // the residual; one that grew it is rejected.
    if (!hs.converged && !(relres < 1.0))
        throw Error(hs.breakdown ? FEM_EBREAKDOWN : FEM_EMAXITER,
                    "Krylov solve stopped after " + std::to_string(hs.its) + " iterations with ||r||/||b|| = " +
                        sci(relres));
    return hs.its;
}

template int krylov_solve<float>(fem_handle *, SolveWork &, const float *, const fem_solve_opts &, double,
                                 fem_solve_stats *, hipStream_t);
template int krylov_solve<double>(fem_handle *, SolveWork &, const double *, const fem_solve_opts &, double,
                                  fem_solve_stats *, hipStream_t);

using clk = std::chrono::steady_clock;
static double ms_since(clk::time_point t0) {
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

template <typename T>
static void assemble_into(fem_handle *h, SolveWork &w, const double *u, const double *theta,
                          const fem_solve_opts &o, hipStream_t s) {
    if (w.v32) {
        if (o.precond == FEM_PRECOND_AMG)
            throw Error(FEM_EINVAL, "the two-level preconditioner takes FP32 or FP64 vectors, not FEM_PREC_MIXED_V64");
        launch_tangent<float>(h, u, theta, static_cast<float *>(w.ke), static_cast<float *>(w.values), w.dinv32, s,
                              kSolverLayout, o.precond);
        if (fold_jacobi(o)) launch_scale_columns<float>(h, static_cast<float *>(w.values), w.dinv32, s);
        const int64_t nd = h->g.nd;
        launch_scale_cast<double, float>(w.dinv32, static_cast<double *>(w.dinv), 1.0,
                                         o.precond == FEM_PRECOND_BLOCK_JACOBI ? h->g.Nn * nd * nd : h->g.N, s);
        return;
    }
    launch_tangent<T>(h, u, theta, static_cast<T *>(w.ke), static_cast<T *>(w.values), static_cast<T *>(w.dinv), s,
                      kSolverLayout, o.precond);
    if (fold_jacobi(o)) launch_scale_columns<T>(h, static_cast<T *>(w.values), static_cast<const T *>(w.dinv), s);
    if (o.precond == FEM_PRECOND_AMG)  // the coarse operator and bounds of this tangent
        amg_refresh<T>(h, static_cast<const T *>(w.values), static_cast<const T *>(w.dinv), o.precision,
                       o.amg_smooth_degree, o.amg_coarse_degree, s);
}

// One correction: assemble K(u), solve K du = b with b = sign * r64, u += du.  Plain:
// one Krylov solve in the solve precision to krylov_rtol on its recursive residual.
// Mixed with opts.refine_rtol > 0: FP32 sweeps, each restarted from the FP64
// residual b - K du of the matrix-free tangent and asked for at most a refine_rtol
// reduction of it, until ||b - K du|| <= krylov_rtol ||b|| (the FP64 iterative
// refinement of the correction itself).
template <typename T>
static int correction(fem_handle *h, SolveWork &w, double *u, const double *theta, const fem_solve_opts &o,
                      fem_solve_stats *st, double rn, double sign, hipStream_t s) {
    const int64_t N = h->g.N;
    auto t0 = clk::now();
    assemble_into<T>(h, w, u, theta, o, s);
    check_status(h, s);
    if (st) st->ms_assemble += ms_since(t0);
    t0 = clk::now();
    int kits = 0;
    double relres = -1.0;
    const bool refine = sizeof(T) == 4 && o.refine_rtol > 0.0;
    if (!refine) {
        launch_scale_cast<T, double>(w.r64, static_cast<T *>(w.b), sign, N, s);
        kits = krylov_solve<T>(h, w, static_cast<const T *>(w.values), o, o.krylov_rtol, st, s);
        launch_axpy_to_f64<T>(static_cast<const T *>(w.x), u, N, s);
    } else {
        // du (FP64) in lam64, the FP64 residual b - K du in res64
        FEM_HIP(hipMemsetAsync(w.lam64, 0, N * sizeof(double), s));
        launch_scale_cast<double, double>(w.r64, w.res64, sign, N, s);
        const double target = o.krylov_rtol * rn;
        double resn = rn;
        for (int sweep = 0; resn > target && sweep < o.adjoint_max_refine; ++sweep) {
            const double eta = std::min(0.5, std::max(o.refine_rtol, 0.5 * target / resn));
            launch_scale_cast<T, double>(w.res64, static_cast<T *>(w.b), 1.0, N, s);
            kits += krylov_solve<T>(h, w, static_cast<const T *>(w.values), o, eta, st, s);
            launch_axpy_to_f64<T>(static_cast<const T *>(w.x), w.lam64, N, s);
            launch_apply_tangent(h, u, theta, w.lam64, w.rscr, w.tmp64, s);
            if (sign > 0) launch_sub(w.r64, w.tmp64, w.res64, N, s);  // b - K du with b = r64
            else launch_neg_sum(w.r64, w.tmp64, w.res64, N, s);       // b - K du with b = -r64
            resn = norm2(h, w.res64, w, s);
            if (!std::isfinite(resn)) throw Error(FEM_ENAN, "non-finite refinement residual");
        }
        relres = rn > 0.0 ? resn / rn : 0.0;
        launch_axpy_to_f64<double>(w.lam64, u, N, s);
    }
    FEM_HIP(hipStreamSynchronize(s));
    if (st) {
        st->ms_krylov += ms_since(t0);
        if (st->n_hist < FEM_MAX_HIST) {
            st->krylov_its[st->n_hist] = kits;
            st->residual_hist[st->n_hist] = rn;
            if (relres >= 0.0) st->krylov_relres[st->n_hist] = relres;
            st->n_hist++;
        }
        st->newton_its++;
    }
    return kits;
}

// One load step of Newton's method, to the load factor lam.  The first iteration
// carries the Dirichlet increment D through the tangent at the previous state
// (du_D = D, K_ff du_f = -r_f - K_fD D); the following iterations solve
// K(u) du = -r(u) with the Dirichlet rows and columns eliminated.
template <typename T>
static void load_step(fem_handle *h, SolveWork &w, double *u, const double *theta, const double *gD, double lam,
                      int k, const fem_solve_opts &o, fem_solve_stats *st, hipStream_t s) {
    const int64_t N = h->g.N;
    auto t0 = clk::now();
    auto t_it = t0;  // start of the current Newton iteration
    // wall time of the Newton iteration whose correction was recorded last
    auto record_iter = [&] {
        if (st && st->n_hist >= 1 && st->n_hist <= FEM_MAX_HIST) st->iter_ms[st->n_hist - 1] = ms_since(t_it);
    };
    launch_dirichlet_increment(h, u, w.u0, gD, lam, w.res64, s);
    launch_residual(h, u, theta, lam, w.rscr, w.r64, s);
    launch_lift(h, u, theta, w.res64, w.rscr, w.lam64, s);
    launch_neg_sum(w.r64, w.lam64, w.r64, N, s);  // predictor right-hand side
    const double bn = norm2(h, w.r64, w, s);
    check_status(h, s);
    if (st) st->ms_residual += ms_since(t0);
    if (!std::isfinite(bn)) throw Error(FEM_ENAN, "non-finite Newton right-hand side");
    const double ref = std::max(bn, lam * h->m.fext_norm);
    const double tol = std::max(o.newton_rtol * ref, o.newton_atol);
    if (st) {
        st->initial_residual = bn;
        st->load_steps = k;
    }
    const int fixed = o.newton_fixed_its;
    int it = 0;
    if (bn > tol || fixed > 0) {
        if (o.newton_max_it < 1) throw Error(FEM_EMAXITER, "newton_max_it = 0");
        correction<T>(h, w, u, theta, o, st, bn, 1.0, s);
        ++it;
    }
    launch_set_dirichlet(h, u, w.u0, gD, lam, s);
    t0 = clk::now();
    launch_residual(h, u, theta, lam, w.rscr, w.r64, s);
    double rn = norm2(h, w.r64, w, s);
    check_status(h, s);
    if (st) st->ms_residual += ms_since(t0);
    if (it > 0) record_iter();
    while (fixed > 0 ? it < fixed : !(rn <= tol)) {
        if (!std::isfinite(rn)) throw Error(FEM_ENAN, "non-finite Newton residual");
        if (rn > 1e8 * std::max(ref, 1e-300)) throw Error(FEM_EDIVERGED, "Newton residual diverged");
        if (fixed == 0 && it >= o.newton_max_it)
            throw Error(FEM_EMAXITER, "Newton did not converge in load step " + std::to_string(k) +
                                          " (|r| = " + sci(rn) + ", tol = " + sci(tol) + ")");
        t_it = clk::now();
        correction<T>(h, w, u, theta, o, st, rn, -1.0, s);
        t0 = clk::now();
        launch_residual(h, u, theta, lam, w.rscr, w.r64, s);
        rn = norm2(h, w.r64, w, s);
        check_status(h, s);
        if (st) st->ms_residual += ms_since(t0);
        record_iter();
        ++it;
    }
    if (st) st->final_residual = rn;
    launch_j2_commit(h, u, theta, s);  // path-dependent laws: the converged step becomes the history
}

// Failures a smaller load increment can cure.
static bool recoverable(int code) {
    return code == FEM_EBREAKDOWN || code == FEM_EMAXITER || code == FEM_EDIVERGED || code == FEM_EINVERTED ||
           code == FEM_ENAN;
}

// Newton's method with incremental loading: load step k of n moves the load factor to
// k/n.  With opts.max_bisections > 0 a failed step is retried from its starting state
// with half the remaining increment (at most max_bisections halvings per load step);
// every converged sub-step commits the history of path-dependent laws.
template <typename T>
static void newton_impl(fem_handle *h, double *u, const double *theta, const double *gD, const fem_solve_opts &o,
                        fem_solve_stats *st, void *ws, size_t wsb, hipStream_t s) {
    Carver c(ws, wsb, false);
    SolveWork w;
    carve_solve<T>(c, h, w, true, o.precision == FEM_PREC_MIXED_V64);
    const int64_t N = h->g.N;
    auto t_all = clk::now();
    reset_status(h, s);
    FEM_HIP(hipMemcpyAsync(w.u0, u, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    const int nsteps = std::max(1, o.n_load_steps);
    double lam_done = 0.0;
    for (int k = 1; k <= nsteps; ++k) {
        const double lam_k = double(k) / nsteps;
        if (o.max_bisections == 0) {
            load_step<T>(h, w, u, theta, gD, lam_k, k, o, st, s);
            lam_done = lam_k;
            continue;
        }
        double inc = lam_k - lam_done;
        int halvings = 0;
        while (lam_done < lam_k) {
            // the last sub-step lands exactly on lam_k
            const double target = (lam_done + inc >= lam_k - 1e-12 * inc) ? lam_k : lam_done + inc;
            FEM_HIP(hipMemcpyAsync(w.ustep, u, N * sizeof(double), hipMemcpyDeviceToDevice, s));
            try {
                load_step<T>(h, w, u, theta, gD, target, k, o, st, s);
                lam_done = target;
            } catch (const Error &e) {
                if (!recoverable(e.code) || halvings >= o.max_bisections) throw;
                FEM_HIP(hipMemcpyAsync(u, w.ustep, N * sizeof(double), hipMemcpyDeviceToDevice, s));
                reset_status(h, s);
                FEM_HIP(hipStreamSynchronize(s));
                inc *= 0.5;
                ++halvings;
                if (st) st->bisections++;
            }
        }
    }
    if (st) st->ms_total += ms_since(t_all);
}

void newton_solve(fem_handle *h, double *u, const double *theta, const double *gD, const fem_solve_opts &o,
                  fem_solve_stats *st, void *ws, size_t wsb, hipStream_t s) {
    if (o.precision == FEM_PREC_MIXED) newton_impl<float>(h, u, theta, gD, o, st, ws, wsb, s);
    else newton_impl<double>(h, u, theta, gD, o, st, ws, wsb, s);
}

template <typename T>
static void adjoint_impl(fem_handle *h, const double *u, const double *theta, const double *dJdu, double *g,
                         double *lam_out, const fem_solve_opts &o, fem_solve_stats *st, void *ws, size_t wsb,
                         hipStream_t s) {
    Carver c(ws, wsb, false);
    SolveWork w;
    carve_solve<T>(c, h, w, true, o.precision == FEM_PREC_MIXED_V64);
    const int64_t N = h->g.N;
    auto t_all = clk::now();
    reset_status(h, s);
    auto t0 = clk::now();
    // All laws here have major-symmetric tangents and the Dirichlet elimination is
    // symmetric, so (dC/du)^T is the assembled K itself.
    assemble_into<T>(h, w, u, theta, o, s);
    launch_mask_copy(h, dJdu, w.res64, s);  // b = dJ/du with Dirichlet entries 0
    double bn = norm2(h, w.res64, w, s);
    check_status(h, s);
    if (st) st->ms_assemble += ms_since(t0);
    FEM_HIP(hipMemsetAsync(w.lam64, 0, N * sizeof(double), s));
    FEM_HIP(hipMemcpyAsync(w.r64, w.res64, N * sizeof(double), hipMemcpyDeviceToDevice, s));  // r64 = b
    double rn = bn;
    const double tol = std::max(o.adjoint_rtol * bn, 0.0);
    int sweeps = 0;
    while (rn > tol) {
        if (!std::isfinite(rn)) throw Error(FEM_ENAN, "non-finite adjoint residual");
        if (sweeps >= o.adjoint_max_refine) throw Error(FEM_EMAXITER, "adjoint refinement did not converge");
        t0 = clk::now();
        launch_scale_cast<T, double>(w.res64, static_cast<T *>(w.b), 1.0, N, s);
        // Each sweep asks only for what is still missing, with a factor 2 of margin for
        // the gap between the recursive and the true residual; with refine_rtol > 0 (mixed)
        // it asks for at most that reduction and restarts from the FP64 residual.
        const double floor_rtol = (sizeof(T) == 4 && o.refine_rtol > 0.0) ? o.refine_rtol : o.krylov_rtol;
        const double eta = std::min(0.5, std::max(floor_rtol, 0.5 * tol / rn));
        int kits = krylov_solve<T>(h, w, static_cast<const T *>(w.values), o, eta, st, s);
        launch_axpy_to_f64<T>(static_cast<const T *>(w.x), w.lam64, N, s);
        if (st) {
            st->ms_krylov += ms_since(t0);
            if (st->n_hist < FEM_MAX_HIST) {
                st->krylov_its[st->n_hist] = kits;
                st->residual_hist[st->n_hist] = rn;
                st->n_hist++;
            }
        }
        // FP64 refinement residual with the matrix-free tangent: res = b - K(u) lambda
        t0 = clk::now();
        launch_apply_tangent(h, u, theta, w.lam64, w.rscr, w.u0, s);
        launch_sub(w.r64, w.u0, w.res64, N, s);
        launch_mask_copy(h, w.res64, w.res64, s);
        rn = norm2(h, w.res64, w, s);
        check_status(h, s);
        if (st) st->ms_residual += ms_since(t0);
        ++sweeps;
    }
    t0 = clk::now();
    launch_vjp(h, u, theta, w.lam64, g, s);
    if (lam_out) FEM_HIP(hipMemcpyAsync(lam_out, w.lam64, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    check_status(h, s);
    if (st) {
        st->ms_vjp += ms_since(t0);
        st->final_residual = rn;
        st->initial_residual = bn;
        st->newton_its += sweeps;
        st->ms_total += ms_since(t_all);
    }
}

template <typename T>
static void amg_apply_impl(fem_handle *h, const double *u, const double *theta, const double *r, double *z,
                           const fem_solve_opts &o, double *lmax_out, double *coarse_values, void *ws, size_t wsb,
                           hipStream_t s) {
    Carver c(ws, wsb, false);
    SolveWork w;
    carve_solve<T>(c, h, w, true, o.precision == FEM_PREC_MIXED_V64);
    const int64_t N = h->g.N;
    reset_status(h, s);
    assemble_into<T>(h, w, u, theta, o, s);
    check_status(h, s);
    launch_scale_cast<T, double>(r, static_cast<T *>(w.b), 1.0, N, s);
    amg_apply<T>(h, static_cast<const T *>(w.values), static_cast<const T *>(w.dinv), static_cast<const T *>(w.b),
                 static_cast<T *>(w.x), nullptr, s);
    FEM_HIP(hipMemsetAsync(z, 0, N * sizeof(double), s));
    launch_axpy_to_f64<T>(static_cast<const T *>(w.x), z, N, s);
    if (coarse_values) amg_coarse_values_f64(h, coarse_values, s);
    FEM_HIP(hipStreamSynchronize(s));
    if (lmax_out) {
        lmax_out[0] = h->amg->lmax;
        lmax_out[1] = h->amg->lmax_c;
    }
}

void amg_apply_once(fem_handle *h, const double *u, const double *theta, const double *r, double *z,
                    const fem_solve_opts &o, double *lmax_out, double *coarse_values, void *ws, size_t wsb,
                    hipStream_t s) {
    if (o.precision == FEM_PREC_MIXED)
        amg_apply_impl<float>(h, u, theta, r, z, o, lmax_out, coarse_values, ws, wsb, s);
    else amg_apply_impl<double>(h, u, theta, r, z, o, lmax_out, coarse_values, ws, wsb, s);
}

void adjoint_vjp(fem_handle *h, const double *u, const double *theta, const double *dJdu, double *g,
                 double *lam_out, const fem_solve_opts &o, fem_solve_stats *st, void *ws, size_t wsb,
                 hipStream_t s) {
    if (o.precision == FEM_PREC_MIXED) adjoint_impl<float>(h, u, theta, dJdu, g, lam_out, o, st, ws, wsb, s);
    else adjoint_impl<double>(h, u, theta, dJdu, g, lam_out, o, st, ws, wsb, s);
}

}  // namespace fem

// Host drivers of Newton, Krylov and adjoint solves (internal).
#pragma once

#include "internal.h"

namespace fem {

// Views into the caller's workspace for one solve.
struct SolveWork {
    double *r64 = nullptr, *u0 = nullptr, *res64 = nullptr, *lam64 = nullptr, *rscr = nullptr;
    double *ustep = nullptr;  // u at the start of a load step (restored by the load-step recovery)
    double *tmp64 = nullptr;  // FP64 scratch vector (tangent products of the refined correction)
    void *ke = nullptr, *values = nullptr, *b = nullptr;
    void *x = nullptr, *r = nullptr, *rh = nullptr, *p = nullptr, *v = nullptr, *s = nullptr, *t = nullptr,
         *ph = nullptr, *sh = nullptr, *dinv = nullptr;
    double *partials = nullptr, *partials2 = nullptr, *norm_partials = nullptr, *norm_out = nullptr;
    KrylovScalars *sc = nullptr;
    // FEM_PREC_MIXED_V64: ke and values hold FP32 under FP64 vectors; the gather writes
    // the FP32 preconditioner to dinv32, cast into dinv
    bool v32 = false;
    float *dinv32 = nullptr;
};

size_t solve_workspace_bytes(const fem_handle *h, const fem_solve_opts *o);
void carve_assemble(const fem_handle *h, void *ws, size_t bytes, void **ke, double **rscr, int dtype);
void check_status(fem_handle *h, hipStream_t s);
void reset_status(fem_handle *h, hipStream_t s);
double norm2(fem_handle *h, const double *r, SolveWork &w, hipStream_t s);
template <typename T>
int krylov_solve(fem_handle *h, SolveWork &w, const T *A, const fem_solve_opts &o, double rtol, fem_solve_stats *st,
                 hipStream_t s);
void newton_solve(fem_handle *h, double *u, const double *theta, const double *gD, const fem_solve_opts &o,
                  fem_solve_stats *st, void *ws, size_t wsb, hipStream_t s);
void adjoint_vjp(fem_handle *h, const double *u, const double *theta, const double *dJdu, double *g, double *lam_out,
                 const fem_solve_opts &o, fem_solve_stats *st, void *ws, size_t wsb, hipStream_t s);
// Assembles K(u), builds the two-level preconditioner for it and applies it once.
void amg_apply_once(fem_handle *h, const double *u, const double *theta, const double *r, double *z,
                    const fem_solve_opts &o, double *lmax_out, double *coarse_values, void *ws, size_t wsb,
                    hipStream_t s);

}  // namespace fem

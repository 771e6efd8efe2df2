// C ABI of libfem: argument checks, handle lifetime, error translation.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "solver.h"

namespace {

thread_local std::string g_last_error;

template <typename F>
int guarded(F &&f) {
    try {
        f();
        g_last_error.clear();
        return FEM_OK;
    } catch (const fem::Error &e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return FEM_ENOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return FEM_EINVAL;
    } catch (...) {
        g_last_error = "unknown error";
        return FEM_EINVAL;
    }
}

void require(bool ok, const char *what) {
    if (!ok) throw fem::Error(FEM_EINVAL, what);
}

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

void bind_device(const fem_handle *h) { FEM_HIP(hipSetDevice(h->device)); }

void validate_opts(const fem_solve_opts *o) {
    require(o != nullptr, "opts is NULL");
    require(o->precision == FEM_PREC_FP64 || o->precision == FEM_PREC_MIXED || o->precision == FEM_PREC_MIXED_V64,
            "opts.precision");
    require(o->krylov == FEM_KRYLOV_CG || o->krylov == FEM_KRYLOV_BICGSTAB, "opts.krylov");
    require(o->n_load_steps >= 1, "opts.n_load_steps must be >= 1");
    require(o->newton_max_it >= 0 && o->krylov_max_it >= 1 && o->check_every >= 1, "opts iteration limits");
    require(o->krylov_rtol > 0.0 && o->krylov_rtol < 1.0, "opts.krylov_rtol must be in (0, 1)");
    require(o->newton_rtol >= 0.0 && o->newton_atol >= 0.0 && o->adjoint_rtol >= 0.0, "opts tolerances");
    require(o->adjoint_max_refine >= 1, "opts.adjoint_max_refine must be >= 1");
    require(o->newton_fixed_its >= 0, "opts.newton_fixed_its must be >= 0");
    require(o->max_bisections >= 0 && o->max_bisections <= 30, "opts.max_bisections must be in [0, 30]");
    require(o->refine_rtol >= 0.0 && o->refine_rtol < 1.0, "opts.refine_rtol must be in [0, 1)");
    require(o->precond == FEM_PRECOND_JACOBI || o->precond == FEM_PRECOND_BLOCK_JACOBI ||
                o->precond == FEM_PRECOND_AMG,
            "opts.precond");
    if (o->precond == FEM_PRECOND_AMG) {
        require(o->krylov == FEM_KRYLOV_CG, "FEM_PRECOND_AMG needs FEM_KRYLOV_CG");
        require(o->precision != FEM_PREC_MIXED_V64, "FEM_PRECOND_AMG takes FEM_PREC_FP64 or FEM_PREC_MIXED");
        require(o->amg_smooth_degree >= 1 && o->amg_smooth_degree <= 64, "opts.amg_smooth_degree must be in [1, 64]");
        require(o->amg_coarse_degree >= 1 && o->amg_coarse_degree <= 64, "opts.amg_coarse_degree must be in [1, 64]");
    }
}

void require_amg_ready(const fem_handle *h, const fem_solve_opts *o) {
    if (o->precond == FEM_PRECOND_AMG && h->g.N > 0)
        require(h->amg != nullptr, "FEM_PRECOND_AMG needs fem_amg_setup on the handle first");
}

void check_workspace(const fem_handle *h, const fem_solve_opts *o, void *ws, size_t bytes) {
    size_t need = fem::solve_workspace_bytes(h, o);
    if (need > 0 && ws == nullptr) throw fem::Error(FEM_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) throw fem::Error(FEM_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < need)
        throw fem::Error(FEM_ENOMEM, "workspace of " + std::to_string(bytes) + " bytes, need " + std::to_string(need));
}

// Host checks of a mesh description, before any device work.
void validate_mesh(const fem_mesh_desc *d) {
    require(d->n_nodes >= 0 && d->n_elems >= 0, "negative mesh size");
    require(d->model == FEM_POISSON || d->model == FEM_LINEAR_ELASTIC || d->model == FEM_NEO_HOOKEAN ||
                d->model == FEM_J2_PLASTIC,
            "model");
    require(d->ndpn == (d->model == FEM_POISSON ? 1 : 3), "ndpn must be 1 for FEM_POISSON and 3 otherwise");
    require(d->pmap == FEM_THETA_IDENTITY || d->pmap == FEM_THETA_SIMP, "pmap");
    require(d->n_nodes < (int64_t(1) << 31) / 3, "too many nodes for 32-bit dof indices");
    require(d->n_nodes == 0 || d->coords != nullptr, "coords is NULL");
    require(d->n_elems == 0 || d->conn != nullptr, "conn is NULL");
    require(d->n_traction_faces >= 0 && (d->n_traction_faces == 0 || (d->traction_faces && d->traction)),
            "traction faces");
    if (d->model == FEM_LINEAR_ELASTIC) require(d->nu > -1.0 && d->nu < 0.5, "nu must be in (-1, 0.5)");
    if (d->model == FEM_NEO_HOOKEAN) require(d->bulk_ratio > 0.0, "bulk_ratio must be > 0");
    if (d->model == FEM_J2_PLASTIC) {
        require(d->nu > -1.0 && d->nu < 0.5, "nu must be in (-1, 0.5)");
        require(d->yield_stress > 0.0 && std::isfinite(d->yield_stress), "yield_stress must be > 0");
    }
    // every node must belong to an element (otherwise its row has no diagonal)
    {
        std::vector<uint8_t> used(d->n_nodes, 0);
        for (int64_t i = 0; i < d->n_elems * 8; ++i) {
            require(d->conn[i] >= 0 && d->conn[i] < d->n_nodes, "connectivity references a missing node");
            used[d->conn[i]] = 1;
        }
        for (int64_t n = 0; n < d->n_nodes; ++n) require(used[n], "a node belongs to no element");
        // A HEX8 element lists 8 distinct nodes: a collapsed element would send two of
        // its node blocks to one matrix block, which the tangent gather adds once.
        for (int64_t e = 0; e < d->n_elems; ++e) {
            const int32_t *c = d->conn + 8 * e;
            for (int a = 0; a < 8; ++a)
                for (int b = a + 1; b < 8; ++b)
                    require(c[a] != c[b], ("element " + std::to_string(e) + " lists a node twice").c_str());
        }
    }
}

}  // namespace

int fem::run_guarded(const std::function<void()> &f) { return guarded(f); }

extern "C" {

const char *fem_last_error(void) { return g_last_error.c_str(); }

int fem_default_opts(fem_solve_opts *o) {
    return guarded([&] {
        require(o != nullptr, "opts is NULL");
        std::memset(o, 0, sizeof(*o));
        o->precision = FEM_PREC_FP64;
        o->krylov = FEM_KRYLOV_BICGSTAB;
        o->n_load_steps = 1;
        o->newton_max_it = 30;
        o->newton_rtol = 1e-10;
        o->newton_atol = 0.0;
        o->krylov_rtol = 1e-6;
        o->krylov_max_it = 20000;
        o->check_every = 16;
        o->adjoint_rtol = 1e-10;
        o->adjoint_max_refine = 20;
        o->profile_spmv = 0;
        o->amg_smooth_degree = 1;
        o->amg_coarse_degree = 16;
        o->newton_fixed_its = 0;
        o->precond = FEM_PRECOND_JACOBI;
    });
}

int fem_build_pattern(const fem_mesh_desc *d, fem_handle **out, int64_t *n_dofs, int64_t *nnz) {
    fem_handle *h = nullptr;
    int rc = guarded([&] {
        require(d != nullptr && out != nullptr, "desc and out must be non-NULL");
        *out = nullptr;
        validate_mesh(d);
        h = new fem_handle();
        FEM_HIP(hipGetDevice(&h->device));
        FEM_HIP(hipDeviceGetAttribute(&h->num_cus, hipDeviceAttributeMultiprocessorCount, h->device));
        h->mat = fem::Material{d->model,   d->pmap,      d->nu,      d->bulk_ratio,
                               d->simp_p, d->simp_emin, d->simp_e0, d->yield_stress};
        const int64_t N = d->n_nodes * d->ndpn;
        h->m.coords = static_cast<double *>(fem::dev_alloc(h, d->n_nodes * 3 * sizeof(double)));
        h->m.conn = static_cast<int32_t *>(fem::dev_alloc(h, d->n_elems * 8 * sizeof(int32_t)));
        h->m.mask = static_cast<uint8_t *>(fem::dev_alloc(h, N));
        if (d->n_nodes) FEM_HIP(hipMemcpy(h->m.coords, d->coords, d->n_nodes * 3 * sizeof(double), hipMemcpyHostToDevice));
        if (d->n_elems) FEM_HIP(hipMemcpy(h->m.conn, d->conn, d->n_elems * 8 * sizeof(int32_t), hipMemcpyHostToDevice));
        h->m.host_mask.assign(N, 0);
        if (d->dirichlet_mask)
            for (int64_t i = 0; i < N; ++i) h->m.host_mask[i] = d->dirichlet_mask[i] ? 1 : 0;
        if (N) FEM_HIP(hipMemcpy(h->m.mask, h->m.host_mask.data(), N, hipMemcpyHostToDevice));
        fem::build_load_vector(h, d);
        fem::build_graph(h, d);
        // SpMV group width: a power of two covering the typical node degree; FEM_SPMV_GROUP overrides it.
        if (const char *gs = std::getenv("FEM_SPMV_GROUP")) {
            int gv = std::atoi(gs);
            if (gv == 4 || gv == 8 || gv == 16 || gv == 32) h->spmv_group = gv;
        }
        h->status = static_cast<int *>(fem::dev_alloc(h, sizeof(int)));
        FEM_HIP(hipMemset(h->status, 0, sizeof(int)));
        FEM_HIP(hipHostMalloc(reinterpret_cast<void **>(&h->host_status), sizeof(int)));
        FEM_HIP(hipHostMalloc(reinterpret_cast<void **>(&h->host_scalar), sizeof(double)));
        FEM_HIP(hipHostMalloc(reinterpret_cast<void **>(&h->host_kry), fem::kScalarsHostBytes));
        if (n_dofs) *n_dofs = h->g.N;
        if (nnz) *nnz = h->g.nnz;
        *out = h;
    });
    if (rc != FEM_OK && h) fem_destroy(h);
    return rc;
}

int fem_pattern_host(const fem_mesh_desc *d, int64_t *n_dofs, int64_t *nnz, int64_t *row_ptr, int32_t *col_idx,
                     double *f_ext) {
    return guarded([&] {
        require(d != nullptr, "desc is NULL");
        validate_mesh(d);
        const int64_t N = d->n_nodes * d->ndpn;
        std::vector<uint8_t> mask(N, 0);
        if (d->dirichlet_mask)
            for (int64_t i = 0; i < N; ++i) mask[i] = d->dirichlet_mask[i] ? 1 : 0;
        const fem::HostGraph g = fem::host_graph(d, mask);
        if (n_dofs) *n_dofs = g.N;
        if (nnz) *nnz = g.nnz;
        if (row_ptr) std::copy(g.row_ptr.begin(), g.row_ptr.end(), row_ptr);
        if (col_idx) {
            // the nd rows of node n list the node's neighbour blocks, component-interleaved
            const int nd = g.nd;
            for (int64_t n = 0; n < g.Nn; ++n)
                for (int c = 0; c < nd; ++c) {
                    int64_t pos = g.row_ptr[nd * n + c];
                    for (int64_t k = g.node_ptr[n]; k < g.node_ptr[n + 1]; ++k)
                        for (int q = 0; q < nd; ++q) col_idx[pos++] = int32_t(int64_t(nd) * g.node_nb[k] + q);
                }
        }
        if (f_ext) {
            const std::vector<double> F = fem::host_load_vector(d);
            std::copy(F.begin(), F.end(), f_ext);
        }
    });
}

void fem_destroy(fem_handle *h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    for (auto &e : h->events) (void)hipEventDestroy(e);
    for (void *p : h->allocations) (void)hipFree(p);
    for (void *p : h->filter.allocations) (void)hipFree(p);
    if (h->host_status) (void)hipHostFree(h->host_status);
    if (h->host_scalar) (void)hipHostFree(h->host_scalar);
    if (h->host_kry) (void)hipHostFree(h->host_kry);
    fem::amg_destroy(h);
    delete h;
}

int fem_pattern_export(fem_handle *h, int64_t *row_ptr, int32_t *col_idx, int32_t *slot_map, int64_t *diag_slot,
                       int32_t *transpose_perm, void *stream) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        bind_device(h);
        fem::launch_export(h, row_ptr, col_idx, slot_map, diag_slot, transpose_perm, as_stream(stream));
    });
}

int fem_load_vector(fem_handle *h, double *f_ext, void *stream) {
    return guarded([&] {
        require(h != nullptr && f_ext != nullptr, "handle and f_ext must be non-NULL");
        bind_device(h);
        if (h->g.N)
            FEM_HIP(hipMemcpyAsync(f_ext, h->m.fext, h->g.N * sizeof(double), hipMemcpyDeviceToDevice,
                                   as_stream(stream)));
    });
}

int fem_workspace_bytes(fem_handle *h, const fem_solve_opts *o, size_t *bytes) {
    return guarded([&] {
        require(h != nullptr && bytes != nullptr, "handle and bytes must be non-NULL");
        if (o) validate_opts(o);
        *bytes = fem::solve_workspace_bytes(h, o);
    });
}

int fem_values_count(fem_handle *h, int32_t layout, int64_t *count) {
    return guarded([&] {
        require(h != nullptr && count != nullptr, "handle and count must be non-NULL");
        require(layout == FEM_LAYOUT_CSR || layout == FEM_LAYOUT_SYM_BLOCK, "layout");
        *count = layout == FEM_LAYOUT_CSR ? h->g.nnz : h->g.nnzb_up * h->g.nd * h->g.nd;
    });
}

int fem_assemble(fem_handle *h, const double *u, const double *theta, double *residual, void *values,
                 int32_t values_dtype, int32_t values_layout, void *workspace, size_t workspace_bytes, void *stream) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        require(values_dtype == FEM_F32 || values_dtype == FEM_F64, "values_dtype");
        require(values_layout == FEM_LAYOUT_CSR || values_layout == FEM_LAYOUT_SYM_BLOCK, "values_layout");
        const int ly = values_layout == FEM_LAYOUT_SYM_BLOCK ? fem::LAYOUT_SYM : fem::LAYOUT_CSR;
        const bool work = h->g.N > 0 && (residual || values);
        if (!work) return;
        require(u != nullptr && theta != nullptr, "u and theta must be non-NULL");
        check_workspace(h, nullptr, workspace, workspace_bytes);
        bind_device(h);
        hipStream_t s = as_stream(stream);
        void *ke;
        double *rscr;
        fem::carve_assemble(h, workspace, workspace_bytes, &ke, &rscr, values_dtype);
        fem::reset_status(h, s);
        if (residual) fem::launch_residual(h, u, theta, 1.0, rscr, residual, s);
        if (values) {
            if (values_dtype == FEM_F32)
                fem::launch_tangent<float>(h, u, theta, static_cast<float *>(ke), static_cast<float *>(values), nullptr, s,
                                           ly);
            else
                fem::launch_tangent<double>(h, u, theta, static_cast<double *>(ke), static_cast<double *>(values), nullptr, s,
                                            ly);
        }
        // enqueue only: the kernels' error bits stay in the status word for fem_check
    });
}

int fem_check(fem_handle *h, void *stream) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        bind_device(h);
        hipStream_t s = as_stream(stream);
        try {
            fem::check_status(h, s);
        } catch (const fem::Error &) {
            fem::reset_status(h, s);  // reported once
            FEM_HIP(hipStreamSynchronize(s));
            throw;
        }
    });
}

int fem_spmv(fem_handle *h, const void *values, int32_t dtype, int32_t layout, int32_t transpose, const void *x,
             void *y, double alpha, double beta, void *stream) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        require(dtype == FEM_F32 || dtype == FEM_F64, "dtype");
        require(layout == FEM_LAYOUT_CSR || layout == FEM_LAYOUT_SYM_BLOCK, "layout");
        if (h->g.N == 0) return;
        require(values && x && y, "values, x and y must be non-NULL");
        bind_device(h);
        if (layout == FEM_LAYOUT_SYM_BLOCK) {
            if (dtype == FEM_F32)
                fem::launch_spmv_sym<float>(h, static_cast<const float *>(values), static_cast<const float *>(x),
                                            static_cast<float *>(y), float(alpha), float(beta), as_stream(stream));
            else
                fem::launch_spmv_sym<double>(h, static_cast<const double *>(values), static_cast<const double *>(x),
                                             static_cast<double *>(y), alpha, beta, as_stream(stream));
            return;
        }
        if (dtype == FEM_F32)
            fem::launch_spmv<float>(h, static_cast<const float *>(values), transpose, static_cast<const float *>(x),
                                    static_cast<float *>(y), float(alpha), float(beta), as_stream(stream));
        else
            fem::launch_spmv<double>(h, static_cast<const double *>(values), transpose, static_cast<const double *>(x),
                                     static_cast<double *>(y), alpha, beta, as_stream(stream));
    });
}

int fem_apply_tangent(fem_handle *h, const double *u, const double *theta, const double *v, double *y,
                      void *workspace, size_t workspace_bytes, void *stream) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        if (h->g.N == 0) return;
        require(u && theta && v && y, "u, theta, v and y must be non-NULL");
        check_workspace(h, nullptr, workspace, workspace_bytes);
        bind_device(h);
        void *ke;
        double *rscr;
        fem::carve_assemble(h, workspace, workspace_bytes, &ke, &rscr, FEM_F64);
        fem::launch_apply_tangent(h, u, theta, v, rscr, y, as_stream(stream));
    });
}

int fem_newton_solve(fem_handle *h, double *u, const double *theta, const double *dirichlet_values,
                     const fem_solve_opts *opts, fem_solve_stats *stats, void *workspace, size_t workspace_bytes,
                     void *stream) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        validate_opts(opts);
        if (stats) std::memset(stats, 0, sizeof(*stats));
        if (h->g.N == 0) return;
        require(u && theta && dirichlet_values, "u, theta and dirichlet_values must be non-NULL");
        require_amg_ready(h, opts);
        check_workspace(h, opts, workspace, workspace_bytes);
        bind_device(h);
        fem::newton_solve(h, u, theta, dirichlet_values, *opts, stats, workspace, workspace_bytes, as_stream(stream));
    });
}

int fem_adjoint_vjp(fem_handle *h, const double *u, const double *theta, const double *dJdu, double *vjp_theta,
                    double *lambda_out, const fem_solve_opts *opts, fem_solve_stats *stats, void *workspace,
                    size_t workspace_bytes, void *stream) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        validate_opts(opts);
        if (stats) std::memset(stats, 0, sizeof(*stats));
        if (h->g.N == 0) return;
        require(h->mat.model != FEM_J2_PLASTIC, "the adjoint is not defined for FEM_J2_PLASTIC");
        require(u && theta && dJdu && vjp_theta, "u, theta, dJdu and vjp_theta must be non-NULL");
        require_amg_ready(h, opts);
        check_workspace(h, opts, workspace, workspace_bytes);
        bind_device(h);
        fem::adjoint_vjp(h, u, theta, dJdu, vjp_theta, lambda_out, *opts, stats, workspace, workspace_bytes,
                         as_stream(stream));
    });
}

int fem_history_copy(fem_handle *h, double *buf, int32_t into_handle, void *stream) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        require(h->mat.model == FEM_J2_PLASTIC, "the handle's law has no history (FEM_J2_PLASTIC only)");
        require(into_handle == 0 || into_handle == 1, "into_handle must be 0 or 1");
        if (h->g.Ne == 0) return;
        require(buf != nullptr, "buf is NULL");
        bind_device(h);
        const size_t bytes = size_t(h->g.Ne) * 96 * sizeof(double);
        if (into_handle)
            FEM_HIP(hipMemcpyAsync(h->hist, buf, bytes, hipMemcpyDeviceToDevice, as_stream(stream)));
        else
            FEM_HIP(hipMemcpyAsync(buf, h->hist, bytes, hipMemcpyDeviceToDevice, as_stream(stream)));
    });
}

int fem_average_stress(fem_handle *h, double *out, void *stream) {
    return guarded([&] {
        require(h != nullptr && out != nullptr, "handle and out must be non-NULL");
        require(h->mat.model == FEM_J2_PLASTIC, "the handle's law has no history (FEM_J2_PLASTIC only)");
        bind_device(h);
        fem::j2_average_stress(h, out, as_stream(stream));
    });
}

int fem_amg_setup(fem_handle *h) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        bind_device(h);
        fem::amg_setup(h);
    });
}

int fem_amg_sizes(fem_handle *h, int64_t *n_aggregates, int64_t *n_coarse_blocks) {
    return guarded([&] {
        require(h != nullptr && n_aggregates != nullptr && n_coarse_blocks != nullptr, "arguments must be non-NULL");
        require(h->amg != nullptr, "fem_amg_setup has not been called");
        *n_aggregates = h->amg->na;
        *n_coarse_blocks = h->amg->nbc;
    });
}

int fem_amg_export(fem_handle *h, int32_t *agg, double *P, int64_t *coarse_ptr, int32_t *coarse_col) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        require(h->amg != nullptr, "fem_amg_setup has not been called");
        bind_device(h);
        const fem::Amg &a = *h->amg;
        const int64_t Nn = h->g.Nn;
        if (agg && Nn) FEM_HIP(hipMemcpy(agg, a.agg, Nn * sizeof(int32_t), hipMemcpyDeviceToDevice));
        if (P && Nn)
            FEM_HIP(hipMemcpy(P, a.P64, size_t(Nn) * h->g.nd * a.nc * sizeof(double), hipMemcpyDeviceToDevice));
        if (coarse_ptr) FEM_HIP(hipMemcpy(coarse_ptr, a.cptr, (a.na + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice));
        if (coarse_col && a.nbc)
            FEM_HIP(hipMemcpy(coarse_col, a.ccol, a.nbc * sizeof(int32_t), hipMemcpyDeviceToDevice));
    });
}

int fem_amg_apply(fem_handle *h, const double *u, const double *theta, const double *r, double *z,
                  const fem_solve_opts *opts, double *lmax_out, double *coarse_values, void *workspace,
                  size_t workspace_bytes, void *stream) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        validate_opts(opts);
        require(opts->precond == FEM_PRECOND_AMG, "opts.precond must be FEM_PRECOND_AMG");
        if (h->g.N == 0) return;
        require(u && theta && r && z && r != z, "u, theta, r and z must be non-NULL (r and z distinct)");
        require_amg_ready(h, opts);
        check_workspace(h, opts, workspace, workspace_bytes);
        bind_device(h);
        fem::amg_apply_once(h, u, theta, r, z, *opts, lmax_out, coarse_values, workspace, workspace_bytes,
                            as_stream(stream));
    });
}

int fem_param_vjp(fem_handle *h, const double *u, const double *theta, const double *lambda, double *vjp_theta,
                  void *stream) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        require(h->mat.model != FEM_J2_PLASTIC, "the parameter VJP is not defined for FEM_J2_PLASTIC");
        if (h->g.Ne == 0) return;
        require(u && theta && lambda && vjp_theta, "u, theta, lambda and vjp_theta must be non-NULL");
        bind_device(h);
        fem::reset_status(h, as_stream(stream));
        fem::launch_vjp(h, u, theta, lambda, vjp_theta, as_stream(stream));
        fem::check_status(h, as_stream(stream));
    });
}

int fem_element_volumes(fem_handle *h, double *volumes, int32_t normalized, void *stream) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        if (h->g.Ne == 0) return;
        require(volumes != nullptr, "volumes must be non-NULL");
        bind_device(h);
        fem::element_volumes(h, volumes, normalized != 0, as_stream(stream));
    });
}

int fem_filter_setup(fem_handle *h, double rmin) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        require(rmin > 0.0 && std::isfinite(rmin), "rmin must be positive");
        bind_device(h);
        fem::filter_setup(h, rmin);
    });
}

int fem_filter_apply(fem_handle *h, int32_t mode, const double *theta, const double *x, double *out, void *stream) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        require(mode == FEM_FILTER_DENSITY || mode == FEM_FILTER_SENSITIVITY, "mode");
        require(h->filter.ready, "fem_filter_setup has not been called");
        if (h->g.Ne == 0) return;
        require(x && out, "x and out must be non-NULL");
        require(x != out, "x and out must be distinct buffers");
        require(mode == FEM_FILTER_DENSITY || theta != nullptr, "the sensitivity filter needs theta");
        bind_device(h);
        fem::filter_apply(h, mode, theta, x, out, as_stream(stream));
    });
}

size_t fem_vector_workspace_bytes(int64_t n) { return fem::vector_workspace_bytes(n < 0 ? 0 : n); }

int fem_dot(const double *a, const double *b, int64_t n, double *result, void *workspace, size_t workspace_bytes,
            void *stream) {
    return guarded([&] {
        require(result != nullptr, "result is NULL");
        require(n >= 0, "n must be >= 0");
        *result = 0.0;
        if (n == 0) return;
        require(a && b, "a and b must be non-NULL");
        require(workspace && workspace_bytes >= fem::vector_workspace_bytes(n), "workspace too small");
        *result = fem::dot(a, b, n, workspace, as_stream(stream));
    });
}

int fem_mma_default_opts(fem_mma_opts *o) {
    return guarded([&] {
        require(o != nullptr, "opts is NULL");
        std::memset(o, 0, sizeof(*o));
        o->xmin = 0.0;
        o->xmax = 1.0;
        o->move = 0.5;
        o->asy_init = 0.5;
        o->asy_decr = 0.7;
        o->asy_incr = 1.2;
        o->albefa = 0.1;
        o->raa0 = 1e-5;
        o->bisect_iters = 100;
    });
}

int fem_mma_update(int64_t n, int32_t iter, const double *x, const double *xold1, const double *xold2,
                   const double *df0, double f1, const double *df1, double *low, double *upp, double *xnew,
                   double *lambda_out, const fem_mma_opts *opts, void *workspace, size_t workspace_bytes,
                   void *stream) {
    return guarded([&] {
        require(opts != nullptr, "opts is NULL");
        require(n >= 0 && iter >= 0, "n and iter must be >= 0");
        require(opts->xmax > opts->xmin && opts->move > 0.0 && opts->asy_init > 0.0 && opts->asy_decr > 0.0 &&
                    opts->asy_incr > 0.0 && opts->albefa > 0.0 && opts->albefa < 1.0 && opts->raa0 >= 0.0 &&
                    opts->bisect_iters >= 0,
                "mma opts");
        require(std::isfinite(f1), "f1 is not finite");
        if (lambda_out) *lambda_out = 0.0;
        if (n == 0) return;
        require(x && xold1 && xold2 && df0 && df1 && low && upp && xnew, "vector arguments must be non-NULL");
        require(workspace && workspace_bytes >= fem::vector_workspace_bytes(n), "workspace too small");
        const double lam = fem::mma_update(n, iter, x, xold1, xold2, df0, f1, df1, low, upp, xnew, *opts, workspace,
                                           as_stream(stream));
        if (lambda_out) *lambda_out = lam;
    });
}

int fem_mass_apply(fem_handle *h, const double *x, double *y, void *workspace, size_t workspace_bytes, void *stream) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        if (h->g.N == 0) return;
        require(x && y && x != y, "x and y must be distinct non-NULL buffers");
        check_workspace(h, nullptr, workspace, workspace_bytes);
        bind_device(h);
        void *ke;
        double *rscr;
        fem::carve_assemble(h, workspace, workspace_bytes, &ke, &rscr, FEM_F64);
        fem::reset_status(h, as_stream(stream));
        fem::launch_mass(h, x, rscr, y, as_stream(stream));
        fem::check_status(h, as_stream(stream));
    });
}

int fem_set_load(fem_handle *h, const double *f_ext, void *stream) {
    return guarded([&] {
        require(h != nullptr, "handle is NULL");
        if (h->g.N == 0) return;
        require(f_ext != nullptr, "f_ext must be non-NULL");
        bind_device(h);
        fem::set_load(h, f_ext, as_stream(stream));
    });
}

int fem_axpby(int64_t n, double a, const double *x, double b, double *y, void *stream) {
    return guarded([&] {
        require(n >= 0, "n must be >= 0");
        if (n == 0) return;
        require(x && y, "x and y must be non-NULL");
        fem::axpby(n, a, x, b, y, as_stream(stream));
    });
}

int fem_obs_misfit(int64_t n, int64_t n_obs, const int64_t *idx, const double *obs, const double *u, double *dJdu,
                   double *J, void *workspace, size_t workspace_bytes, void *stream) {
    return guarded([&] {
        require(J != nullptr, "J is NULL");
        require(n >= 0 && n_obs >= 0, "sizes must be >= 0");
        *J = 0.0;
        require(u && dJdu && (n_obs == 0 || (idx && obs)), "vector arguments must be non-NULL");
        require(workspace && workspace_bytes >= fem::vector_workspace_bytes(n_obs), "workspace too small");
        *J = fem::obs_misfit(n, n_obs, idx, obs, u, dJdu, workspace, as_stream(stream));
    });
}

}  // extern "C"

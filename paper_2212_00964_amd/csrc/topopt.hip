// SIMP compliance optimisation around the gradient (Sec. 3.2): element volumes, the
// convolution filter over element centroids, a deterministic FP64 dot product and
// the method of moving asymptotes (Svanberg 1987) for one constraint.
//
// All reductions use a fixed grid; the per-block partials are summed on the host in
// block order, so results are bit-reproducible.  The MMA dual (one multiplier) is
// solved on the host by doubling and bisection, one reduction kernel per step.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"
#include "solver.h"

namespace fem {

namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n) { return unsigned(std::max<int64_t>(1, (n + kThreads - 1) / kThreads)); }

__device__ void block_partial(double v, double *partials) {
    __shared__ double red[kThreads / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kThreads / 64; ++k) t += red[k];
        partials[blockIdx.x] = t;
    }
}

// ------------------------------------------------------------------ element volumes
// v_e = sum over the 2x2x2 Gauss points (weights 1) of det J; HEX8 node a sits at
// reference corner (x, y, z) = ((a ^ (a >> 1)) & 1, (a >> 1) & 1, (a >> 2) & 1).
__global__ __launch_bounds__(kThreads) void k_element_volumes(int64_t Ne, const double *__restrict__ coords,
                                                             const int32_t *__restrict__ conn,
                                                             double *__restrict__ vol) {
    const int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (e >= Ne) return;
    double X[8][3];
    for (int a = 0; a < 8; ++a)
        for (int i = 0; i < 3; ++i) X[a][i] = coords[3 * int64_t(conn[8 * e + a]) + i];
    const double gq = 0.57735026918962576451;
    double v = 0.0;
    for (int q = 0; q < 8; ++q) {
        const double xi[3] = {(q & 1) ? gq : -gq, (q & 2) ? gq : -gq, (q & 4) ? gq : -gq};
        double J[3][3] = {};
        for (int a = 0; a < 8; ++a) {
            const int bits[3] = {(a ^ (a >> 1)) & 1, (a >> 1) & 1, (a >> 2) & 1};
            double s[3], l[3];
            for (int j = 0; j < 3; ++j) {
                s[j] = bits[j] ? 1.0 : -1.0;
                l[j] = 0.5 * (1.0 + s[j] * xi[j]);
            }
            const double dN[3] = {0.5 * s[0] * l[1] * l[2], 0.5 * s[1] * l[0] * l[2], 0.5 * s[2] * l[0] * l[1]};
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) J[i][j] += X[a][i] * dN[j];
        }
        v += J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
             J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    }
    vol[e] = v;
}

// ------------------------------------------------------------------ filter
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_filter(int64_t Ne, const int64_t *__restrict__ ptr,
                                                    const int32_t *__restrict__ idx, const double *__restrict__ w,
                                                    const double *__restrict__ wsum, const double *__restrict__ theta,
                                                    const double *__restrict__ x, double *__restrict__ out) {
    const int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (e >= Ne) return;
    double s = 0.0;
    for (int64_t k = ptr[e]; k < ptr[e + 1]; ++k) {
        const int64_t f = idx[k];
        s += (MODE == FEM_FILTER_SENSITIVITY) ? w[k] * theta[f] * x[f] : w[k] * x[f];
    }
    out[e] = (MODE == FEM_FILTER_SENSITIVITY) ? s / (fmax(1e-3, theta[e]) * wsum[e]) : s / wsum[e];
}

// ------------------------------------------------------------------ dot
__global__ __launch_bounds__(kThreads) void k_dot(int64_t n, const double *__restrict__ a,
                                                 const double *__restrict__ b, double *partials) {
    double d = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += int64_t(gridDim.x) * kThreads)
        d += a[i] * b[i];
    block_partial(d, partials);
}

__global__ __launch_bounds__(kThreads) void k_sum(int64_t n, const double *__restrict__ a, double *partials) {
    double d = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += int64_t(gridDim.x) * kThreads)
        d += a[i];
    block_partial(d, partials);
}

__global__ __launch_bounds__(kThreads) void k_scale(int64_t n, double c, double *__restrict__ a) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) a[i] *= c;
}

__global__ __launch_bounds__(kThreads) void k_axpby(int64_t n, double a, const double *__restrict__ x, double b,
                                                   double *__restrict__ y) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) y[i] = (b == 0.0) ? a * x[i] : a * x[i] + b * y[i];
}

__global__ __launch_bounds__(kThreads) void k_fill(int64_t n, double v, double *__restrict__ y) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) y[i] = v;
}

// Misfit at observed dofs: r_k = u[idx_k] - obs_k; dJdu[idx_k] = 2 r_k (dJdu zeroed
// before); partials of sum r_k^2.  The observed indices are distinct.
__global__ __launch_bounds__(kThreads) void k_obs_misfit(int64_t n_obs, const int64_t *__restrict__ idx,
                                                        const double *__restrict__ obs, const double *__restrict__ u,
                                                        double *__restrict__ dJdu, double *partials) {
    double acc = 0.0;
    for (int64_t k = int64_t(blockIdx.x) * kThreads + threadIdx.x; k < n_obs; k += int64_t(gridDim.x) * kThreads) {
        const double r = u[idx[k]] - obs[k];
        dJdu[idx[k]] = 2.0 * r;
        acc += r * r;
    }
    block_partial(acc, partials);
}

// sum of squares over the dofs that are not Dirichlet dofs (mask may be null)
__global__ __launch_bounds__(kThreads) void k_sumsq_free(int64_t n, const double *__restrict__ a,
                                                        const uint8_t *__restrict__ mask, double *partials) {
    double d = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += int64_t(gridDim.x) * kThreads)
        if (!(mask && mask[i])) d += a[i] * a[i];
    block_partial(d, partials);
}

// ------------------------------------------------------------------ MMA
struct MmaArrays {
    double *alpha, *beta, *p0, *q0, *p1, *q1;
};

// Asymptotes, move limits and the coefficients of the convex approximations of f0
// and f1 at x; partials of sum_j (p1_j / (U_j - x_j) + q1_j / (x_j - L_j)).
__global__ __launch_bounds__(kThreads) void k_mma_prep(int64_t n, int iter, const double *__restrict__ x,
                                                      const double *__restrict__ xold1,
                                                      const double *__restrict__ xold2,
                                                      const double *__restrict__ df0, const double *__restrict__ df1,
                                                      double *__restrict__ low, double *__restrict__ upp,
                                                      fem_mma_opts o, MmaArrays A, double *partials) {
    const double box = o.xmax - o.xmin;
    double acc = 0.0;
    for (int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x; j < n; j += int64_t(gridDim.x) * kThreads) {
        const double xj = x[j];
        double L, U;
        if (iter < 2) {
            L = xj - o.asy_init * box;
            U = xj + o.asy_init * box;
        } else {
            const double osc = (xj - xold1[j]) * (xold1[j] - xold2[j]);
            const double f = osc > 0.0 ? o.asy_incr : (osc < 0.0 ? o.asy_decr : 1.0);
            L = xj - f * (xold1[j] - low[j]);
            U = xj + f * (upp[j] - xold1[j]);
            L = fmin(fmax(L, xj - 10.0 * box), xj - 0.01 * box);
            U = fmin(fmax(U, xj + 0.01 * box), xj + 10.0 * box);
        }
        low[j] = L;
        upp[j] = U;
        A.alpha[j] = fmax(fmax(o.xmin, L + o.albefa * (xj - L)), xj - o.move * box);
        A.beta[j] = fmin(fmin(o.xmax, U - o.albefa * (U - xj)), xj + o.move * box);
        const double ux2 = (U - xj) * (U - xj), xl2 = (xj - L) * (xj - L), reg = o.raa0 / box;
        const double g0p = fmax(df0[j], 0.0), g0m = fmax(-df0[j], 0.0);
        const double g1p = fmax(df1[j], 0.0), g1m = fmax(-df1[j], 0.0);
        A.p0[j] = ux2 * (1.001 * g0p + 0.001 * g0m + reg);
        A.q0[j] = xl2 * (0.001 * g0p + 1.001 * g0m + reg);
        const double p1 = ux2 * (1.001 * g1p + 0.001 * g1m + reg);
        const double q1 = xl2 * (0.001 * g1p + 1.001 * g1m + reg);
        A.p1[j] = p1;
        A.q1[j] = q1;
        acc += p1 / (U - xj) + q1 / (xj - L);
    }
    block_partial(acc, partials);
}

// Minimiser of the Lagrangian approximation for multiplier lam, clamped to the move limits.
__device__ __forceinline__ double mma_x(int64_t j, double lam, const double *low, const double *upp,
                                        const MmaArrays &A) {
    const double P = A.p0[j] + lam * A.p1[j], Q = A.q0[j] + lam * A.q1[j];
    const double sp = sqrt(P), sq = sqrt(Q);
    const double xv = (low[j] * sp + upp[j] * sq) / (sp + sq);
    return fmin(fmax(xv, A.alpha[j]), A.beta[j]);
}

__global__ __launch_bounds__(kThreads) void k_mma_eval(int64_t n, double lam, const double *__restrict__ low,
                                                      const double *__restrict__ upp, MmaArrays A,
                                                      double *partials) {
    double acc = 0.0;
    for (int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x; j < n; j += int64_t(gridDim.x) * kThreads) {
        const double xj = mma_x(j, lam, low, upp, A);
        acc += A.p1[j] / (upp[j] - xj) + A.q1[j] / (xj - low[j]);
    }
    block_partial(acc, partials);
}

__global__ __launch_bounds__(kThreads) void k_mma_final(int64_t n, double lam, const double *__restrict__ low,
                                                       const double *__restrict__ upp, MmaArrays A,
                                                       double *__restrict__ xnew) {
    const int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (j < n) xnew[j] = mma_x(j, lam, low, upp, A);
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

double host_sum(const double *partials_dev, double *pinned, hipStream_t s) {
    FEM_HIP(hipMemcpyAsync(pinned, partials_dev, kRedGrid * sizeof(double), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    double t = 0.0;
    for (int b = 0; b < kRedGrid; ++b) t += pinned[b];
    return t;
}

// Host read-back slots for the partials, one array per host thread (ordinary host
// memory: the calls that read partials back allocate nothing).
double *readback_partials() {
    static thread_local double p[kRedGrid];
    return p;
}

}  // namespace

size_t vector_workspace_bytes(int64_t n) { return 6 * align256(size_t(n) * sizeof(double)) + align256(kRedGrid * sizeof(double)); }

void element_volumes(fem_handle *h, double *vol, bool normalized, hipStream_t s) {
    if (h->g.Ne == 0) return;
    hipLaunchKernelGGL(k_element_volumes, dim3(grid_for(h->g.Ne)), dim3(kThreads), 0, s, h->g.Ne, h->m.coords,
                       h->m.conn, vol);
    FEM_HIP(hipGetLastError());
    if (!normalized) return;
    // total by the deterministic reduction, then v_e / total
    hipLaunchKernelGGL(k_sum, dim3(kRedGrid), dim3(kThreads), 0, s, h->g.Ne, vol, h->red_partials);
    FEM_HIP(hipGetLastError());
    const double total = host_sum(h->red_partials, readback_partials(), s);
    hipLaunchKernelGGL(k_scale, dim3(grid_for(h->g.Ne)), dim3(kThreads), 0, s, h->g.Ne, 1.0 / total, vol);
    FEM_HIP(hipGetLastError());
    FEM_HIP(hipStreamSynchronize(s));
}

void filter_setup(fem_handle *h, double rmin) {
    const int64_t Ne = h->g.Ne, Nn = h->g.Nn;
    Filter &F = h->filter;
    for (void *p : F.allocations) (void)hipFree(p);
    F = Filter{};
    std::vector<double> xyz(3 * Nn);
    std::vector<int32_t> conn(8 * Ne);
    if (Nn) FEM_HIP(hipMemcpy(xyz.data(), h->m.coords, xyz.size() * sizeof(double), hipMemcpyDeviceToHost));
    if (Ne) FEM_HIP(hipMemcpy(conn.data(), h->m.conn, conn.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<double> c(3 * Ne, 0.0);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t e = 0; e < Ne; ++e) {
        for (int a = 0; a < 8; ++a)
            for (int i = 0; i < 3; ++i) c[3 * e + i] += xyz[3 * int64_t(conn[8 * e + a]) + i];
        for (int i = 0; i < 3; ++i) {
            c[3 * e + i] /= 8.0;
            lo[i] = std::min(lo[i], c[3 * e + i]);
            hi[i] = std::max(hi[i], c[3 * e + i]);
        }
    }
    // uniform grid of cells of size rmin: neighbours within rmin lie in the 27 cells around
    int64_t nc[3];
    for (int i = 0; i < 3; ++i) nc[i] = Ne ? std::max<int64_t>(1, int64_t((hi[i] - lo[i]) / rmin) + 1) : 1;
    auto cell_of = [&](int64_t e, int i) {
        return std::min<int64_t>(nc[i] - 1, int64_t((c[3 * e + i] - lo[i]) / rmin));
    };
    const int64_t ncell = nc[0] * nc[1] * nc[2];
    std::vector<int64_t> cptr(ncell + 1, 0);
    std::vector<int64_t> ecell(Ne);
    for (int64_t e = 0; e < Ne; ++e) {
        ecell[e] = cell_of(e, 0) + nc[0] * (cell_of(e, 1) + nc[1] * cell_of(e, 2));
        cptr[ecell[e] + 1]++;
    }
    for (int64_t k = 0; k < ncell; ++k) cptr[k + 1] += cptr[k];
    std::vector<int32_t> cell_elems(Ne);
    {
        std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
        for (int64_t e = 0; e < Ne; ++e) cell_elems[fill[ecell[e]]++] = int32_t(e);
    }
    std::vector<int64_t> ptr(Ne + 1, 0);
    std::vector<int32_t> idx;
    std::vector<double> w, wsum(Ne, 0.0);
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t e = 0; e < Ne; ++e) {
        row.clear();
        const int64_t ce[3] = {cell_of(e, 0), cell_of(e, 1), cell_of(e, 2)};
        for (int64_t dz = -1; dz <= 1; ++dz)
            for (int64_t dy = -1; dy <= 1; ++dy)
                for (int64_t dx = -1; dx <= 1; ++dx) {
                    const int64_t cx = ce[0] + dx, cy = ce[1] + dy, cz = ce[2] + dz;
                    if (cx < 0 || cy < 0 || cz < 0 || cx >= nc[0] || cy >= nc[1] || cz >= nc[2]) continue;
                    const int64_t cell = cx + nc[0] * (cy + nc[1] * cz);
                    for (int64_t k = cptr[cell]; k < cptr[cell + 1]; ++k) {
                        const int32_t f = cell_elems[k];
                        const double d0 = c[3 * e] - c[3 * int64_t(f)], d1 = c[3 * e + 1] - c[3 * int64_t(f) + 1],
                                     d2 = c[3 * e + 2] - c[3 * int64_t(f) + 2];
                        const double wt = rmin - std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                        if (wt > 0.0) row.push_back({f, wt});
                    }
                }
        std::sort(row.begin(), row.end());
        for (auto &pw : row) {
            idx.push_back(pw.first);
            w.push_back(pw.second);
            wsum[e] += pw.second;
        }
        ptr[e + 1] = int64_t(idx.size());
    }
    auto up = [&](const auto &v) {
        using T = typename std::decay_t<decltype(v)>::value_type;
        T *p = nullptr;
        FEM_HIP(hipMalloc(reinterpret_cast<void **>(&p), std::max<size_t>(256, v.size() * sizeof(T))));
        F.allocations.push_back(p);
        if (!v.empty()) FEM_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
        return p;
    };
    F.ptr = up(ptr);
    F.idx = up(idx);
    F.w = up(w);
    F.wsum = up(wsum);
    F.nnz = int64_t(idx.size());
    F.ready = true;
}

void filter_apply(const fem_handle *h, int mode, const double *theta, const double *x, double *out, hipStream_t s) {
    const Filter &F = h->filter;
    if (h->g.Ne == 0) return;
    if (mode == FEM_FILTER_SENSITIVITY)
        hipLaunchKernelGGL(k_filter<FEM_FILTER_SENSITIVITY>, dim3(grid_for(h->g.Ne)), dim3(kThreads), 0, s, h->g.Ne,
                           F.ptr, F.idx, F.w, F.wsum, theta, x, out);
    else
        hipLaunchKernelGGL(k_filter<FEM_FILTER_DENSITY>, dim3(grid_for(h->g.Ne)), dim3(kThreads), 0, s, h->g.Ne, F.ptr,
                           F.idx, F.w, F.wsum, theta, x, out);
    FEM_HIP(hipGetLastError());
}

double dot(const double *a, const double *b, int64_t n, void *ws, hipStream_t s) {
    double *partials = static_cast<double *>(ws);
    hipLaunchKernelGGL(k_dot, dim3(kRedGrid), dim3(kThreads), 0, s, n, a, b, partials);
    FEM_HIP(hipGetLastError());
    return host_sum(partials, readback_partials(), s);
}

void axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(kThreads), 0, s, n, a, x, b, y);
    FEM_HIP(hipGetLastError());
}

double obs_misfit(int64_t n, int64_t n_obs, const int64_t *idx, const double *obs, const double *u, double *dJdu,
                  void *ws, hipStream_t s) {
    double *partials = static_cast<double *>(ws);
    if (n) hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kThreads), 0, s, n, 0.0, dJdu);
    hipLaunchKernelGGL(k_obs_misfit, dim3(kRedGrid), dim3(kThreads), 0, s, n_obs, idx, obs, u, dJdu, partials);
    FEM_HIP(hipGetLastError());
    return host_sum(partials, readback_partials(), s);
}

void set_load(fem_handle *h, const double *f, hipStream_t s) {
    const int64_t N = h->g.N;
    if (N == 0) return;
    FEM_HIP(hipMemcpyAsync(h->m.fext, f, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_sumsq_free, dim3(kRedGrid), dim3(kThreads), 0, s, N, h->m.fext, h->m.mask, h->red_partials);
    FEM_HIP(hipGetLastError());
    h->m.fext_norm = std::sqrt(host_sum(h->red_partials, readback_partials(), s));
}

double mma_update(int64_t n, int iter, const double *x, const double *xold1, const double *xold2, const double *df0,
                  double f1, const double *df1, double *low, double *upp, double *xnew, const fem_mma_opts &o,
                  void *ws, hipStream_t s) {
    char *base = static_cast<char *>(ws);
    const size_t vb = align256(size_t(n) * sizeof(double));
    MmaArrays A{reinterpret_cast<double *>(base), reinterpret_cast<double *>(base + vb),
                reinterpret_cast<double *>(base + 2 * vb), reinterpret_cast<double *>(base + 3 * vb),
                reinterpret_cast<double *>(base + 4 * vb), reinterpret_cast<double *>(base + 5 * vb)};
    double *partials = reinterpret_cast<double *>(base + 6 * vb);
    double *pin = readback_partials();
    hipLaunchKernelGGL(k_mma_prep, dim3(kRedGrid), dim3(kThreads), 0, s, n, iter, x, xold1, xold2, df0, df1, low, upp,
                       o, A, partials);
    FEM_HIP(hipGetLastError());
    const double r1 = f1 - host_sum(partials, pin, s);
    auto g = [&](double lam) {
        hipLaunchKernelGGL(k_mma_eval, dim3(kRedGrid), dim3(kThreads), 0, s, n, lam, low, upp, A, partials);
        FEM_HIP(hipGetLastError());
        return r1 + host_sum(partials, pin, s);
    };
    // Dual in the multiplier: doubling until the approximated constraint is met, then
    // bisection.  If it cannot be met inside the move limits (2^200 reached), the step
    // takes that multiplier: the point of the move box minimising the approximation.
    constexpr int kMaxDoublings = 200;
    double lam = 0.0;
    if (g(0.0) > 0.0) {
        double lo = 0.0, hi = 1.0;
        for (int k = 0; k < kMaxDoublings && g(hi) > 0.0; ++k) {
            lo = hi;
            hi *= 2.0;
        }
        if (g(hi) > 0.0) {
            lam = hi;
        } else {
            for (int k = 0; k < o.bisect_iters; ++k) {
                const double mid = 0.5 * (lo + hi);
                if (g(mid) > 0.0) lo = mid;
                else hi = mid;
            }
            lam = 0.5 * (lo + hi);
        }
    }
    hipLaunchKernelGGL(k_mma_final, dim3(grid_for(n)), dim3(kThreads), 0, s, n, lam, low, upp, A, xnew);
    FEM_HIP(hipGetLastError());
    FEM_HIP(hipStreamSynchronize(s));
    return lam;
}

}  // namespace fem

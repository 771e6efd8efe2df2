// Two-level aggregation preconditioner for the Krylov solves (FEM_PRECOND_AMG).
//
// The paper names the Jacobi-preconditioned linear solver as the bottleneck of its
// method (Sec. 5, item 2).  This preconditioner keeps the Jacobi-scaled tangent as
// the smoother and adds a coarse space:
//   * aggregates of the node graph (host, once per handle): in node order, a node
//     whose whole neighbourhood is still free founds an aggregate of exactly that
//     neighbourhood; leftover nodes join the aggregate of their first aggregated
//     neighbour (ascending), or found a singleton;
//   * per aggregate the 6 rigid-body modes (3 translations, rotations (-y, x, 0),
//     (0, -z, y), (z, 0, -x) about the node centroid; the constant when ndpn = 1),
//     Dirichlet dofs zeroed, orthonormalised by modified Gram-Schmidt in that order
//     (a column below 1e-10 of its original norm is dropped);
//   * the Galerkin coarse operator A_c = P^T A P from the assembled values (one wave
//     per coarse block, summing its fine blocks in ascending order, so the result is
//     deterministic), with a unit diagonal for dropped columns;
//   * Chebyshev iteration (Saad, Iterative Methods for Sparse Linear Systems, Alg.
//     12.1) on the interval [lmax / 30, lmax] of the Jacobi-scaled operator; on the
//     fine level lmax is the Gershgorin bound (the power estimate fell below the top of
//     the spectrum of some tangents, and an interval that misses it makes M indefinite),
//     on the coarse level min(1.2 x a 12-step power estimate from x_i = sin(1 + i), the
//     Gershgorin bound) (the coarse polynomial's higher degree pays for a tight end);
//   * one application z = M r: Chebyshev smoothing from 0, restriction of the residual,
//     Chebyshev steps on A_c from 0, prolongation, Chebyshev smoothing continued from
//     z.  Equal pre- and post-smoothers make M symmetric, so plain CG applies.
// Everything after the host setup runs in the solve precision T.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "lanes.h"

namespace fem {

namespace {

constexpr int kThreads = 256;
constexpr int kWavesPerBlock = kThreads / 64;
constexpr int kPowerSteps = 12;
constexpr double kLmaxSafety = 1.2;
constexpr double kChebRatio = 30.0;
constexpr double kDropTol = 1e-10;

inline unsigned grid_for(int64_t n, int per) { return unsigned(std::max<int64_t>(1, (n + per - 1) / per)); }

__device__ __forceinline__ bool halted(const KrylovScalars *sc) {
    return sc != nullptr && (sc->converged | sc->breakdown);
}

// Sum over the 64 lanes of a wavefront; every lane receives it (fixed order).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    v = lane_sum16(v);
    v += swap_rows(v, v, (threadIdx.x & 31) >= 16);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// Sum over the 32-lane half of a wavefront holding this lane; every lane receives it.
template <typename T>
__device__ __forceinline__ T half_sum(T v) {
    v = lane_sum16(v);
    v += swap_rows(v, v, (threadIdx.x & 31) >= 16);
    return v;
}

// ------------------------------------------------------------------ coarse operator
// One 32-lane group per coarse block c = (I, J): sum over its fine blocks (i, j) of
// P_i^T A_ij P_j.
template <int ND, int NC, typename T>
__global__ __launch_bounds__(kThreads) void k_amg_coarse(int64_t nbc, const int64_t *__restrict__ cbp,
                                                         const int32_t *__restrict__ cbk,
                                                         const int32_t *__restrict__ crow,
                                                         const int32_t *__restrict__ ccol,
                                                         const uint8_t *__restrict__ dropped,
                                                         const int32_t *__restrict__ blk_row,
                                                         const int64_t *__restrict__ node_ptr,
                                                         const int32_t *__restrict__ node_nb,
                                                         const int64_t *__restrict__ row_ptr,
                                                         const T *__restrict__ values, const T *__restrict__ P,
                                                         T *__restrict__ cvals) {
    // one 32-lane group per coarse block (two per wavefront); a group past the end
    // recomputes the last block and stores nothing, so every lane stays active
    const int64_t c_raw = int64_t(blockIdx.x) * (kThreads / 32) + (threadIdx.x >> 5);
    const bool valid = c_raw < nbc;
    const int64_t c = valid ? c_raw : nbc - 1;
    const int lane = threadIdx.x & 31;
    T acc[NC][NC];
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int l = 0; l < NC; ++l) acc[k][l] = T(0);
    for (int64_t q = cbp[c] + lane; q < cbp[c + 1]; q += 32) {
        const int64_t kb = cbk[q];
        const int64_t i = blk_row[kb], j = node_nb[kb];
        const int64_t pos = kb - node_ptr[i];
        const T *Pi = P + i * ND * NC, *Pj = P + j * ND * NC;
        T t[ND][NC];
#pragma unroll
        for (int r = 0; r < ND; ++r) {
            T a[ND];
#pragma unroll
            for (int cc = 0; cc < ND; ++cc) a[cc] = values[row_ptr[ND * i + r] + ND * pos + cc];
#pragma unroll
            for (int l = 0; l < NC; ++l) {
                T v = T(0);
#pragma unroll
                for (int cc = 0; cc < ND; ++cc) v += a[cc] * Pj[cc * NC + l];
                t[r][l] = v;
            }
        }
#pragma unroll
        for (int k = 0; k < NC; ++k)
#pragma unroll
            for (int l = 0; l < NC; ++l) {
                T v = T(0);
#pragma unroll
                for (int r = 0; r < ND; ++r) v += Pi[r * NC + k] * t[r][l];
                acc[k][l] += v;
            }
    }
    const bool diag = crow[c] == ccol[c];
    const unsigned dmask = diag ? dropped[crow[c]] : 0u;
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int l = 0; l < NC; ++l) {
            T v = half_sum(acc[k][l]);
            if (k == l && ((dmask >> k) & 1u)) v = T(1);
            if (valid && lane == 0) cvals[(c * NC + k) * NC + l] = v;
        }
}

// Inverse diagonal of the coarse operator.
template <int NC, typename T>
__global__ __launch_bounds__(kThreads) void k_amg_cdinv(int64_t na, const int64_t *__restrict__ cdiag,
                                                        const T *__restrict__ cvals, T *__restrict__ cdinv) {
    const int64_t t = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (t >= na * NC) return;
    const int64_t I = t / NC;
    const int k = int(t - I * NC);
    cdinv[t] = T(1) / cvals[(cdiag[I] * NC + k) * NC + k];
}

// y = alpha A_c x, one thread per coarse row (I, k).
template <int NC, typename T>
__global__ __launch_bounds__(kThreads) void k_amg_cspmv(int64_t na, const int64_t *__restrict__ cptr,
                                                        const int32_t *__restrict__ ccol,
                                                        const T *__restrict__ cvals, const T *__restrict__ x,
                                                        T *__restrict__ y, T alpha, const KrylovScalars *sc) {
    if (halted(sc)) return;
    const int64_t t = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (t >= na * NC) return;
    const int64_t I = t / NC;
    const int k = int(t - I * NC);
    T s = T(0);
    for (int64_t b = cptr[I]; b < cptr[I + 1]; ++b) {
        const T *row = cvals + (b * NC + k) * NC;
        const T *xj = x + int64_t(ccol[b]) * NC;
#pragma unroll
        for (int l = 0; l < NC; ++l) s += row[l] * xj[l];
    }
    y[t] = alpha * s;
}

// ------------------------------------------------------------------ grid transfers
// bc[I] = sum over the nodes i of aggregate I of P_i^T (r_i - w_i); one wavefront per
// aggregate.
template <int ND, int NC, typename T>
__global__ __launch_bounds__(kThreads) void k_amg_restrict(int64_t na, const int64_t *__restrict__ agg_ptr,
                                                           const int32_t *__restrict__ agg_nodes,
                                                           const T *__restrict__ P, const T *__restrict__ r,
                                                           const T *__restrict__ w, T *__restrict__ bc,
                                                           const KrylovScalars *sc) {
    if (halted(sc)) return;
    const int64_t I = int64_t(blockIdx.x) * kWavesPerBlock + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (I >= na) return;  // wave-uniform
    T acc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) acc[k] = T(0);
    for (int64_t q = agg_ptr[I] + lane; q < agg_ptr[I + 1]; q += 64) {
        const int64_t i = agg_nodes[q];
#pragma unroll
        for (int rr = 0; rr < ND; ++rr) {
            const T t = r[ND * i + rr] - w[ND * i + rr];
#pragma unroll
            for (int k = 0; k < NC; ++k) acc[k] += P[(i * ND + rr) * NC + k] * t;
        }
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const T v = wave_sum(acc[k]);
        if (lane == 0) bc[I * NC + k] = v;
    }
}

// z_i += P_i zc[agg(i)], one thread per node.
template <int ND, int NC, typename T>
__global__ __launch_bounds__(kThreads) void k_amg_prolong(int64_t Nn, const int32_t *__restrict__ agg,
                                                          const T *__restrict__ P, const T *__restrict__ zc,
                                                          T *__restrict__ z, const KrylovScalars *sc) {
    if (halted(sc)) return;
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= Nn) return;
    const T *e = zc + int64_t(agg[i]) * NC;
#pragma unroll
    for (int rr = 0; rr < ND; ++rr) {
        T v = T(0);
#pragma unroll
        for (int k = 0; k < NC; ++k) v += P[(i * ND + rr) * NC + k] * e[k];
        z[ND * i + rr] += v;
    }
}

// ------------------------------------------------------------------ Chebyshev steps
// Start: rc = r - w (w may be null: rc = r), d = dinv rc / theta, z = d or z += d.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cheb_start(int64_t n, const T *__restrict__ r, const T *__restrict__ w,
                                                         T *__restrict__ rc, T *__restrict__ d, T *__restrict__ z,
                                                         const T *__restrict__ dinv, T inv_theta, int cont,
                                                         const KrylovScalars *sc) {
    if (halted(sc)) return;
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    const T ri = w ? r[i] - w[i] : r[i];
    rc[i] = ri;
    const T di = dinv[i] * ri * inv_theta;
    d[i] = di;
    z[i] = cont ? z[i] + di : di;
}

// Step: rc -= w (w = A d), d = c1 d + c2 dinv rc, z += d.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cheb_step(int64_t n, const T *__restrict__ w, T *__restrict__ rc,
                                                        T *__restrict__ d, T *__restrict__ z,
                                                        const T *__restrict__ dinv, T c1, T c2,
                                                        const KrylovScalars *sc) {
    if (halted(sc)) return;
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    const T ri = rc[i] - w[i];
    rc[i] = ri;
    const T di = c1 * d[i] + c2 * dinv[i] * ri;
    d[i] = di;
    z[i] += di;
}

// ------------------------------------------------------------------ spectrum bounds
// Block partials of max_i dinv_i sum_j |A_ij| (Gershgorin) over the fine rows: one
// 32-lane group per node (lane = neighbour block, the node's ND rows at once).
template <int ND, typename T>
__global__ __launch_bounds__(kThreads) void k_gersh_fine(int64_t Nn, const int64_t *__restrict__ node_ptr,
                                                         const T *__restrict__ values, const T *__restrict__ dinv,
                                                         double *partials) {
    __shared__ double red[kThreads / 32];
    const int lane = threadIdx.x & 31;
    const int64_t g0 = int64_t(blockIdx.x) * (kThreads / 32) + (threadIdx.x >> 5);
    const int64_t stride = int64_t(gridDim.x) * (kThreads / 32);
    double m = 0.0;
    for (int64_t n = g0; n < Nn; n += stride) {  // group-uniform loop
        const int64_t b0 = node_ptr[n];
        const int deg = int(node_ptr[n + 1] - b0);
        double sr[ND];
#pragma unroll
        for (int i = 0; i < ND; ++i) sr[i] = 0.0;
        for (int l = lane; l < deg; l += 32)
#pragma unroll
            for (int i = 0; i < ND; ++i)
#pragma unroll
                for (int k = 0; k < ND; ++k)
                    sr[i] += fabs(double(values[int64_t(ND) * ND * b0 + int64_t(i) * ND * deg + ND * l + k]));
#pragma unroll
        for (int i = 0; i < ND; ++i) m = fmax(m, half_sum(sr[i]) * fabs(double(dinv[ND * n + i])));
    }
    if (lane == 0) red[threadIdx.x >> 5] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kThreads / 32; ++k) t = fmax(t, red[k]);
        partials[blockIdx.x] = t;
    }
}

template <int NC, typename T>
__global__ __launch_bounds__(kThreads) void k_gersh_coarse(int64_t na, const int64_t *__restrict__ cptr,
                                                           const T *__restrict__ cvals, const T *__restrict__ cdinv,
                                                           double *partials) {
    __shared__ double red[kWavesPerBlock];
    double m = 0.0;
    for (int64_t t = int64_t(blockIdx.x) * kThreads + threadIdx.x; t < na * NC; t += int64_t(gridDim.x) * kThreads) {
        const int64_t I = t / NC;
        const int k = int(t - I * NC);
        double s = 0.0;
        for (int64_t b = cptr[I]; b < cptr[I + 1]; ++b)
#pragma unroll
            for (int l = 0; l < NC; ++l) s += fabs(double(cvals[(b * NC + k) * NC + l]));
        m = fmax(m, s * fabs(double(cdinv[t])));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kWavesPerBlock; ++k) t = fmax(t, red[k]);
        partials[blockIdx.x] = t;
    }
}

// x_i = sin(1 + i); block partials of sum x_i^2.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_power_start(int64_t n, T *__restrict__ x, double *partials) {
    __shared__ double red[kWavesPerBlock];
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += int64_t(gridDim.x) * kThreads) {
        const double v = sin(1.0 + double(i));
        x[i] = T(v);
        s += v * v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kWavesPerBlock; ++k) t += red[k];
        partials[blockIdx.x] = t;
    }
}

// y = dinv w (in place in w); block partials of sum y_i^2.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_power_scale(int64_t n, T *__restrict__ w, const T *__restrict__ dinv,
                                                          double *partials) {
    __shared__ double red[kWavesPerBlock];
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += int64_t(gridDim.x) * kThreads) {
        const T y = dinv[i] * w[i];
        w[i] = y;
        s += double(y) * double(y);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kWavesPerBlock; ++k) t += red[k];
        partials[blockIdx.x] = t;
    }
}

// ------------------------------------------------------------------ preconditioned CG pieces
// alpha = rho_pp[it & 1] / (p, q); x += alpha p; r -= alpha q.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_xr_plain(int64_t N, T *__restrict__ x, T *__restrict__ r,
                                                          const T *__restrict__ p, const T *__restrict__ q,
                                                          const double *__restrict__ pq_partials, int pq_count,
                                                          KrylovScalars *sc, int it) {
    if (halted(sc)) return;
    __shared__ double red[kWavesPerBlock];
    double t = 0.0;
    for (int b = threadIdx.x; b < pq_count; b += kThreads) t += pq_partials[b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    double pq = 0.0;
    for (int k = 0; k < kWavesPerBlock; ++k) pq += red[k];
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) sc->breakdown = 1;
        return;
    }
    const double alpha = sc->rho_pp[it & 1] / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->alpha = alpha;
    const T al = T(alpha);
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < N; i += int64_t(gridDim.x) * kThreads) {
        x[i] += al * p[i];
        r[i] -= al * q[i];
    }
}

// Block partials of (r, z) and (r, r), partials[b] and partials[G + b].
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dot_rz_rr(int64_t N, const T *__restrict__ r, const T *__restrict__ z,
                                                        double *partials, const KrylovScalars *sc) {
    if (halted(sc)) return;
    __shared__ double red[kWavesPerBlock][2];
    double a = 0.0, b = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < N; i += int64_t(gridDim.x) * kThreads) {
        const double ri = double(r[i]);
        a += ri * double(z[i]);
        b += ri * ri;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6][0] = a;
        red[threadIdx.x >> 6][1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
        for (int k = 0; k < kWavesPerBlock; ++k) {
            ta += red[k][0];
            tb += red[k][1];
        }
        partials[blockIdx.x] = ta;
        partials[gridDim.x + blockIdx.x] = tb;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_copy_vec(int64_t n, const T *__restrict__ a, T *__restrict__ b) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) b[i] = a[i];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_widen(int64_t n, const T *__restrict__ a, double *__restrict__ b) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) b[i] = double(a[i]);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_zero_vec(int64_t n, T *__restrict__ a) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) a[i] = T(0);
}

__global__ void k_fin_init_amg(int G, const double *__restrict__ partials, KrylovScalars *sc, double rtol) {
    if (threadIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (int k = 0; k < G; ++k) {
        a += partials[k];
        b += partials[G + k];
    }
    sc->rho = a;
    sc->rho_pp[0] = a;
    sc->rho_pp[1] = a;
    sc->rho_old = 1.0;
    sc->alpha = 1.0;
    sc->omega = 1.0;
    sc->beta = 0.0;
    sc->bnorm2 = b;
    sc->rnorm2 = b;
    sc->tol2 = rtol * rtol * b;
    sc->its = 0;
    sc->rh2 = b;
    sc->rmin2 = b;
    sc->restart_at = -1;
    sc->breakdown = (isfinite(a) && isfinite(b)) ? ((b > 0.0 && !(a > 0.0)) ? 1 : 0) : 2;
    sc->converged = (b == 0.0) ? 1 : 0;
}

double host_max(const double *partials_dev, int G, double *pinned, hipStream_t s) {
    FEM_HIP(hipMemcpyAsync(pinned, partials_dev, G * sizeof(double), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    double t = 0.0;
    for (int b = 0; b < G; ++b) t = std::max(t, pinned[b]);
    return t;
}

double host_sum(const double *partials_dev, int G, double *pinned, hipStream_t s) {
    FEM_HIP(hipMemcpyAsync(pinned, partials_dev, G * sizeof(double), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    double t = 0.0;
    for (int b = 0; b < G; ++b) t += pinned[b];
    return t;
}

// Chebyshev coefficients of the steps after the first: c1_k = rho_k rho_{k-1},
// c2_k = 2 rho_k / delta, rho_0 = delta / theta, rho_k = 1 / (2 theta / delta - rho_{k-1}).
struct Cheb {
    double inv_theta;
    std::vector<double> c1, c2;
};

Cheb chebyshev_coeffs(double lmax, int degree) {
    const double a = lmax / kChebRatio, b = lmax;
    const double theta = 0.5 * (b + a), delta = 0.5 * (b - a), sigma = theta / delta;
    Cheb c;
    c.inv_theta = 1.0 / theta;
    double rho = 1.0 / sigma;
    for (int k = 1; k < degree; ++k) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        c.c1.push_back(rn * rho);
        c.c2.push_back(2.0 * rn / delta);
        rho = rn;
    }
    return c;
}

template <typename T>
struct AmgView {
    T *w, *rc, *d;             // fine temporaries
    T *bc, *zc, *rcc, *dc, *wc;  // coarse temporaries
    T *P, *cvals, *cdinv;
};

template <typename T>
AmgView<T> view(const fem_handle *h) {
    const Amg &a = *h->amg;
    AmgView<T> v;
    T *f = static_cast<T *>(a.fine_tmp);
    const int64_t N = h->g.N, M = a.na * a.nc;
    v.w = f;
    v.rc = f + N;
    v.d = f + 2 * N;
    T *c = static_cast<T *>(a.coarse_tmp);
    v.bc = c;
    v.zc = c + M;
    v.rcc = c + 2 * M;
    v.dc = c + 3 * M;
    v.wc = c + 4 * M;
    if constexpr (sizeof(T) == 4) v.P = a.P32;
    else v.P = a.P64;
    v.cvals = static_cast<T *>(a.cvals);
    v.cdinv = static_cast<T *>(a.cdinv);
    return v;
}

template <typename T>
void coarse_spmv(const fem_handle *h, const T *x, T *y, T alpha, const KrylovScalars *sc, hipStream_t s) {
    const Amg &a = *h->amg;
    const unsigned G = grid_for(a.na * a.nc, kThreads);
    if (a.nc == 6)
        hipLaunchKernelGGL((k_amg_cspmv<6, T>), dim3(G), dim3(kThreads), 0, s, a.na, a.cptr, a.ccol,
                           static_cast<const T *>(a.cvals), x, y, alpha, sc);
    else
        hipLaunchKernelGGL((k_amg_cspmv<1, T>), dim3(G), dim3(kThreads), 0, s, a.na, a.cptr, a.ccol,
                           static_cast<const T *>(a.cvals), x, y, alpha, sc);
    FEM_HIP(hipGetLastError());
}

// `degree` Chebyshev steps on the operator applied by op(x, y) (y = A x), from z = 0
// (cont = 0, w unused) or continuing from z with w = A z already formed (cont = 1).
template <typename T, typename Op>
void chebyshev_run(int64_t n, const Cheb &c, Op op, const T *r, const T *dinv, T *z, T *w, T *rc, T *d, int cont,
                   const KrylovScalars *sc, hipStream_t s) {
    const unsigned G = grid_for(n, kThreads);
    hipLaunchKernelGGL((k_cheb_start<T>), dim3(G), dim3(kThreads), 0, s, n, r, cont ? w : nullptr, rc, d, z, dinv,
                       T(c.inv_theta), cont, sc);
    for (size_t k = 0; k < c.c1.size(); ++k) {
        op(d, w);
        hipLaunchKernelGGL((k_cheb_step<T>), dim3(G), dim3(kThreads), 0, s, n, w, rc, d, z, dinv, T(c.c1[k]),
                           T(c.c2[k]), sc);
    }
    FEM_HIP(hipGetLastError());
}

// Largest-eigenvalue bound of dinv A: min(1.2 x power estimate, Gershgorin bound g).
// The iterates are scaled by 1/g instead of being normalised (|y_k| stays between
// (1/30)^k and 1 of the start), so only the last two norms are read back:
// ||dinv A x_{K-1}|| / ||x_{K-1}|| = g ||y_K|| / ||y_{K-1}||.
template <typename T, typename Op>
double lmax_bound(fem_handle *h, int64_t n, Op op, const T *dinv, T *x, T *y, double gersh, hipStream_t s) {
    Amg &a = *h->amg;
    if (!(gersh > 0.0) || !std::isfinite(gersh)) throw Error(FEM_ENAN, "preconditioner spectrum bound failed");
    hipLaunchKernelGGL((k_power_start<T>), dim3(kRedGrid), dim3(kThreads), 0, s, n, x, a.red);
    for (int k = 0; k < kPowerSteps; ++k) {
        op(x, y, T(1.0 / gersh));
        hipLaunchKernelGGL((k_power_scale<T>), dim3(kRedGrid), dim3(kThreads), 0, s, n, y, dinv,
                           a.red + (k & 1) * kRedGrid);
        std::swap(x, y);
    }
    FEM_HIP(hipMemcpyAsync(a.host_red, a.red, 2 * kRedGrid * sizeof(double), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    double n_last = 0.0, n_prev = 0.0;
    const int last = (kPowerSteps - 1) & 1;
    for (int b = 0; b < kRedGrid; ++b) {
        n_last += a.host_red[last * kRedGrid + b];
        n_prev += a.host_red[(1 - last) * kRedGrid + b];
    }
    const double lam = gersh * std::sqrt(n_last / n_prev);
    if (!(lam > 0.0) || !std::isfinite(lam)) throw Error(FEM_ENAN, "preconditioner spectrum estimate failed");
    return std::min(kLmaxSafety * lam, gersh);
}

}  // namespace

// ------------------------------------------------------------------ host setup
void amg_setup(fem_handle *h) {
    if (h->amg) return;
    const Graph &g = h->g;
    const int nd = g.nd, nc = nd == 3 ? 6 : 1;
    const int64_t Nn = g.Nn, N = g.N, nnzb = g.nnzb;
    std::vector<int64_t> node_ptr(Nn + 1);
    std::vector<int32_t> node_nb(nnzb);
    std::vector<double> X(3 * Nn);
    std::vector<uint8_t> mask(N);
    FEM_HIP(hipMemcpy(node_ptr.data(), g.node_ptr, (Nn + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    if (nnzb) FEM_HIP(hipMemcpy(node_nb.data(), g.node_nb, nnzb * sizeof(int32_t), hipMemcpyDeviceToHost));
    FEM_HIP(hipMemcpy(X.data(), h->m.coords, 3 * Nn * sizeof(double), hipMemcpyDeviceToHost));
    FEM_HIP(hipMemcpy(mask.data(), h->m.mask, N, hipMemcpyDeviceToHost));
    // aggregation
    std::vector<int32_t> agg(Nn, -1);
    int32_t na = 0;
    for (int64_t i = 0; i < Nn; ++i) {
        if (agg[i] >= 0) continue;
        bool free = true;
        for (int64_t k = node_ptr[i]; k < node_ptr[i + 1] && free; ++k) free = agg[node_nb[k]] < 0;
        if (!free) continue;
        for (int64_t k = node_ptr[i]; k < node_ptr[i + 1]; ++k) agg[node_nb[k]] = na;
        ++na;
    }
    for (int64_t i = 0; i < Nn; ++i) {
        if (agg[i] >= 0) continue;
        int32_t owner = -1;
        for (int64_t k = node_ptr[i]; k < node_ptr[i + 1] && owner < 0; ++k) owner = agg[node_nb[k]];
        agg[i] = owner >= 0 ? owner : na++;
    }
    std::vector<int64_t> agg_ptr(na + 1, 0);
    for (int64_t i = 0; i < Nn; ++i) agg_ptr[agg[i] + 1]++;
    for (int32_t a = 0; a < na; ++a) agg_ptr[a + 1] += agg_ptr[a];
    std::vector<int32_t> agg_nodes(Nn);
    {
        std::vector<int64_t> fill(agg_ptr.begin(), agg_ptr.end() - 1);
        for (int64_t i = 0; i < Nn; ++i) agg_nodes[fill[agg[i]]++] = int32_t(i);
    }
    // prolongator: rigid-body modes per aggregate, modified Gram-Schmidt
    std::vector<double> P(size_t(Nn) * nd * nc, 0.0);
    std::vector<uint8_t> dropped(na, 0);
    for (int32_t a = 0; a < na; ++a) {
        const int64_t b0 = agg_ptr[a], m = agg_ptr[a + 1] - b0;
        double c[3] = {0, 0, 0};
        for (int64_t q = b0; q < b0 + m; ++q)
            for (int j = 0; j < 3; ++j) c[j] += X[3 * int64_t(agg_nodes[q]) + j];
        for (int j = 0; j < 3; ++j) c[j] /= double(m);
        const int64_t rows = m * nd;
        std::vector<double> B(rows * nc, 0.0), Q(rows * nc, 0.0);  // column-major rows x nc
        for (int64_t q = 0; q < m; ++q) {
            const int64_t node = agg_nodes[b0 + q];
            if (nd == 1) {
                B[q] = mask[node] ? 0.0 : 1.0;
                continue;
            }
            const double x = X[3 * node] - c[0], y = X[3 * node + 1] - c[1], z = X[3 * node + 2] - c[2];
            const double modes[3][6] = {{1, 0, 0, -y, 0, z}, {0, 1, 0, x, -z, 0}, {0, 0, 1, 0, y, -x}};
            for (int r = 0; r < 3; ++r)
                for (int k = 0; k < 6; ++k) B[k * rows + 3 * q + r] = mask[3 * node + r] ? 0.0 : modes[r][k];
        }
        for (int j = 0; j < nc; ++j) {
            double *v = &Q[j * rows];
            const double *bj = &B[j * rows];
            double n0 = 0.0;
            for (int64_t t = 0; t < rows; ++t) {
                v[t] = bj[t];
                n0 += bj[t] * bj[t];
            }
            n0 = std::sqrt(n0);
            for (int k = 0; k < j; ++k) {
                const double *qk = &Q[k * rows];
                double dot = 0.0;
                for (int64_t t = 0; t < rows; ++t) dot += qk[t] * v[t];
                for (int64_t t = 0; t < rows; ++t) v[t] -= dot * qk[t];
            }
            double nv = 0.0;
            for (int64_t t = 0; t < rows; ++t) nv += v[t] * v[t];
            nv = std::sqrt(nv);
            if (n0 > 0.0 && nv > kDropTol * n0) {
                for (int64_t t = 0; t < rows; ++t) v[t] /= nv;
            } else {
                for (int64_t t = 0; t < rows; ++t) v[t] = 0.0;
                dropped[a] |= uint8_t(1u << j);
            }
        }
        for (int64_t q = 0; q < m; ++q) {
            const int64_t node = agg_nodes[b0 + q];
            for (int r = 0; r < nd; ++r)
                for (int k = 0; k < nc; ++k) P[(node * nd + r) * nc + k] = Q[k * rows + q * nd + r];
        }
    }
    // coarse block graph and the fine blocks of every coarse block
    std::vector<int64_t> cptr(na + 1, 0);
    std::vector<int32_t> ccol;
    {
        std::vector<int32_t> seen(na, -1), list;
        for (int32_t a = 0; a < na; ++a) {
            list.clear();
            for (int64_t q = agg_ptr[a]; q < agg_ptr[a + 1]; ++q) {
                const int64_t i = agg_nodes[q];
                for (int64_t k = node_ptr[i]; k < node_ptr[i + 1]; ++k) {
                    const int32_t b = agg[node_nb[k]];
                    if (seen[b] != a) {
                        seen[b] = a;
                        list.push_back(b);
                    }
                }
            }
            std::sort(list.begin(), list.end());
            ccol.insert(ccol.end(), list.begin(), list.end());
            cptr[a + 1] = int64_t(ccol.size());
        }
    }
    const int64_t nbc = int64_t(ccol.size());
    std::vector<int32_t> crow(nbc);
    std::vector<int64_t> cdiag(na);
    for (int32_t a = 0; a < na; ++a)
        for (int64_t b = cptr[a]; b < cptr[a + 1]; ++b) {
            crow[b] = a;
            if (ccol[b] == a) cdiag[a] = b;
        }
    std::vector<int64_t> fb(nnzb);  // coarse block of every fine block
    std::vector<int64_t> cbp(nbc + 1, 0);
    for (int64_t i = 0; i < Nn; ++i) {
        const int32_t I = agg[i];
        const int32_t *c0 = ccol.data() + cptr[I], *c1 = ccol.data() + cptr[I + 1];
        for (int64_t k = node_ptr[i]; k < node_ptr[i + 1]; ++k) {
            const int32_t J = agg[node_nb[k]];
            fb[k] = cptr[I] + (std::lower_bound(c0, c1, J) - c0);
            cbp[fb[k] + 1]++;
        }
    }
    for (int64_t c = 0; c < nbc; ++c) cbp[c + 1] += cbp[c];
    std::vector<int32_t> cbk(nnzb);
    {
        std::vector<int64_t> fill(cbp.begin(), cbp.end() - 1);
        for (int64_t k = 0; k < nnzb; ++k) cbk[fill[fb[k]]++] = int32_t(k);
    }
    // upload
    auto up = [&](const auto &v) {
        using E = typename std::decay_t<decltype(v)>::value_type;
        E *p = static_cast<E *>(dev_alloc(h, v.size() * sizeof(E)));
        if (!v.empty()) FEM_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(E), hipMemcpyHostToDevice));
        return p;
    };
    Amg *a = new Amg();
    a->na = na;
    a->nbc = nbc;
    a->nc = nc;
    a->agg = up(agg);
    a->agg_ptr = up(agg_ptr);
    a->agg_nodes = up(agg_nodes);
    a->P64 = up(P);
    {
        std::vector<float> P32(P.begin(), P.end());
        a->P32 = up(P32);
    }
    a->cptr = up(cptr);
    a->ccol = up(ccol);
    a->crow = up(crow);
    a->cdiag = up(cdiag);
    a->cbp = up(cbp);
    a->cbk = up(cbk);
    a->dropped = up(dropped);
    a->cvals = dev_alloc(h, size_t(nbc) * nc * nc * sizeof(double));
    a->cdinv = dev_alloc(h, size_t(na) * nc * sizeof(double));
    a->fine_tmp = dev_alloc(h, 3 * size_t(N) * sizeof(double));
    a->coarse_tmp = dev_alloc(h, 5 * size_t(na) * nc * sizeof(double));
    a->red = static_cast<double *>(dev_alloc(h, 2 * kRedGrid * sizeof(double)));
    FEM_HIP(hipHostMalloc(reinterpret_cast<void **>(&a->host_red), 2 * kRedGrid * sizeof(double)));
    h->amg = a;
}

void amg_destroy(fem_handle *h) {
    if (!h->amg) return;
    if (h->amg->host_red) (void)hipHostFree(h->amg->host_red);
    delete h->amg;
    h->amg = nullptr;
}

// ------------------------------------------------------------------ per tangent
template <typename T>
void amg_refresh(fem_handle *h, const T *values, const T *dinv, int precision, int smooth_degree, int coarse_degree,
                 hipStream_t s) {
    if (!h->amg) throw Error(FEM_EINVAL, "FEM_PRECOND_AMG needs fem_amg_setup on the handle first");
    Amg &a = *h->amg;
    const Graph &g = h->g;
    AmgView<T> v = view<T>(h);
    const unsigned Gc = grid_for(a.nbc, kThreads / 32);
#define FEM_COARSE(ND, NC)                                                                                       \
    hipLaunchKernelGGL((k_amg_coarse<ND, NC, T>), dim3(Gc), dim3(kThreads), 0, s, a.nbc, a.cbp, a.cbk, a.crow,   \
                       a.ccol, a.dropped, g.blk_row, g.node_ptr, g.node_nb, g.row_ptr, values, v.P, v.cvals)
    if (a.nbc > 0) {
        if (a.nc == 6) FEM_COARSE(3, 6);
        else FEM_COARSE(1, 1);
    }
#undef FEM_COARSE
    FEM_HIP(hipGetLastError());
    const int64_t M = a.na * a.nc;
    if (a.nc == 6)
        hipLaunchKernelGGL((k_amg_cdinv<6, T>), dim3(grid_for(M, kThreads)), dim3(kThreads), 0, s, a.na, a.cdiag,
                           v.cvals, v.cdinv);
    else
        hipLaunchKernelGGL((k_amg_cdinv<1, T>), dim3(grid_for(M, kThreads)), dim3(kThreads), 0, s, a.na, a.cdiag,
                           v.cvals, v.cdinv);
    // spectrum bounds
    if (g.nd == 3)
        hipLaunchKernelGGL((k_gersh_fine<3, T>), dim3(kRedGrid), dim3(kThreads), 0, s, g.Nn, g.node_ptr, values, dinv,
                           a.red);
    else
        hipLaunchKernelGGL((k_gersh_fine<1, T>), dim3(kRedGrid), dim3(kThreads), 0, s, g.Nn, g.node_ptr, values, dinv,
                           a.red);
    const double gf = host_max(a.red, kRedGrid, a.host_red, s);
    if (a.nc == 6)
        hipLaunchKernelGGL((k_gersh_coarse<6, T>), dim3(kRedGrid), dim3(kThreads), 0, s, a.na, a.cptr, v.cvals,
                           v.cdinv, a.red);
    else
        hipLaunchKernelGGL((k_gersh_coarse<1, T>), dim3(kRedGrid), dim3(kThreads), 0, s, a.na, a.cptr, v.cvals,
                           v.cdinv, a.red);
    const double gc = host_max(a.red, kRedGrid, a.host_red, s);
    if (!(gf > 0.0) || !std::isfinite(gf)) throw Error(FEM_ENAN, "preconditioner spectrum bound failed");
    a.lmax = gf;
    a.lmax_c = lmax_bound<T>(
        h, M, [&](const T *x, T *y, T alpha) { coarse_spmv<T>(h, x, y, alpha, nullptr, s); }, v.cdinv, v.rcc, v.dc,
        gc, s);
    a.precision = precision;
    a.sdeg = smooth_degree;
    a.cdeg = coarse_degree;
}

// z = M r (one V-cycle).
template <typename T>
static void vcycle(fem_handle *h, const T *values, const T *dinv, const T *r, T *z, int sdeg, int cdeg,
                   const KrylovScalars *sc, hipStream_t s) {
    Amg &a = *h->amg;
    const Graph &g = h->g;
    AmgView<T> v = view<T>(h);
    const Cheb cf = chebyshev_coeffs(a.lmax, sdeg), cc = chebyshev_coeffs(a.lmax_c, cdeg);
    auto fine_op = [&](const T *x, T *y) { launch_spmv_sc<T>(h, values, x, y, T(1), T(0), sc, s); };
    auto coarse_op = [&](const T *x, T *y) { coarse_spmv<T>(h, x, y, T(1), sc, s); };
    const int64_t M = a.na * a.nc;
    // pre-smoothing from 0
    chebyshev_run<T>(g.N, cf, fine_op, r, dinv, z, v.w, v.rc, v.d, 0, sc, s);
    // restriction of r - A z
    fine_op(z, v.w);
    const unsigned Ga = grid_for(a.na, kWavesPerBlock);
    if (a.nc == 6)
        hipLaunchKernelGGL((k_amg_restrict<3, 6, T>), dim3(Ga), dim3(kThreads), 0, s, a.na, a.agg_ptr, a.agg_nodes,
                           v.P, r, v.w, v.bc, sc);
    else
        hipLaunchKernelGGL((k_amg_restrict<1, 1, T>), dim3(Ga), dim3(kThreads), 0, s, a.na, a.agg_ptr, a.agg_nodes,
                           v.P, r, v.w, v.bc, sc);
    // coarse correction
    chebyshev_run<T>(M, cc, coarse_op, v.bc, v.cdinv, v.zc, v.wc, v.rcc, v.dc, 0, sc, s);
    if (a.nc == 6)
        hipLaunchKernelGGL((k_amg_prolong<3, 6, T>), dim3(grid_for(g.Nn, kThreads)), dim3(kThreads), 0, s, g.Nn,
                           a.agg, v.P, v.zc, z, sc);
    else
        hipLaunchKernelGGL((k_amg_prolong<1, 1, T>), dim3(grid_for(g.Nn, kThreads)), dim3(kThreads), 0, s, g.Nn,
                           a.agg, v.P, v.zc, z, sc);
    FEM_HIP(hipGetLastError());
    // post-smoothing continued from z
    fine_op(z, v.w);
    chebyshev_run<T>(g.N, cf, fine_op, r, dinv, z, v.w, v.rc, v.d, 1, sc, s);
}

template <typename T>
void amg_apply(fem_handle *h, const T *values, const T *dinv, const T *r, T *z, const KrylovScalars *sc,
               hipStream_t s) {
    vcycle<T>(h, values, dinv, r, z, h->amg->sdeg, h->amg->cdeg, sc, s);
}

template <typename T>
void kry_cg_amg_init(fem_handle *h, const KrylovVecs<T> &k, const T *b, double rtol, hipStream_t s) {
    const int64_t N = h->g.N;
    const unsigned G = grid_for(N, kThreads);
    hipLaunchKernelGGL((k_copy_vec<T>), dim3(G), dim3(kThreads), 0, s, N, b, k.r);
    hipLaunchKernelGGL((k_zero_vec<T>), dim3(G), dim3(kThreads), 0, s, N, k.x);
    vcycle<T>(h, k.A, k.dinv, k.r, k.rh, h->amg->sdeg, h->amg->cdeg, nullptr, s);
    hipLaunchKernelGGL((k_copy_vec<T>), dim3(G), dim3(kThreads), 0, s, N, k.rh, k.p);
    const int Gd = krylov_grid(h);
    hipLaunchKernelGGL((k_dot_rz_rr<T>), dim3(Gd), dim3(kThreads), 0, s, N, k.r, k.rh, k.partials, nullptr);
    hipLaunchKernelGGL(k_fin_init_amg, dim3(1), dim3(64), 0, s, Gd, k.partials, k.sc, rtol);
    FEM_HIP(hipGetLastError());
}

template <typename T>
void kry_cg_amg_iter(fem_handle *h, const KrylovVecs<T> &k, int it, hipStream_t s, hipEvent_t *ev) {
    const int64_t N = h->g.N;
    if (ev) FEM_HIP(hipEventRecord(ev[0], s));
    const int G = kry_spmv_q<T>(h, k, s);  // q = K p, (p, q) partials
    if (ev) FEM_HIP(hipEventRecord(ev[1], s));
    const int Gv = krylov_vec_grid_of(h);
    hipLaunchKernelGGL((k_cg_xr_plain<T>), dim3(Gv), dim3(kThreads), 0, s, N, k.x, k.r, k.p, k.v, k.partials, G,
                       k.sc, it);
    vcycle<T>(h, k.A, k.dinv, k.r, k.rh, h->amg->sdeg, h->amg->cdeg, k.sc, s);
    hipLaunchKernelGGL((k_dot_rz_rr<T>), dim3(Gv), dim3(kThreads), 0, s, N, k.r, k.rh, k.partials2, k.sc);
    FEM_HIP(hipGetLastError());
    kry_cg_p_update<T>(h, k, it, s);
}

// The current coarse operator, widened to FP64, to a device buffer.
void amg_coarse_values_f64(const fem_handle *h, double *out, hipStream_t s) {
    const Amg &a = *h->amg;
    const int64_t n = a.nbc * a.nc * a.nc;
    if (n == 0) return;
    if (a.precision == FEM_PREC_MIXED)
        hipLaunchKernelGGL((k_widen<float>), dim3(grid_for(n, kThreads)), dim3(kThreads), 0, s, n,
                           static_cast<const float *>(a.cvals), out);
    else
        hipLaunchKernelGGL((k_widen<double>), dim3(grid_for(n, kThreads)), dim3(kThreads), 0, s, n,
                           static_cast<const double *>(a.cvals), out);
    FEM_HIP(hipGetLastError());
}

template void amg_refresh<float>(fem_handle *, const float *, const float *, int, int, int, hipStream_t);
template void amg_refresh<double>(fem_handle *, const double *, const double *, int, int, int, hipStream_t);
template void amg_apply<float>(fem_handle *, const float *, const float *, const float *, float *,
                               const KrylovScalars *, hipStream_t);
template void amg_apply<double>(fem_handle *, const double *, const double *, const double *, double *,
                                const KrylovScalars *, hipStream_t);
template void kry_cg_amg_init<float>(fem_handle *, const KrylovVecs<float> &, const float *, double, hipStream_t);
template void kry_cg_amg_init<double>(fem_handle *, const KrylovVecs<double> &, const double *, double, hipStream_t);
template void kry_cg_amg_iter<float>(fem_handle *, const KrylovVecs<float> &, int, hipStream_t, hipEvent_t *);
template void kry_cg_amg_iter<double>(fem_handle *, const KrylovVecs<double> &, int, hipStream_t, hipEvent_t *);

}  // namespace fem

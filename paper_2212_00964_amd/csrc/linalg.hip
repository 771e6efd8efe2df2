// Sparse matrix-vector products and Jacobi-preconditioned Krylov kernels.
//
// The CSR matrix is stored over all dofs with node-major interleaved components, so
// the ND rows of node n are contiguous and each of them lists the node's neighbour
// blocks in the same order.  The SpMV therefore walks the node graph (one 32-bit
// column index per ND x ND block) instead of the scalar column array: a group of 32
// lanes owns one node, lane l takes the l-th neighbour block, and the ND row sums
// are finished with a 32-lane reduction built from cross-lane register moves.
//
// Krylov inner products are FP64 and deterministic: every block stores its partial
// sum (fixed lane order), and the next kernel sums the partials in block order,
// either in a one-block finalize kernel or redundantly in every block of the next
// vector kernel (CG).  Scalars of the method live on the device; the host only reads
// the convergence flag every few iterations.
//
// Paper: BiCGSTAB with a Jacobi preconditioner is the linear solver inside Newton
// (Sec. 5, item 2; van der Vorst 1992).
#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "lanes.h"

namespace fem {

namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n, int threads) { return unsigned((n + threads - 1) / threads); }

template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

// Row sums of node n: acc[i] = sum_j sum_k K[(n,i),(m_j,k)] x[(m_j,k)] (or K^T),
// computed by a group of G lanes (lane l takes blocks l, l+G, ...).  Every lane of
// the group returns the same totals.
template <int ND, int G, bool TRANS, typename T>
__device__ __forceinline__ void node_rows(int64_t n, int lane, const int64_t *__restrict__ node_ptr,
                                          const int32_t *__restrict__ node_nb, const int32_t *__restrict__ mirror,
                                          const T *__restrict__ values, const T *__restrict__ x, T acc[ND]) {
#pragma unroll
    for (int i = 0; i < ND; ++i) acc[i] = T(0);
    const int64_t b0 = node_ptr[n];
    const int deg = int(node_ptr[n + 1] - b0);
    const T *vb = values + int64_t(ND) * ND * b0;
#pragma unroll 4
    for (int l = lane; l < deg; l += G) {
        const int64_t m = node_nb[b0 + l];
        T xm[ND];
#pragma unroll
        for (int k = 0; k < ND; ++k) xm[k] = x[ND * m + k];
        if constexpr (!TRANS) {
#pragma unroll
            for (int i = 0; i < ND; ++i) {
                const T *row = vb + int64_t(i) * ND * deg + ND * l;
#pragma unroll
                for (int k = 0; k < ND; ++k) acc[i] += __builtin_nontemporal_load(row + k) * xm[k];
            }
        } else {
            // (K^T)[(n,i),(m,k)] = K[(m,k),(n,i)], stored in block (m, n) = mirror
            const int64_t kb = mirror[b0 + l];
            const int64_t mb0 = node_ptr[m];
            const int mdeg = int(node_ptr[m + 1] - mb0);
            const T *mv = values + int64_t(ND) * ND * mb0 + ND * (kb - mb0);
#pragma unroll
            for (int k = 0; k < ND; ++k)
#pragma unroll
                for (int i = 0; i < ND; ++i) acc[i] += mv[int64_t(k) * ND * mdeg + i] * xm[k];
        }
    }
#pragma unroll
    for (int i = 0; i < ND; ++i) acc[i] = group_sum<G>(acc[i]);
}

template <int ND, int G, bool TRANS, typename T>
__global__ __launch_bounds__(kThreads) void k_spmv(int64_t Nn, const int64_t *__restrict__ node_ptr,
                                                   const int32_t *__restrict__ node_nb,
                                                   const int32_t *__restrict__ mirror, const T *__restrict__ values,
                                                   const T *__restrict__ x, T *__restrict__ y, T alpha, T beta) {
    const int lane = threadIdx.x % G;
    const int64_t n = int64_t(blockIdx.x) * (kThreads / G) + threadIdx.x / G;
    if (n >= Nn) return;  // uniform per group
    T acc[ND];
    node_rows<ND, G, TRANS, T>(n, lane, node_ptr, node_nb, mirror, values, x, acc);
    if (lane < ND) {
        T s = acc[0];
#pragma unroll
        for (int i = 1; i < ND; ++i)
            if (lane == i) s = acc[i];
        T out = alpha * s;
        if (beta != T(0)) out += beta * y[ND * n + lane];
        y[ND * n + lane] = out;
    }
}

// ------------------------------------------------------------------ deterministic reductions
// Grid-wide FP64 sums are done in two kernels: every block of the producing kernel
// stores its block total to partials[c * G + blockIdx.x] (plain stores, no fences or
// atomics: on a multi-XCD device a device-scope fence per block would write back the
// XCD's L2 every time), and a one-block finalize kernel launched next on the same
// stream adds the G partials in block order.  The result is bit-reproducible.
template <int NV>
__device__ void block_store_partials(const double v[NV], double *partials) {
    __shared__ double red[kThreads / 64][NV];
    double w[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        double t = v[c];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        w[c] = t;
    }
    const int wave = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) red[wave][c] = w[c];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            double t = 0.0;
            for (int k = 0; k < kThreads / 64; ++k) t += red[k][c];
            partials[c * gridDim.x + blockIdx.x] = t;
        }
    }
}

// In a one-block finalize kernel: totals of the G partials of each of NV sums.
template <int NV>
__device__ void sum_partials(const double *partials, int G, double tot[NV]) {
    __shared__ double red[kThreads / 64][NV];
    double v[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        double t = 0.0;
        for (int b = threadIdx.x; b < G; b += kThreads) t += partials[c * G + b];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        v[c] = t;
    }
    const int wave = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) red[wave][c] = v[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        double t = 0.0;
        for (int k = 0; k < kThreads / 64; ++k) t += red[k][c];
        tot[c] = t;
    }
}

// Contiguous node range of this block.  Blocks are dealt round-robin to the 8 XCDs,
// so the logical block index groups the blocks of one XCD onto adjacent ranges and
// each XCD's L2 sees a compact slab of the mesh (the x-vector gathers stay local).
__device__ __forceinline__ void block_range(int64_t Nn, int64_t &n0, int64_t &n1) {
    const unsigned G = gridDim.x, b = blockIdx.x;
    const unsigned per = G / 8;
    unsigned L = (G % 8 == 0) ? (b % 8) * per + b / 8 : b;
    int64_t chunk = (Nn + G - 1) / G;
    n0 = int64_t(L) * chunk;
    n1 = n0 + chunk < Nn ? n0 + chunk : Nn;
}

__device__ __forceinline__ bool stopped(const KrylovScalars *sc) { return sc->converged | sc->breakdown; }

// Persistent SpMV over this block's contiguous node range.  The range's row
// pointers are staged in LDS once; each 32-lane group then takes P nodes at a time
// and issues all their column-index and value loads before any of them is used, so
// a wave keeps P times more HBM traffic in flight than a one-node-at-a-time walk,
// and the next P nodes' loads are issued before the current x gathers are awaited.
// Lane l of a group handles neighbour block l of each of its nodes (node degrees
// above 32 fall back to a strided loop); the ND row sums are finished with a
// reduce-scatter over the group (a row swap and four DPP steps, no LDS traffic).
// Row results are kept in LDS and written (with the dot-product terms) after the
// chunk.  D16: column blocks read as 16-bit offsets from the row node (half the index
// bytes) when the node numbering allows it.
//
// MODE 0: y = alpha K x + beta y
// MODE 1: y = K x and alpha = rho / (w0, y)                 (BiCGSTAB v = K ph, CG q = K p)
// MODE 2: y = K x and omega = (w0, y) / (y, y), w0 = s      (BiCGSTAB t = K sh)
constexpr int kSpmvGroup = 32;
constexpr int kMaxChunk = 1024;  // nodes per block staged in LDS

// Nodes in flight per 32-lane group: as many as fit with the double-buffered loads
// at an occupancy of four (FP32 values) or two (FP64 values) wavefronts per SIMD.
// TV is the type of the stored values.  FP32 values under FP64 vectors (the mixed form
// with FP64 Krylov vectors): four nodes at three wavefronts per SIMD (149 registers;
// measured 243 us per launch at the 100^3 workload against 254 us with three nodes at
// four wavefronts, which fit in 128).
template <int ND, typename TV, typename T = TV>
constexpr int spmv_batch() { return ND == 1 ? 4 : (sizeof(TV) == 4 ? 4 : 2); }

template <typename TV, typename T>
constexpr int spmv_waves() { return sizeof(TV) == 4 ? (sizeof(T) == 4 ? 4 : 3) : 2; }

template <int ND, int P, int MODE, typename T, bool D16, typename TV = T>
__global__ __launch_bounds__(kThreads, (spmv_waves<TV, T>())) void k_spmv_nodes(int64_t Nn, const int64_t *__restrict__ node_ptr,
                                                         const int32_t *__restrict__ node_nb,
                                                         const int16_t *__restrict__ node_dnb,
                                                         const TV *__restrict__ values, const T *__restrict__ x,
                                                         T *__restrict__ y, const T *__restrict__ w0, T alpha,
                                                         T beta, double *partials, KrylovScalars *sc, int cg,
                                                         int big) {
    constexpr int G = kSpmvGroup;
    constexpr int GPB = kThreads / G;  // groups per block
    static_assert(G == 32 && (ND == 1 || ND == 3), "32-lane groups, 1 or 3 dofs per node");
    __shared__ int64_t sptr[kMaxChunk + 1];
    __shared__ T sy[kMaxChunk * ND];  // the chunk's results, written out at its end
    constexpr int NDOT = MODE == 2 ? 3 : MODE;  // (w0, y); MODE 2 also (y, y) and (w0, w0)
    __shared__ double sdot[MODE != 0 ? NDOT * kThreads : 1];  // per-thread dot terms (no registers in the node loop)
    if ((MODE != 0 || sc != nullptr) && stopped(sc)) return;  // MODE 0 with sc: inside a Krylov loop
    if (MODE != 0)
        for (int c = 0; c < NDOT; ++c) sdot[c * kThreads + threadIdx.x] = 0.0;
    int64_t r0, r1;
    block_range(Nn, r0, r1);
    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    // after the group reduction, lanes 0, 8, 16 hold rows 0, 1, 2 of the node
    const int row = (lane & 7) == 0 && lane < 8 * ND ? lane / 8 : -1;
    for (int64_t n0 = r0; n0 < r1; n0 += kMaxChunk) {
        const int cnt = int(r1 - n0 < kMaxChunk ? r1 - n0 : kMaxChunk);
        __syncthreads();  // previous sub-chunk finished with sptr
        for (int i = threadIdx.x; i <= cnt; i += kThreads) sptr[i] = node_ptr[n0 + i];
        __syncthreads();
        int64_t b0[P];
        int deg[P];
        int32_t m[P];
        TV v[P][ND][ND];
        // Column indices and values of P nodes.  Addresses are clamped (a slot past the
        // chunk re-reads its last node, a lane past the degree reads block 0), so the
        // loads are branch-free; the results of such slots are masked.
        auto load_batch = [&](int base) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                int ln = base + p * GPB;
                ln = ln < cnt ? ln : cnt - 1;
                b0[p] = sptr[ln];
                deg[p] = int(sptr[ln + 1] - b0[p]);
                const int lc = lane < deg[p] ? lane : 0;
                if constexpr (D16)
                    m[p] = int32_t(n0 + ln) + int32_t(__builtin_nontemporal_load(node_dnb + b0[p] + lc));
                else
                    m[p] = __builtin_nontemporal_load(node_nb + b0[p] + lc);
                const TV *vb = values + int64_t(ND) * ND * b0[p] + ND * lc;
#pragma unroll
                for (int i = 0; i < ND; ++i)
#pragma unroll
                    for (int k = 0; k < ND; ++k)
                        v[p][i][k] = __builtin_nontemporal_load(vb + int64_t(i) * ND * deg[p] + k);
            }
        };
        load_batch(grp);
        for (int base = grp; base < cnt; base += P * GPB) {
            // Software pipeline: the x gathers of this batch go out first, then the next
            // batch's index and value loads, so waiting for the gathers leaves the next
            // batch in flight (memory counters complete in issue order).
            T xm[P][ND];
            TV cv[P][ND][ND];
            int cdeg[P];
#pragma unroll
            for (int p = 0; p < P; ++p) {
#pragma unroll
                for (int k = 0; k < ND; ++k) xm[p][k] = x[int64_t(ND) * m[p] + k];
                cdeg[p] = deg[p];
#pragma unroll
                for (int i = 0; i < ND; ++i)
#pragma unroll
                    for (int k = 0; k < ND; ++k) cv[p][i][k] = v[p][i][k];
            }
            load_batch(base + P * GPB);
#pragma unroll
            for (int p = 0; p < P; ++p) {
                T acc[ND];
#pragma unroll
                for (int i = 0; i < ND; ++i) {
                    T a = T(0);
#pragma unroll
                    for (int k = 0; k < ND; ++k) a += T(cv[p][i][k]) * xm[p][k];
                    acc[i] = lane < cdeg[p] ? a : T(0);
                }
                T sv;
                if constexpr (ND == 3) sv = group32_sum3(acc[0], acc[1], acc[2], lane);
                else sv = group32_sum(acc[0], lane);
                const int ln = base + p * GPB;
                if (ln < cnt && row >= 0) sy[ND * ln + row] = sv;
            }
        }
        __syncthreads();
        if (big) {  // neighbours beyond the 32nd of high-degree nodes (none on structured meshes)
            for (int ln = grp; ln < cnt; ln += GPB) {
                const int64_t b = sptr[ln];
                const int dg = int(sptr[ln + 1] - b);
                if (dg <= G) continue;
                T acc[ND];
#pragma unroll
                for (int i = 0; i < ND; ++i) acc[i] = T(0);
                for (int l = lane + G; l < dg; l += G) {
                    const int64_t mm = node_nb[b + l];
                    const TV *vb = values + int64_t(ND) * ND * b + ND * l;
#pragma unroll
                    for (int i = 0; i < ND; ++i)
#pragma unroll
                        for (int k = 0; k < ND; ++k) acc[i] += T(vb[int64_t(i) * ND * dg + k]) * x[ND * mm + k];
                }
                T sv;
                if constexpr (ND == 3) sv = group32_sum3(acc[0], acc[1], acc[2], lane);
                else sv = group32_sum(acc[0], lane);
                if (row >= 0) sy[ND * ln + row] += sv;
            }
            __syncthreads();
        }
        // The chunk's rows go out as one coalesced pass.  Stores share the vector
        // memory counter with loads here, so a store inside the node loop would make
        // every later wait for a load also wait for that store's acknowledgement.
        double d0 = 0.0, d1 = 0.0, d2 = 0.0;
        // (non-temporal stores: measured 4% faster than cached ones for this pass)
        for (int i = threadIdx.x; i < ND * cnt; i += kThreads) {
            const int64_t d = int64_t(ND) * n0 + i;
            const T sv = sy[i];
            if (MODE == 0) {
                T out = alpha * sv;
                if (beta != T(0)) out += beta * y[d];
                __builtin_nontemporal_store(out, y + d);
            } else {
                __builtin_nontemporal_store(sv, y + d);
                const double wd = double(w0[d]);
                d0 += wd * double(sv);
                if (MODE == 2) {
                    d1 += double(sv) * double(sv);
                    d2 += wd * wd;
                }
            }
        }
        if (MODE != 0) {
            sdot[threadIdx.x] += d0;
            if (MODE == 2) {
                sdot[kThreads + threadIdx.x] += d1;
                sdot[2 * kThreads + threadIdx.x] += d2;
            }
        }
    }
    if constexpr (MODE != 0) {
        double vv[NDOT];
        for (int c = 0; c < NDOT; ++c) vv[c] = sdot[c * kThreads + threadIdx.x];
        block_store_partials<NDOT>(vv, partials);
    }
}

// SpMV on the symmetric block layout (blocks (n, m) with m >= n stored, block-major).
// Node n's row needs its upper blocks, which are contiguous from up_base[n], and its
// lower blocks (n, m), m < n, which are the transposes of the stored blocks (m, n)
// (index lo_val).  Those were streamed moments earlier by the block range holding
// node m, so they come from L2 or the Infinity Cache; HBM traffic is the stored half
// of the matrix.  Same persistent scheme as k_spmv_nodes (LDS-staged row data, P
// nodes in flight per 32-lane group, branch-free loads on clamped addresses).
template <int ND, int P, int MODE, typename T>
__global__ __launch_bounds__(kThreads) void k_spmv_sym(int64_t Nn, const int64_t *__restrict__ node_ptr,
                                                       const int64_t *__restrict__ up_base,
                                                       const int32_t *__restrict__ node_nb,
                                                       const int32_t *__restrict__ lo_val,
                                                       const T *__restrict__ values, const T *__restrict__ x,
                                                       T *__restrict__ y, const T *__restrict__ w0, T alpha, T beta,
                                                       double *partials, KrylovScalars *sc, int cg) {
    constexpr int G = kSpmvGroup;
    constexpr int GPB = kThreads / G;
    constexpr int CH = kMaxChunk / 2;
    constexpr int BS = ND * ND;
    __shared__ int64_t sptr[CH + 1];
    __shared__ int64_t sup[CH + 1];
    if (MODE != 0 && stopped(sc)) return;
    int64_t r0, r1;
    block_range(Nn, r0, r1);
    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    double d0 = 0.0, d1 = 0.0, d2 = 0.0;
    for (int64_t n0 = r0; n0 < r1; n0 += CH) {
        const int cnt = int(r1 - n0 < CH ? r1 - n0 : CH);
        __syncthreads();
        for (int i = threadIdx.x; i <= cnt; i += kThreads) {
            sptr[i] = node_ptr[n0 + i];
            sup[i] = up_base[n0 + i];
        }
        __syncthreads();
        for (int base = grp; base < cnt; base += P * GPB) {
            int64_t b0[P], ub[P];
            int deg[P], dpos[P];
            int32_t m[P];
            T v[P][BS];
            T xm[P][ND];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int ln = base + p * GPB;
                const bool ok = ln < cnt;
                b0[p] = ok ? sptr[ln] : 0;
                deg[p] = ok ? int(sptr[ln + 1] - sptr[ln]) : 0;
                ub[p] = ok ? sup[ln] : 0;
                dpos[p] = ok ? deg[p] - int(sup[ln + 1] - sup[ln]) : 0;
            }
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const bool act = lane < deg[p];
                const bool lower = lane < dpos[p];
                m[p] = __builtin_nontemporal_load(node_nb + b0[p] + (act ? lane : 0));
                const int32_t lv = __builtin_nontemporal_load(lo_val + b0[p] + (lower ? lane : 0));
                const int64_t ku = lower ? int64_t(lv) : (act ? ub[p] + (lane - dpos[p]) : ub[p]);
                const T *vb = values + BS * ku;
#pragma unroll
                for (int q = 0; q < BS; ++q) v[p][q] = vb[q];
            }
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int k = 0; k < ND; ++k) xm[p][k] = x[int64_t(ND) * m[p] + k];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const bool act = lane < deg[p];
                const bool lower = lane < dpos[p];
                T acc[ND];
#pragma unroll
                for (int i = 0; i < ND; ++i) {
                    T a = T(0);
#pragma unroll
                    for (int k = 0; k < ND; ++k) a += (lower ? v[p][k * ND + i] : v[p][i * ND + k]) * xm[p][k];
                    acc[i] = act ? a : T(0);
                }
                for (int l = lane + G; l < deg[p]; l += G) {  // high-degree nodes
                    const int64_t mm = node_nb[b0[p] + l];
                    const bool lw = l < dpos[p];
                    const int64_t kk = lw ? int64_t(lo_val[b0[p] + l]) : ub[p] + (l - dpos[p]);
                    const T *vb = values + BS * kk;
#pragma unroll
                    for (int i = 0; i < ND; ++i)
#pragma unroll
                        for (int k = 0; k < ND; ++k) acc[i] += (lw ? vb[k * ND + i] : vb[i * ND + k]) * x[ND * mm + k];
                }
#pragma unroll
                for (int i = 0; i < ND; ++i) acc[i] = group_sum<G>(acc[i]);
                const int ln = base + p * GPB;
                if (ln < cnt && lane < ND) {
                    T sv = acc[0];
#pragma unroll
                    for (int i = 1; i < ND; ++i)
                        if (lane == i) sv = acc[i];
                    const int64_t d = int64_t(ND) * (n0 + ln) + lane;
                    if (MODE == 0) {
                        T out = alpha * sv;
                        if (beta != T(0)) out += beta * y[d];
                        y[d] = out;
                    } else {
                        y[d] = sv;
                        const double wd = double(w0[d]);
                        d0 += wd * double(sv);
                        if (MODE == 2) {
                            d1 += double(sv) * double(sv);
                            d2 += wd * wd;
                        }
                    }
                }
            }
        }
    }
    if constexpr (MODE != 0) {
        constexpr int NDOT = MODE == 2 ? 3 : MODE;
        double vv[3] = {d0, d1, d2};
        block_store_partials<NDOT>(vv, partials);
    }
}

// alpha = rho / (w0, y)
__global__ __launch_bounds__(kThreads) void k_fin_alpha(int G, const double *__restrict__ partials,
                                                        KrylovScalars *sc, int cg) {
    if (stopped(sc)) return;
    double tot[1];
    sum_partials<1>(partials, G, tot);
    if (threadIdx.x == 0) {
        bool bad = !(tot[0] != 0.0) || !isfinite(tot[0]) || (cg && !(tot[0] > 0.0));
        if (bad) sc->breakdown = 1;
        else sc->alpha = sc->rho / tot[0];
    }
}

// omega = (t, s) / (t, t)
__global__ __launch_bounds__(kThreads) void k_fin_omega(int G, const double *__restrict__ partials,
                                                        KrylovScalars *sc) {
    if (stopped(sc)) return;
    double tot[2];
    sum_partials<2>(partials, G, tot);
    if (threadIdx.x == 0) sc->omega = (tot[1] > 0.0 && isfinite(tot[1])) ? tot[0] / tot[1] : 0.0;
}

// BiCGSTAB (block Jacobi form): x += alpha ph + omega sh; r = s - omega t; rho_new = (rh, r); |r|^2
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bicg_xr(int64_t N, T *__restrict__ x, T *__restrict__ r,
                                                      const T *__restrict__ rh, const T *__restrict__ ph,
                                                      const T *__restrict__ s, const T *__restrict__ sh,
                                                      const T *__restrict__ t, double *partials, KrylovScalars *sc) {
    if (stopped(sc)) return;
    const T al = T(sc->alpha), om = T(sc->omega);
    double d0 = 0.0, d1 = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < N; i += int64_t(gridDim.x) * kThreads) {
        x[i] += al * ph[i] + om * sh[i];
        T ri = s[i] - om * t[i];
        r[i] = ri;
        d0 += double(rh[i]) * double(ri);
        d1 += double(ri) * double(ri);
    }
    double v[2] = {d0, d1};
    block_store_partials<2>(v, partials);
}

// BiCGSTAB: rho_new = (rhat, r), |r|^2; convergence, divergence and restart tests
__global__ __launch_bounds__(kThreads) void k_fin_bicg_xr(int G, const double *__restrict__ partials,
                                                          KrylovScalars *sc) {
    if (stopped(sc)) return;
    double tot[2];
    sum_partials<2>(partials, G, tot);
    if (threadIdx.x == 0) {
        sc->rho_old = sc->rho;
        sc->rho = tot[0];
        sc->rnorm2 = tot[1];
        sc->its += 1;
        if (!isfinite(tot[0]) || !isfinite(tot[1])) {
            sc->breakdown = 2;
        } else if (tot[1] <= sc->tol2) {
            sc->converged = 1;
        } else if (tot[1] > 1e12 * sc->bnorm2) {
            sc->breakdown = 1;  // diverged
        } else if (!(fabs(tot[0]) > 1e-9 * sqrt(sc->rh2 * tot[1])) || sc->omega == 0.0 ||
                   tot[1] > 1e6 * sc->rmin2) {
            // (rhat, r) lost its size relative to |rhat||r|, omega vanished, or the
            // residual grew 1000x above its best value: restart from the current r
            sc->restart_at = sc->its;
            sc->rho = tot[1];
            sc->rh2 = tot[1];
        }
        sc->rmin2 = fmin(sc->rmin2, tot[1]);
    }
}

// 16-byte vector view of an FP32 (4 lanes) or FP64 (2 lanes) array.
template <typename T>
struct Vec16 {
    static constexpr int W = 16 / int(sizeof(T));
    typedef T type __attribute__((ext_vector_type(W)));
    __device__ static type ld(const T *a, int64_t i) { return reinterpret_cast<const type *>(a)[i]; }
    __device__ static void st(T *a, int64_t i, type v) { reinterpret_cast<type *>(a)[i] = v; }
    __device__ static void st_nt(T *a, int64_t i, type v) { __builtin_nontemporal_store(v, reinterpret_cast<type *>(a) + i); }
};

// CG with the scalar updates folded into the vector kernels.  Each block sums the
// previous kernel's per-block partials itself (same order in every block, so all
// blocks agree bit for bit), which removes the one-block finalize launches.
//
// Iteration it: alpha = rho_pp[it & 1] / (p, q) with q = K p from the SpMV partials;
// x += alpha p; r -= alpha q; z = Dinv r; partials of (r, z) and |r|^2.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_xr_fused(int64_t N, T *__restrict__ x, T *__restrict__ r,
                                                          T *__restrict__ z, const T *__restrict__ p,
                                                          const T *__restrict__ q, const T *__restrict__ dinv,
                                                          const double *__restrict__ pq_partials, int pq_count,
                                                          double *partials, KrylovScalars *sc, int it) {
    if (stopped(sc)) return;
    double pq[1];
    sum_partials<1>(pq_partials, pq_count, pq);
    if (!(pq[0] > 0.0) || !isfinite(pq[0])) {  // CG needs (p, K p) > 0
        if (blockIdx.x == 0 && threadIdx.x == 0) sc->breakdown = 1;
        return;
    }
    const double alpha = sc->rho_pp[it & 1] / pq[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->alpha = alpha;
    const T al = T(alpha);
    double d0 = 0.0, d1 = 0.0;
    auto update = [&](int64_t i) {
        x[i] += al * p[i];
        T ri = r[i] - al * q[i];
        r[i] = ri;
        T zi = dinv[i] * ri;
        z[i] = zi;
        d0 += double(ri) * double(zi);
        d1 += double(ri) * double(ri);
    };
    // 16-byte accesses over the bulk (the vectors are 256-byte aligned), scalar tail
    using V = Vec16<T>;
    constexpr int W = V::W;
    const int64_t NV = N / W;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < NV; i += int64_t(gridDim.x) * kThreads) {
        typename V::type xv = V::ld(x, i), pv = V::ld(p, i), rv = V::ld(r, i), qv = V::ld(q, i), dv = V::ld(dinv, i);
        xv += al * pv;
        rv -= al * qv;
        const typename V::type zv = dv * rv;
        V::st_nt(x, i, xv);
        V::st_nt(r, i, rv);
        V::st_nt(z, i, zv);
#pragma unroll
        for (int c = 0; c < W; ++c) {
            d0 += double(rv[c]) * double(zv[c]);
            d1 += double(rv[c]) * double(rv[c]);
        }
    }
    if (blockIdx.x == 0)
        for (int64_t i = NV * W + threadIdx.x; i < N; i += kThreads) update(i);
    double v[2] = {d0, d1};
    block_store_partials<2>(v, partials);
}

// rho = (r, z), |r|^2 from the partials; convergence test; beta = rho / rho_pp[it & 1];
// p = z + beta p.  Block 0 publishes the scalars (the new rho to the other slot).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_p_fused(int64_t N, const T *__restrict__ z, T *__restrict__ p,
                                                         const double *__restrict__ rz_partials, int rz_count,
                                                         KrylovScalars *sc, int it) {
    if (stopped(sc)) return;
    double tot[2];
    sum_partials<2>(rz_partials, rz_count, tot);
    const double rho_prev = sc->rho_pp[it & 1];
    const bool nan = !isfinite(tot[0]) || !isfinite(tot[1]);
    const bool conv = !nan && tot[1] <= sc->tol2;
    const double beta = tot[0] / rho_prev;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->rho_old = rho_prev;
        sc->rho = tot[0];
        sc->rho_pp[(it + 1) & 1] = tot[0];
        sc->beta = beta;
        sc->rnorm2 = tot[1];
        sc->its = it + 1;
        if (nan) sc->breakdown = 2;
        else if (conv) sc->converged = 1;
    }
    if (nan || conv) return;
    const T bt = T(beta);
    using V = Vec16<T>;
    constexpr int W = V::W;
    const int64_t NV = N / W;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < NV; i += int64_t(gridDim.x) * kThreads)
        V::st_nt(p, i, V::ld(z, i) + bt * V::ld(p, i));
    if (blockIdx.x == 0)
        for (int64_t i = NV * W + threadIdx.x; i < N; i += kThreads) p[i] = z[i] + bt * p[i];
}

// ------------------------------------------------------------------ fused BiCGSTAB
// The point-Jacobi BiCGSTAB with its scalar updates folded into the vector kernels
// (every block sums the previous kernel's partials in block order, so all blocks agree
// bit for bit and no one-block finalize kernel is launched).  Iteration i:
//   p-kernel:  rho_i, |r_i|^2 from the (rhat, r), (r, r) partials of iteration i - 1;
//              convergence, divergence and restart tests; p = r + beta (p - omega v)
//              (or p = r, rhat = r on a restart); ph = Dinv p
//   SpMV:      v = K ph with the (rhat, v) partials
//   s-kernel:  alpha = rho_i / (rhat, v); s = r - alpha v; sh = Dinv s
//   SpMV:      t = K sh with the (t, s), (t, t) partials
//   xr-kernel: omega = (t, s) / (t, t); x += alpha ph + omega sh; r = s - omega t, and
//              the (rhat, r), (r, r) partials for iteration i + 1.
// The scalars of iteration i go to slot i & 1 (see KrylovScalars).

// Finite-precision safeguards of the fused BiCGSTAB, for FP32 vectors.  Omega limit:
// when t and s are nearly orthogonal (|(t, s)| < Omega |t| |s|), omega = (t, s) / (t, t)
// is scaled up by Omega / cos(t, s), which keeps the BiCG coefficients of the next
// steps accurate (Sleijpen and van der Vorst's 'limited omega', Omega = 0.7).  Restart
// floor: see bicg_rho_floor.  Measured on the 5-step 100^3 and 200x100x100 neo-Hookean
// solves: FP32 sweeps without the floor diverged on the larger one; the limit cut its
// FP32 iterations by a third (27,704 against 41,951) but cost the FP64 vectors 48% more
// (23,236 against 15,705), so FP64 runs plain BiCGSTAB.
constexpr double kOmegaLimitF32 = 0.7;
constexpr double kRhoFloorF32 = 1e-5;

template <typename T>
__device__ __forceinline__ double bicg_omega_limit() { return sizeof(T) == 4 ? kOmegaLimitF32 : 0.0; }

struct BicgStart {
    double rho, r2, rh2, rmin2;
    bool nan, conv, div, restart;
};

// Restart floor of |(rhat, r)| / (|rhat| |r|): below it the shadow inner product has
// lost its meaning.  In FP32 the vectors carry relative errors near 1e-7 that grow over
// long solves, so the floor sits well above that noise; FP64 keeps the classic 1e-9.
template <typename T>
__device__ __forceinline__ double bicg_rho_floor() { return sizeof(T) == 4 ? kRhoFloorF32 : 1e-9; }

// Tests at the start of iteration i (>= 1) from the partial sums tot = ((rhat, r), |r|^2)
// of iteration i - 1: the same rules as the unfused finalize.
__device__ BicgStart bicg_start(const double tot[2], const KrylovScalars *sc, int i, double rho_floor) {
    const int q = (i - 1) & 1;
    BicgStart b;
    b.r2 = tot[1];
    b.nan = !isfinite(tot[0]) || !isfinite(tot[1]);
    b.conv = !b.nan && tot[1] <= sc->tol2;
    b.div = !b.nan && !b.conv && tot[1] > 1e12 * sc->bnorm2;
    const double rh2 = sc->rh2_pp[q], rmin2 = sc->rmin2_pp[q];
    // (rhat, r) lost its size relative to |rhat||r|, omega vanished, or the residual
    // grew 1000x above its best value: restart from the current r
    b.restart = !(fabs(tot[0]) > rho_floor * sqrt(rh2 * tot[1])) || sc->omega_pp[q] == 0.0 || tot[1] > 1e6 * rmin2;
    b.rho = b.restart ? tot[1] : tot[0];
    b.rh2 = b.restart ? tot[1] : rh2;
    b.rmin2 = fmin(rmin2, tot[1]);
    return b;
}

__device__ __forceinline__ void bicg_publish_start(const BicgStart &b, KrylovScalars *sc, int i) {
    sc->its = i;
    sc->rnorm2 = b.r2;
    if (b.nan) sc->breakdown = 2;
    else if (b.conv) sc->converged = 1;
    else if (b.div) sc->breakdown = 1;
}

// FOLD: the point-Jacobi scaling sits in the stored operator (K D^{-1}, see
// k_scale_columns), so the SpMV inputs are p and s themselves and ph, sh are not written.
template <typename T, bool FOLD = false>
__global__ __launch_bounds__(kThreads) void k_bicg_p_fused(int64_t N, int it, const T *__restrict__ r,
                                                           T *__restrict__ p, const T *__restrict__ v,
                                                           T *__restrict__ ph, T *__restrict__ rh,
                                                           const T *__restrict__ dinv,
                                                           const double *__restrict__ xr_partials, int xr_count,
                                                           KrylovScalars *sc) {
    if (stopped(sc)) return;
    bool restart = false;
    double beta = 0.0, omega = 0.0;
    if (it > 0) {
        double tot[2];
        sum_partials<2>(xr_partials, xr_count, tot);
        const BicgStart b = bicg_start(tot, sc, it, bicg_rho_floor<T>());
        const int q = (it - 1) & 1;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            bicg_publish_start(b, sc, it);
            sc->rho_old = sc->rho_pp[q];
            sc->rho = b.rho;
            sc->rho_pp[it & 1] = b.rho;
            sc->rh2_pp[it & 1] = b.rh2;
            sc->rmin2_pp[it & 1] = b.rmin2;
            if (b.restart) sc->restart_at = it;
        }
        if (b.nan || b.conv || b.div) return;
        restart = b.restart;
        omega = sc->omega_pp[q];
        if (!restart) beta = (b.rho / sc->rho_pp[q]) * (sc->alpha_pp[q] / omega);
    }
    const T bt = T(beta), om = T(omega);
    using V = Vec16<T>;
    constexpr int W = V::W;
    const int64_t NV = N / W;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < NV; i += int64_t(gridDim.x) * kThreads) {
        const typename V::type rv = V::ld(r, i);
        const typename V::type pv = restart ? rv : rv + bt * (V::ld(p, i) - om * V::ld(v, i));
        V::st(p, i, pv);
        if (!FOLD) V::st(ph, i, V::ld(dinv, i) * pv);
        if (restart) V::st(rh, i, rv);
    }
    if (blockIdx.x == 0)
        for (int64_t i = NV * W + threadIdx.x; i < N; i += kThreads) {
            const T ri = r[i];
            const T pi = restart ? ri : ri + bt * (p[i] - om * v[i]);
            p[i] = pi;
            if (!FOLD) ph[i] = dinv[i] * pi;
            if (restart) rh[i] = ri;
        }
}

template <typename T, bool FOLD = false>
__global__ __launch_bounds__(kThreads) void k_bicg_s_fused(int64_t N, int it, const T *__restrict__ r,
                                                           const T *__restrict__ v, T *__restrict__ s,
                                                           T *__restrict__ sh, const T *__restrict__ dinv,
                                                           const double *__restrict__ sp_partials, int sp_count,
                                                           KrylovScalars *sc) {
    if (stopped(sc)) return;
    double tot[1];
    sum_partials<1>(sp_partials, sp_count, tot);
    if (!(tot[0] != 0.0) || !isfinite(tot[0])) {  // (rhat, v) vanished
        if (blockIdx.x == 0 && threadIdx.x == 0) sc->breakdown = 1;
        return;
    }
    const double alpha = sc->rho_pp[it & 1] / tot[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->alpha_pp[it & 1] = alpha;
        sc->alpha = alpha;
    }
    const T al = T(alpha);
    using V = Vec16<T>;
    constexpr int W = V::W;
    const int64_t NV = N / W;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < NV; i += int64_t(gridDim.x) * kThreads) {
        const typename V::type sv = V::ld(r, i) - al * V::ld(v, i);
        V::st(s, i, sv);
        if (!FOLD) V::st(sh, i, V::ld(dinv, i) * sv);
    }
    if (blockIdx.x == 0)
        for (int64_t i = NV * W + threadIdx.x; i < N; i += kThreads) {
            const T si = r[i] - al * v[i];
            s[i] = si;
            if (!FOLD) sh[i] = dinv[i] * si;
        }
}

template <typename T, bool FOLD = false>
__global__ __launch_bounds__(kThreads) void k_bicg_xr_fused(int64_t N, int it, T *__restrict__ x, T *__restrict__ r,
                                                            const T *__restrict__ rh, const T *__restrict__ ph,
                                                            const T *__restrict__ s, const T *__restrict__ sh,
                                                            const T *__restrict__ t,
                                                            const double *__restrict__ sp_partials, int sp_count,
                                                            double *xr_partials, KrylovScalars *sc) {
    if (stopped(sc)) return;
    double tot[3];  // (t, s), (t, t), (s, s)
    sum_partials<3>(sp_partials, sp_count, tot);
    double omega = (tot[1] > 0.0 && isfinite(tot[1])) ? tot[0] / tot[1] : 0.0;
    const double om_lim = bicg_omega_limit<T>();
    if (om_lim > 0.0 && omega != 0.0 && tot[2] > 0.0) {
        const double c = fabs(tot[0]) / sqrt(tot[1] * tot[2]);
        if (c < om_lim) omega *= om_lim / c;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->omega_pp[it & 1] = omega;
        sc->omega = omega;
    }
    const T al = T(sc->alpha_pp[it & 1]), om = T(omega);
    double d0 = 0.0, d1 = 0.0;
    using V = Vec16<T>;
    constexpr int W = V::W;
    const int64_t NV = N / W;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < NV; i += int64_t(gridDim.x) * kThreads) {
        const typename V::type sv = V::ld(s, i);
        V::st(x, i, V::ld(x, i) + al * V::ld(ph, i) + om * (FOLD ? sv : V::ld(sh, i)));
        const typename V::type rv = sv - om * V::ld(t, i);
        const typename V::type hv = V::ld(rh, i);
        V::st(r, i, rv);
#pragma unroll
        for (int c = 0; c < W; ++c) {
            d0 += double(hv[c]) * double(rv[c]);
            d1 += double(rv[c]) * double(rv[c]);
        }
    }
    if (blockIdx.x == 0)
        for (int64_t i = NV * W + threadIdx.x; i < N; i += kThreads) {
            const T si = s[i];
            x[i] += al * ph[i] + om * (FOLD ? si : sh[i]);
            const T ri = si - om * t[i];
            r[i] = ri;
            d0 += double(rh[i]) * double(ri);
            d1 += double(ri) * double(ri);
        }
    double vv[2] = {d0, d1};
    block_store_partials<2>(vv, xr_partials);
}

// Convergence, divergence and NaN flags after iteration it - 1 (one block; the next
// p-kernel repeats the same tests and also takes the restart decision).
__global__ __launch_bounds__(kThreads) void k_bicg_check(int it, const double *__restrict__ xr_partials,
                                                         int xr_count, KrylovScalars *sc, double rho_floor) {
    if (stopped(sc) || it == 0) return;
    double tot[2];
    sum_partials<2>(xr_partials, xr_count, tot);
    const BicgStart b = bicg_start(tot, sc, it, rho_floor);
    if (threadIdx.x == 0) bicg_publish_start(b, sc, it);
}

// ------------------------------------------------------------------ block Jacobi variants
// The same vector kernels with the node-block preconditioner: one thread per node,
// z_n = M_n r_n with M_n the inverse of node n's ND x ND diagonal block (row-major).
template <int ND, typename T>
__device__ __forceinline__ void node_block_apply(const T *__restrict__ M, int64_t n, const T r[ND], T z[ND]) {
    const T *m = M + int64_t(ND) * ND * n;
#pragma unroll
    for (int i = 0; i < ND; ++i) {
        T a = T(0);
#pragma unroll
        for (int c = 0; c < ND; ++c) a += m[i * ND + c] * r[c];
        z[i] = a;
    }
}

template <int ND, typename T>
__global__ __launch_bounds__(kThreads) void k_kry_init_bj(int64_t Nn, int cg, const T *__restrict__ b,
                                                          T *__restrict__ x, T *__restrict__ r, T *__restrict__ rh,
                                                          T *__restrict__ p, T *__restrict__ v,
                                                          const T *__restrict__ M, double *partials) {
    double d0 = 0.0, d1 = 0.0;
    for (int64_t n = int64_t(blockIdx.x) * kThreads + threadIdx.x; n < Nn; n += int64_t(gridDim.x) * kThreads) {
        T bi[ND], zi[ND];
#pragma unroll
        for (int c = 0; c < ND; ++c) bi[c] = b[ND * n + c];
        if (cg) node_block_apply<ND>(M, n, bi, zi);
#pragma unroll
        for (int c = 0; c < ND; ++c) {
            const int64_t i = ND * n + c;
            x[i] = T(0);
            r[i] = bi[c];
            if (cg) {
                rh[i] = zi[c];
                p[i] = zi[c];
                d0 += double(bi[c]) * double(zi[c]);
            } else {
                rh[i] = bi[c];
                p[i] = T(0);
                v[i] = T(0);
                d0 += double(bi[c]) * double(bi[c]);
            }
            d1 += double(bi[c]) * double(bi[c]);
        }
    }
    double vv[2] = {d0, d1};
    block_store_partials<2>(vv, partials);
}

template <int ND, typename T>
__global__ __launch_bounds__(kThreads) void k_cg_xr_fused_bj(int64_t Nn, T *__restrict__ x, T *__restrict__ r,
                                                             T *__restrict__ z, const T *__restrict__ p,
                                                             const T *__restrict__ q, const T *__restrict__ M,
                                                             const double *__restrict__ pq_partials, int pq_count,
                                                             double *partials, KrylovScalars *sc, int it) {
    if (stopped(sc)) return;
    double pq[1];
    sum_partials<1>(pq_partials, pq_count, pq);
    if (!(pq[0] > 0.0) || !isfinite(pq[0])) {
        if (blockIdx.x == 0 && threadIdx.x == 0) sc->breakdown = 1;
        return;
    }
    const double alpha = sc->rho_pp[it & 1] / pq[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->alpha = alpha;
    const T al = T(alpha);
    double d0 = 0.0, d1 = 0.0;
    for (int64_t n = int64_t(blockIdx.x) * kThreads + threadIdx.x; n < Nn; n += int64_t(gridDim.x) * kThreads) {
        T ri[ND], zi[ND];
#pragma unroll
        for (int c = 0; c < ND; ++c) {
            const int64_t i = ND * n + c;
            x[i] += al * p[i];
            ri[c] = r[i] - al * q[i];
            r[i] = ri[c];
        }
        node_block_apply<ND>(M, n, ri, zi);
#pragma unroll
        for (int c = 0; c < ND; ++c) {
            z[ND * n + c] = zi[c];
            d0 += double(ri[c]) * double(zi[c]);
            d1 += double(ri[c]) * double(ri[c]);
        }
    }
    double v[2] = {d0, d1};
    block_store_partials<2>(v, partials);
}

template <int ND, typename T>
__global__ __launch_bounds__(kThreads) void k_bicg_p_bj(int64_t Nn, const T *__restrict__ r, T *__restrict__ p,
                                                        const T *__restrict__ v, T *__restrict__ ph,
                                                        T *__restrict__ rh, const T *__restrict__ M,
                                                        const KrylovScalars *sc) {
    if (stopped(sc)) return;
    const bool restart = sc->restart_at == sc->its;
    const double beta = (sc->its == 0 || restart) ? 0.0 : (sc->rho / sc->rho_old) * (sc->alpha / sc->omega);
    const T bt = T(beta), om = T(sc->omega);
    for (int64_t n = int64_t(blockIdx.x) * kThreads + threadIdx.x; n < Nn; n += int64_t(gridDim.x) * kThreads) {
        T pi[ND], zi[ND];
#pragma unroll
        for (int c = 0; c < ND; ++c) {
            const int64_t i = ND * n + c;
            const T ri = r[i];
            pi[c] = restart ? ri : ri + bt * (p[i] - om * v[i]);
            p[i] = pi[c];
            if (restart) rh[i] = ri;
        }
        node_block_apply<ND>(M, n, pi, zi);
#pragma unroll
        for (int c = 0; c < ND; ++c) ph[ND * n + c] = zi[c];
    }
}

template <int ND, typename T>
__global__ __launch_bounds__(kThreads) void k_bicg_s_bj(int64_t Nn, const T *__restrict__ r, const T *__restrict__ v,
                                                        T *__restrict__ s, T *__restrict__ sh,
                                                        const T *__restrict__ M, const KrylovScalars *sc) {
    if (stopped(sc)) return;
    const T al = T(sc->alpha);
    for (int64_t n = int64_t(blockIdx.x) * kThreads + threadIdx.x; n < Nn; n += int64_t(gridDim.x) * kThreads) {
        T si[ND], zi[ND];
#pragma unroll
        for (int c = 0; c < ND; ++c) {
            const int64_t i = ND * n + c;
            si[c] = r[i] - al * v[i];
            s[i] = si[c];
        }
        node_block_apply<ND>(M, n, si, zi);
#pragma unroll
        for (int c = 0; c < ND; ++c) sh[ND * n + c] = zi[c];
    }
}

// Krylov start with x0 = 0: r = rh = b, p = v = 0 (BiCGSTAB) or r = b, z = Dinv b,
// p = z (CG); reduces |b|^2 and the first rho.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_kry_init(int64_t N, int cg, const T *__restrict__ b,
                                                       T *__restrict__ x, T *__restrict__ r, T *__restrict__ rh,
                                                       T *__restrict__ p, T *__restrict__ v,
                                                       const T *__restrict__ dinv, double *partials,
                                                       KrylovScalars *sc, double rtol) {
    double d0 = 0.0, d1 = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < N; i += int64_t(gridDim.x) * kThreads) {
        T bi = b[i];
        x[i] = T(0);
        r[i] = bi;
        if (cg) {
            T zi = dinv[i] * bi;
            rh[i] = zi;  // z
            p[i] = zi;
            d0 += double(bi) * double(zi);
        } else {
            rh[i] = bi;
            p[i] = T(0);
            v[i] = T(0);
            d0 += double(bi) * double(bi);
        }
        d1 += double(bi) * double(bi);
    }
    double vv[2] = {d0, d1};
    block_store_partials<2>(vv, partials);
}

__global__ __launch_bounds__(kThreads) void k_fin_init(int G, const double *__restrict__ partials,
                                                       KrylovScalars *sc, double rtol) {
    double tot[2];
    sum_partials<2>(partials, G, tot);
    if (threadIdx.x == 0) {
        sc->rho = tot[0];
        sc->rho_pp[0] = tot[0];
        sc->rho_pp[1] = tot[0];
        sc->rho_old = 1.0;
        sc->alpha = 1.0;
        sc->omega = 1.0;
        sc->beta = 0.0;
        sc->bnorm2 = tot[1];
        sc->rnorm2 = tot[1];
        sc->tol2 = rtol * rtol * tot[1];
        sc->its = 0;
        sc->rh2 = tot[1];
        sc->rmin2 = tot[1];
        sc->restart_at = -1;
        sc->alpha_pp[0] = sc->alpha_pp[1] = 1.0;
        sc->omega_pp[0] = sc->omega_pp[1] = 1.0;
        sc->rh2_pp[0] = sc->rh2_pp[1] = tot[1];
        sc->rmin2_pp[0] = sc->rmin2_pp[1] = tot[1];
        sc->breakdown = isfinite(tot[1]) ? 0 : 2;
        sc->converged = (tot[1] == 0.0) ? 1 : 0;
    }
}

// ------------------------------------------------------------------ vector helpers
__global__ __launch_bounds__(kThreads) void k_dot_self(int64_t N, const double *__restrict__ r, double *partials) {
    double d = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < N; i += int64_t(gridDim.x) * kThreads)
        d += r[i] * r[i];
    double v[1] = {d};
    block_store_partials<1>(v, partials);
}

__global__ __launch_bounds__(kThreads) void k_fin_dot(int G, const double *__restrict__ partials, double *out) {
    double tot[1];
    sum_partials<1>(partials, G, tot);
    if (threadIdx.x == 0) *out = tot[0];
}

template <typename TO, typename TI>
__global__ __launch_bounds__(kThreads) void k_scale_cast(int64_t n, const TI *__restrict__ in, TO *__restrict__ out,
                                                         double alpha) {
    int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) out[i] = TO(alpha * double(in[i]));
}

template <typename TI>
__global__ __launch_bounds__(kThreads) void k_axpy_f64(int64_t n, const TI *__restrict__ x, double *__restrict__ y) {
    int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) y[i] += double(x[i]);
}

__global__ __launch_bounds__(kThreads) void k_set_dirichlet(int64_t n, const uint8_t *__restrict__ mask,
                                                            double *__restrict__ u, const double *__restrict__ u0,
                                                            const double *__restrict__ g, double lam) {
    int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n && mask[i]) u[i] = u0[i] + lam * (g[i] - u0[i]);
}

__global__ __launch_bounds__(kThreads) void k_dirichlet_increment(int64_t n, const uint8_t *__restrict__ mask,
                                                                  const double *__restrict__ u,
                                                                  const double *__restrict__ u0,
                                                                  const double *__restrict__ g, double lam,
                                                                  double *__restrict__ delta) {
    int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) delta[i] = mask[i] ? (u0[i] + lam * (g[i] - u0[i]) - u[i]) : 0.0;
}

__global__ __launch_bounds__(kThreads) void k_neg_sum(int64_t n, const double *__restrict__ a,
                                                      const double *__restrict__ b, double *__restrict__ out) {
    int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) out[i] = -(a[i] + b[i]);
}

__global__ __launch_bounds__(kThreads) void k_mask_copy(int64_t n, const uint8_t *__restrict__ mask,
                                                        const double *__restrict__ in, double *__restrict__ out) {
    int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) out[i] = (mask && mask[i]) ? 0.0 : in[i];
}

__global__ __launch_bounds__(kThreads) void k_sub(int64_t n, const double *__restrict__ a,
                                                  const double *__restrict__ b, double *__restrict__ out) {
    int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) out[i] = a[i] - b[i];
}

// ------------------------------------------------------------------ pattern export
template <int ND>
__global__ __launch_bounds__(kThreads) void k_export_cols(int64_t nnzb, const int64_t *__restrict__ node_ptr,
                                                          const int32_t *__restrict__ node_nb,
                                                          const int32_t *__restrict__ blk_row,
                                                          const int32_t *__restrict__ mirror,
                                                          const int64_t *__restrict__ row_ptr,
                                                          int32_t *__restrict__ col_idx, int32_t *__restrict__ tperm) {
    int64_t t = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (t >= nnzb * ND * ND) return;
    int64_t kb = t / (ND * ND);
    int r = int(t - kb * ND * ND);
    int i = r / ND, k = r % ND;
    int64_t n = blk_row[kb], m = node_nb[kb];
    int64_t pos = row_ptr[ND * n + i] + ND * (kb - node_ptr[n]) + k;
    if (col_idx) col_idx[pos] = int32_t(ND * m + k);
    if (tperm) tperm[pos] = int32_t(row_ptr[ND * m + k] + ND * (mirror[kb] - node_ptr[m]) + i);
}

template <int ND>
__global__ __launch_bounds__(kThreads) void k_export_slots(int64_t Ne, const int32_t *__restrict__ conn,
                                                           const int32_t *__restrict__ bslot,
                                                           const int64_t *__restrict__ node_ptr,
                                                           const int64_t *__restrict__ row_ptr,
                                                           int32_t *__restrict__ slot) {
    constexpr int Nd = 8 * ND;
    int64_t t = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (t >= Ne * Nd * Nd) return;
    int64_t e = t / (Nd * Nd);
    int r = int(t - e * Nd * Nd);
    int p = r / Nd, q = r % Nd;
    int a = p / ND, i = p % ND, b = q / ND, k = q % ND;
    int64_t n = conn[8 * e + a];
    int64_t kb = bslot[e * 64 + a * 8 + b];
    slot[t] = int32_t(row_ptr[ND * n + i] + ND * (kb - node_ptr[n]) + k);
}

template <int ND>
__global__ __launch_bounds__(kThreads) void k_export_diag(int64_t N, const int32_t *__restrict__ bdiag,
                                                          const int64_t *__restrict__ node_ptr,
                                                          const int64_t *__restrict__ row_ptr,
                                                          int64_t *__restrict__ diag) {
    int64_t d = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (d >= N) return;
    int64_t n = d / ND;
    int i = int(d - n * ND);
    diag[d] = row_ptr[d] + ND * (bdiag[n] - node_ptr[n]) + i;
}

}  // namespace

int krylov_grid(const fem_handle *h) {
    // Largest persistent grid: 8 resident blocks of 4 waves per CU (8 waves per SIMD).
    return 8 * h->num_cus;
}

// Grid of the fused CG vector kernels: every block also sums the previous kernel's
// partials, so fewer, fuller blocks (4 per CU) keep that redundant work small.
static int krylov_vec_grid(const fem_handle *h) { return 4 * h->num_cus; }

// Persistent grid of a kernel: the blocks that can be resident at once (runtime
// occupancy of this kernel variant), a multiple of the 8 XCDs.
template <typename K>
static int resident_grid(const fem_handle *h, K kernel) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int G = std::min(per_cu, 8) * h->num_cus;
    return std::max(8, (G / 8) * 8);
}

size_t krylov_partials_bytes(const fem_handle *h) { return size_t(krylov_grid(h)) * 3 * sizeof(double); }

template <int ND, int G, typename T>
static void spmv_launch(const fem_handle *h, const T *values, int transpose, const T *x, T *y, T alpha, T beta,
                        hipStream_t s) {
    const Graph &g = h->g;
    dim3 grid(grid_for(g.Nn, kThreads / G));
    if (transpose)
        hipLaunchKernelGGL((k_spmv<ND, G, true, T>), grid, dim3(kThreads), 0, s, g.Nn, g.node_ptr, g.node_nb, g.mirror,
                           values, x, y, alpha, beta);
    else if (g.node_dnb)
        hipLaunchKernelGGL((k_spmv_nodes<ND, spmv_batch<ND, T>(), 0, T, true>),
                           dim3(resident_grid(h, k_spmv_nodes<ND, spmv_batch<ND, T>(), 0, T, true>)),
                           dim3(kThreads), 0, s, g.Nn, g.node_ptr, g.node_nb, g.node_dnb, values, x, y, nullptr,
                           alpha, beta, nullptr, nullptr, 0, int(g.max_deg > kSpmvGroup));
    else
        hipLaunchKernelGGL((k_spmv_nodes<ND, spmv_batch<ND, T>(), 0, T, false>),
                           dim3(resident_grid(h, k_spmv_nodes<ND, spmv_batch<ND, T>(), 0, T, false>)),
                           dim3(kThreads), 0, s, g.Nn, g.node_ptr, g.node_nb, g.node_dnb, values, x, y, nullptr,
                           alpha, beta, nullptr, nullptr, 0, int(g.max_deg > kSpmvGroup));
}

#define FEM_DISPATCH_GROUP(G_RT, ND_RT, CALL)                                                      \
    do {                                                                                           \
        if ((ND_RT) == 1) {                                                                        \
            constexpr int ND = 1;                                                                  \
            switch (G_RT) {                                                                        \
            case 4: { constexpr int G = 4; CALL; break; }                                          \
            case 8: { constexpr int G = 8; CALL; break; }                                          \
            case 16: { constexpr int G = 16; CALL; break; }                                        \
            default: { constexpr int G = 32; CALL; break; }                                        \
            }                                                                                      \
        } else {                                                                                   \
            constexpr int ND = 3;                                                                  \
            switch (G_RT) {                                                                        \
            case 4: { constexpr int G = 4; CALL; break; }                                          \
            case 8: { constexpr int G = 8; CALL; break; }                                          \
            case 16: { constexpr int G = 16; CALL; break; }                                        \
            default: { constexpr int G = 32; CALL; break; }                                        \
            }                                                                                      \
        }                                                                                          \
    } while (0)

template <typename T>
void launch_spmv(const fem_handle *h, const T *values, int transpose, const T *x, T *y, T alpha, T beta,
                 hipStream_t s) {
    const Graph &g = h->g;
    if (g.Nn == 0) return;
    FEM_DISPATCH_GROUP(h->spmv_group, g.nd, (spmv_launch<ND, G, T>(h, values, transpose, x, y, alpha, beta, s)));
    FEM_HIP(hipGetLastError());
}

template <typename T>
void launch_spmv_sym(const fem_handle *h, const T *values, const T *x, T *y, T alpha, T beta, hipStream_t s) {
    const Graph &g = h->g;
    if (g.Nn == 0) return;
#define FEM_SYM0(ND)                                                                                            \
    hipLaunchKernelGGL((k_spmv_sym<ND, 4, 0, T>), dim3(resident_grid(h, k_spmv_sym<ND, 4, 0, T>)), dim3(kThreads),  \
                       0, s, g.Nn, g.node_ptr, g.up_base, g.node_nb, g.lo_val, values, x, y, nullptr, alpha, beta,  \
                       nullptr, nullptr, 0)
    if (g.nd == 1) FEM_SYM0(1);
    else FEM_SYM0(3);
#undef FEM_SYM0
    FEM_HIP(hipGetLastError());
}
template void launch_spmv_sym<float>(const fem_handle *, const float *, const float *, float *, float, float,
                                     hipStream_t);
template void launch_spmv_sym<double>(const fem_handle *, const double *, const double *, double *, double, double,
                                      hipStream_t);

template <typename T>
void kry_bicg_init(const fem_handle *h, const KrylovVecs<T> &k, const T *b, double rtol, hipStream_t s) {
    if (k.bj) {
        if (h->g.nd == 1)
            hipLaunchKernelGGL((k_kry_init_bj<1, T>), dim3(krylov_grid(h)), dim3(kThreads), 0, s, h->g.Nn, 0, b, k.x,
                               k.r, k.rh, k.p, k.v, k.dinv, k.partials);
        else
            hipLaunchKernelGGL((k_kry_init_bj<3, T>), dim3(krylov_grid(h)), dim3(kThreads), 0, s, h->g.Nn, 0, b, k.x,
                               k.r, k.rh, k.p, k.v, k.dinv, k.partials);
    } else {
        hipLaunchKernelGGL((k_kry_init<T>), dim3(krylov_grid(h)), dim3(kThreads), 0, s, h->g.N, 0, b, k.x, k.r, k.rh,
                           k.p, k.v, k.dinv, k.partials, k.sc, rtol);
    }
    hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(kThreads), 0, s, krylov_grid(h), k.partials, k.sc, rtol);
    FEM_HIP(hipGetLastError());
}

template <typename T>
void kry_cg_init(const fem_handle *h, const KrylovVecs<T> &k, const T *b, double rtol, hipStream_t s) {
    // CG keeps z in the slot of rh
    if (k.bj) {
        if (h->g.nd == 1)
            hipLaunchKernelGGL((k_kry_init_bj<1, T>), dim3(krylov_grid(h)), dim3(kThreads), 0, s, h->g.Nn, 1, b, k.x,
                               k.r, k.rh, k.p, k.v, k.dinv, k.partials);
        else
            hipLaunchKernelGGL((k_kry_init_bj<3, T>), dim3(krylov_grid(h)), dim3(kThreads), 0, s, h->g.Nn, 1, b, k.x,
                               k.r, k.rh, k.p, k.v, k.dinv, k.partials);
    } else {
        hipLaunchKernelGGL((k_kry_init<T>), dim3(krylov_grid(h)), dim3(kThreads), 0, s, h->g.N, 1, b, k.x, k.r, k.rh,
                           k.p, k.v, k.dinv, k.partials, k.sc, rtol);
    }
    hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(kThreads), 0, s, krylov_grid(h), k.partials, k.sc, rtol);
    FEM_HIP(hipGetLastError());
}

// Launches the fused SpMV (partials into k.partials) and, unless the caller folds it
// into its next kernel, the one-block finalize; returns the SpMV grid size.
template <int ND, int P, int MODE, typename T, typename TV = T>
static int kry_spmv_launch(const fem_handle *h, const T *x, T *y, const T *w0, const KrylovVecs<T> &k, int cg,
                           const TV *values, bool finalize, hipStream_t s) {
    const Graph &g = h->g;
    int G;
    if (k.layout == LAYOUT_SYM) {
        if constexpr (std::is_same<T, TV>::value) {
            G = resident_grid(h, k_spmv_sym<ND, P, MODE, T>);
            hipLaunchKernelGGL((k_spmv_sym<ND, P, MODE, T>), dim3(G), dim3(kThreads), 0, s, g.Nn, g.node_ptr,
                               g.up_base, g.node_nb, g.lo_val, values, x, y, w0, T(1), T(0), k.partials, k.sc, cg);
        } else {
            throw Error(FEM_EINVAL, "the symmetric block layout takes values of the vector type");
        }
    } else if (g.node_dnb) {
        G = resident_grid(h, k_spmv_nodes<ND, P, MODE, T, true, TV>);
        hipLaunchKernelGGL((k_spmv_nodes<ND, P, MODE, T, true, TV>), dim3(G), dim3(kThreads), 0, s, g.Nn,
                           g.node_ptr, g.node_nb, g.node_dnb, values, x, y, w0, T(1), T(0), k.partials, k.sc, cg,
                           int(g.max_deg > kSpmvGroup));
    } else {
        G = resident_grid(h, k_spmv_nodes<ND, P, MODE, T, false, TV>);
        hipLaunchKernelGGL((k_spmv_nodes<ND, P, MODE, T, false, TV>), dim3(G), dim3(kThreads), 0, s, g.Nn,
                           g.node_ptr, g.node_nb, g.node_dnb, values, x, y, w0, T(1), T(0), k.partials, k.sc, cg,
                           int(g.max_deg > kSpmvGroup));
    }
    if (finalize) {
        if (MODE == 1) hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(kThreads), 0, s, G, k.partials, k.sc, cg);
        else hipLaunchKernelGGL(k_fin_omega, dim3(1), dim3(kThreads), 0, s, G, k.partials, k.sc);
    }
    return G;
}

// The Krylov SpMV on the solve's operator: k.A, or the FP32 tangent k.A32 under FP64
// vectors (products and sums in FP64).
template <typename T, int MODE>
static int kry_spmv(const fem_handle *h, const T *x, T *y, const T *w0, const KrylovVecs<T> &k, int cg,
                    const T *values, hipStream_t s, bool finalize = true) {
    if constexpr (sizeof(T) == 8) {
        if (k.A32) {
            if (h->g.nd == 1)
                return kry_spmv_launch<1, spmv_batch<1, float, T>(), MODE, T, float>(h, x, y, w0, k, cg, k.A32,
                                                                                     finalize, s);
            return kry_spmv_launch<3, spmv_batch<3, float, T>(), MODE, T, float>(h, x, y, w0, k, cg, k.A32, finalize,
                                                                                 s);
        }
    }
    if (h->g.nd == 1) return kry_spmv_launch<1, spmv_batch<1, T>(), MODE, T>(h, x, y, w0, k, cg, values, finalize, s);
    return kry_spmv_launch<3, spmv_batch<3, T>(), MODE, T>(h, x, y, w0, k, cg, values, finalize, s);
}

template <typename T>
int kry_spmv_q(const fem_handle *h, const KrylovVecs<T> &k, hipStream_t s) {
    return kry_spmv<T, 1>(h, k.p, k.v, k.p, k, 1, k.A, s, false);
}

int krylov_vec_grid_of(const fem_handle *h) { return krylov_vec_grid(h); }

// p = z + beta p from the (r, z) and |r|^2 partials in k.partials2 (krylov_vec_grid of them).
template <typename T>
void kry_cg_p_update(const fem_handle *h, const KrylovVecs<T> &k, int it, hipStream_t s) {
    const int G = krylov_vec_grid(h);
    hipLaunchKernelGGL((k_cg_p_fused<T>), dim3(G), dim3(kThreads), 0, s, h->g.N, k.rh, k.p, k.partials2, G, k.sc, it);
    FEM_HIP(hipGetLastError());
}

// y = alpha K x + beta y inside a Krylov loop: skipped once sc reports convergence.
template <typename T>
void launch_spmv_sc(const fem_handle *h, const T *values, const T *x, T *y, T alpha, T beta, const KrylovScalars *sc,
                    hipStream_t s) {
    const Graph &g = h->g;
    if (g.N == 0) return;
    KrylovScalars *scw = const_cast<KrylovScalars *>(sc);
#define FEM_SPMV_SC(ND, D16)                                                                                       \
    hipLaunchKernelGGL((k_spmv_nodes<ND, spmv_batch<ND, T>(), 0, T, D16>),                                         \
                       dim3(resident_grid(h, k_spmv_nodes<ND, spmv_batch<ND, T>(), 0, T, D16>)), dim3(kThreads), 0, \
                       s, g.Nn, g.node_ptr, g.node_nb, g.node_dnb, values, x, y, nullptr, alpha, beta, nullptr,   \
                       scw, 0, int(g.max_deg > kSpmvGroup))
    if (g.nd == 1) {
        if (g.node_dnb) FEM_SPMV_SC(1, true);
        else FEM_SPMV_SC(1, false);
    } else {
        if (g.node_dnb) FEM_SPMV_SC(3, true);
        else FEM_SPMV_SC(3, false);
    }
#undef FEM_SPMV_SC
    FEM_HIP(hipGetLastError());
}

template <typename T>
void kry_bicg_iter(const fem_handle *h, const KrylovVecs<T> &k, int it, hipStream_t s, hipEvent_t *ev) {
    const int64_t N = h->g.N;
    const T *A = k.A;
    const int64_t Nn = h->g.Nn;
    if (!k.bj) {
        dim3 grid(krylov_vec_grid(h)), blk(kThreads);
        // folded Jacobi: the operator is K D^{-1} and the SpMVs take p and s directly
        T *ph = k.fold ? k.p : k.ph, *sh = k.fold ? k.s : k.sh;
        if (k.fold)
            hipLaunchKernelGGL((k_bicg_p_fused<T, true>), grid, blk, 0, s, N, it, k.r, k.p, k.v, ph, k.rh, k.dinv,
                               k.partials2, int(grid.x), k.sc);
        else
            hipLaunchKernelGGL((k_bicg_p_fused<T, false>), grid, blk, 0, s, N, it, k.r, k.p, k.v, ph, k.rh, k.dinv,
                               k.partials2, int(grid.x), k.sc);
        if (ev) FEM_HIP(hipEventRecord(ev[0], s));
        int G = kry_spmv<T, 1>(h, ph, k.v, k.rh, k, 0, A, s, false);
        if (ev) FEM_HIP(hipEventRecord(ev[1], s));
        if (k.fold)
            hipLaunchKernelGGL((k_bicg_s_fused<T, true>), grid, blk, 0, s, N, it, k.r, k.v, k.s, sh, k.dinv,
                               k.partials, G, k.sc);
        else
            hipLaunchKernelGGL((k_bicg_s_fused<T, false>), grid, blk, 0, s, N, it, k.r, k.v, k.s, sh, k.dinv,
                               k.partials, G, k.sc);
        if (ev) FEM_HIP(hipEventRecord(ev[2], s));
        G = kry_spmv<T, 2>(h, sh, k.t, k.s, k, 0, A, s, false);
        if (ev) FEM_HIP(hipEventRecord(ev[3], s));
        if (k.fold)
            hipLaunchKernelGGL((k_bicg_xr_fused<T, true>), grid, blk, 0, s, N, it, k.x, k.r, k.rh, ph, k.s, sh, k.t,
                               k.partials, G, k.partials2, k.sc);
        else
            hipLaunchKernelGGL((k_bicg_xr_fused<T, false>), grid, blk, 0, s, N, it, k.x, k.r, k.rh, ph, k.s, sh, k.t,
                               k.partials, G, k.partials2, k.sc);
        FEM_HIP(hipGetLastError());
        return;
    }
    // block Jacobi: separate vector kernels with one-block finalizes
    dim3 grid(krylov_grid(h)), blk(kThreads);
    if (h->g.nd == 1) hipLaunchKernelGGL((k_bicg_p_bj<1, T>), grid, blk, 0, s, Nn, k.r, k.p, k.v, k.ph, k.rh, k.dinv, k.sc);
    else hipLaunchKernelGGL((k_bicg_p_bj<3, T>), grid, blk, 0, s, Nn, k.r, k.p, k.v, k.ph, k.rh, k.dinv, k.sc);
    if (ev) FEM_HIP(hipEventRecord(ev[0], s));
    kry_spmv<T, 1>(h, k.ph, k.v, k.rh, k, 0, A, s);
    if (ev) FEM_HIP(hipEventRecord(ev[1], s));
    if (h->g.nd == 1) hipLaunchKernelGGL((k_bicg_s_bj<1, T>), grid, blk, 0, s, Nn, k.r, k.v, k.s, k.sh, k.dinv, k.sc);
    else hipLaunchKernelGGL((k_bicg_s_bj<3, T>), grid, blk, 0, s, Nn, k.r, k.v, k.s, k.sh, k.dinv, k.sc);
    if (ev) FEM_HIP(hipEventRecord(ev[2], s));
    kry_spmv<T, 2>(h, k.sh, k.t, k.s, k, 0, A, s);
    if (ev) FEM_HIP(hipEventRecord(ev[3], s));
    hipLaunchKernelGGL((k_bicg_xr<T>), grid, blk, 0, s, N, k.x, k.r, k.rh, k.ph, k.s, k.sh, k.t, k.partials, k.sc);
    hipLaunchKernelGGL(k_fin_bicg_xr, dim3(1), blk, 0, s, int(grid.x), k.partials, k.sc);
    FEM_HIP(hipGetLastError());
}

template <typename T>
void kry_bicg_check(const fem_handle *h, const KrylovVecs<T> &k, int it, hipStream_t s) {
    if (k.bj) return;  // the unfused iteration finalizes its own scalars
    hipLaunchKernelGGL(k_bicg_check, dim3(1), dim3(kThreads), 0, s, it, k.partials2, krylov_vec_grid(h), k.sc,
                       sizeof(T) == 4 ? kRhoFloorF32 : 1e-9);
    FEM_HIP(hipGetLastError());
}

// One CG iteration in three kernels: q = K p with (p, q) partials; the x/r/z update
// with alpha taken from those partials; the p update with beta taken from the
// (r, z) partials.  The two partial buffers alternate so that no kernel overwrites
// partials that blocks of the same kernel are still reading.
template <typename T>
void kry_cg_iter(const fem_handle *h, const KrylovVecs<T> &k, int it, hipStream_t s, hipEvent_t *ev) {
    const int64_t N = h->g.N;
    dim3 grid(krylov_vec_grid(h)), blk(kThreads);
    const T *A = k.A;
    // slots: z = rh, q = v
    if (ev) FEM_HIP(hipEventRecord(ev[0], s));
    const int G = kry_spmv<T, 1>(h, k.p, k.v, k.p, k, 1, A, s, false);
    if (ev) FEM_HIP(hipEventRecord(ev[1], s));
    if (!k.bj)
        hipLaunchKernelGGL((k_cg_xr_fused<T>), grid, blk, 0, s, N, k.x, k.r, k.rh, k.p, k.v, k.dinv, k.partials, G,
                           k.partials2, k.sc, it);
    else if (h->g.nd == 1)
        hipLaunchKernelGGL((k_cg_xr_fused_bj<1, T>), grid, blk, 0, s, h->g.Nn, k.x, k.r, k.rh, k.p, k.v, k.dinv,
                           k.partials, G, k.partials2, k.sc, it);
    else
        hipLaunchKernelGGL((k_cg_xr_fused_bj<3, T>), grid, blk, 0, s, h->g.Nn, k.x, k.r, k.rh, k.p, k.v, k.dinv,
                           k.partials, G, k.partials2, k.sc, it);
    hipLaunchKernelGGL((k_cg_p_fused<T>), grid, blk, 0, s, N, k.rh, k.p, k.partials2, int(grid.x), k.sc, it);
    FEM_HIP(hipGetLastError());
}

template void kry_bicg_init<float>(const fem_handle *, const KrylovVecs<float> &, const float *, double, hipStream_t);
template void kry_bicg_init<double>(const fem_handle *, const KrylovVecs<double> &, const double *, double,
                                    hipStream_t);
template void kry_cg_init<float>(const fem_handle *, const KrylovVecs<float> &, const float *, double, hipStream_t);
template void kry_cg_init<double>(const fem_handle *, const KrylovVecs<double> &, const double *, double, hipStream_t);
template void kry_bicg_iter<float>(const fem_handle *, const KrylovVecs<float> &, int, hipStream_t, hipEvent_t *);
template void kry_bicg_iter<double>(const fem_handle *, const KrylovVecs<double> &, int, hipStream_t, hipEvent_t *);
template void kry_bicg_check<float>(const fem_handle *, const KrylovVecs<float> &, int, hipStream_t);
template void kry_bicg_check<double>(const fem_handle *, const KrylovVecs<double> &, int, hipStream_t);
template int kry_spmv_q<float>(const fem_handle *, const KrylovVecs<float> &, hipStream_t);
template int kry_spmv_q<double>(const fem_handle *, const KrylovVecs<double> &, hipStream_t);
template void kry_cg_p_update<float>(const fem_handle *, const KrylovVecs<float> &, int, hipStream_t);
template void kry_cg_p_update<double>(const fem_handle *, const KrylovVecs<double> &, int, hipStream_t);
template void launch_spmv_sc<float>(const fem_handle *, const float *, const float *, float *, float, float,
                                    const KrylovScalars *, hipStream_t);
template void launch_spmv_sc<double>(const fem_handle *, const double *, const double *, double *, double, double,
                                     const KrylovScalars *, hipStream_t);
template void kry_cg_iter<float>(const fem_handle *, const KrylovVecs<float> &, int, hipStream_t, hipEvent_t *);
template void kry_cg_iter<double>(const fem_handle *, const KrylovVecs<double> &, int, hipStream_t, hipEvent_t *);
template void launch_spmv<float>(const fem_handle *, const float *, int, const float *, float *, float, float,
                                 hipStream_t);
template void launch_spmv<double>(const fem_handle *, const double *, int, const double *, double *, double, double,
                                  hipStream_t);

void launch_norm2_free(const fem_handle *h, const double *r, double *partials, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_self, dim3(krylov_grid(h)), dim3(kThreads), 0, s, h->g.N, r, partials);
    hipLaunchKernelGGL(k_fin_dot, dim3(1), dim3(kThreads), 0, s, krylov_grid(h), partials, out);
    FEM_HIP(hipGetLastError());
}

template <typename TO, typename TI>
void launch_scale_cast(const TI *in, TO *out, double alpha, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL((k_scale_cast<TO, TI>), dim3(grid_for(n, kThreads)), dim3(kThreads), 0, s, n, in, out, alpha);
    FEM_HIP(hipGetLastError());
}
template void launch_scale_cast<float, double>(const double *, float *, double, int64_t, hipStream_t);
template void launch_scale_cast<double, double>(const double *, double *, double, int64_t, hipStream_t);
template void launch_scale_cast<double, float>(const float *, double *, double, int64_t, hipStream_t);

// Right point-Jacobi scaling folded into the stored tangent: every value of column
// dof j is multiplied by dinv[j], so BiCGSTAB runs on K D^{-1} (the same iterates as
// right preconditioning with D, without the D^{-1} p and D^{-1} s vectors), and its
// iterate y maps back as x = D^{-1} y.  One 32-lane group per node, lane = block.
template <int ND, typename T>
__global__ __launch_bounds__(kThreads) void k_scale_columns(int64_t Nn, const int64_t *__restrict__ node_ptr,
                                                            const int32_t *__restrict__ node_nb,
                                                            T *__restrict__ values, const T *__restrict__ dinv) {
    constexpr int G = 32;
    const int lane = threadIdx.x % G;
    for (int64_t n = (int64_t(blockIdx.x) * kThreads + threadIdx.x) / G; n < Nn;
         n += int64_t(gridDim.x) * (kThreads / G)) {
        const int64_t b0 = node_ptr[n];
        const int deg = int(node_ptr[n + 1] - b0);
        for (int l = lane; l < deg; l += G) {
            const int64_t m = node_nb[b0 + l];
            T d[ND];
#pragma unroll
            for (int c = 0; c < ND; ++c) d[c] = dinv[ND * m + c];
            T *vb = values + int64_t(ND) * ND * b0 + ND * l;
#pragma unroll
            for (int i = 0; i < ND; ++i)
#pragma unroll
                for (int c = 0; c < ND; ++c) vb[int64_t(i) * ND * deg + c] *= d[c];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_mul_inplace(int64_t n, T *__restrict__ x, const T *__restrict__ d) {
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += int64_t(gridDim.x) * kThreads)
        x[i] *= d[i];
}

template <typename T>
void launch_scale_columns(const fem_handle *h, T *values, const T *dinv, hipStream_t s) {
    const Graph &g = h->g;
    if (g.Nn == 0) return;
    dim3 grid(grid_for(g.Nn, kThreads / 32));
    if (g.nd == 1)
        hipLaunchKernelGGL((k_scale_columns<1, T>), grid, dim3(kThreads), 0, s, g.Nn, g.node_ptr, g.node_nb, values,
                           dinv);
    else
        hipLaunchKernelGGL((k_scale_columns<3, T>), grid, dim3(kThreads), 0, s, g.Nn, g.node_ptr, g.node_nb, values,
                           dinv);
    FEM_HIP(hipGetLastError());
}
template void launch_scale_columns<float>(const fem_handle *, float *, const float *, hipStream_t);
template void launch_scale_columns<double>(const fem_handle *, double *, const double *, hipStream_t);

template <typename T>
void launch_mul_inplace(T *x, const T *d, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL((k_mul_inplace<T>), dim3(grid_for(n, kThreads)), dim3(kThreads), 0, s, n, x, d);
    FEM_HIP(hipGetLastError());
}
template void launch_mul_inplace<float>(float *, const float *, int64_t, hipStream_t);
template void launch_mul_inplace<double>(double *, const double *, int64_t, hipStream_t);

template <typename TI>
void launch_axpy_to_f64(const TI *x, double *y, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL((k_axpy_f64<TI>), dim3(grid_for(n, kThreads)), dim3(kThreads), 0, s, n, x, y);
    FEM_HIP(hipGetLastError());
}
template void launch_axpy_to_f64<float>(const float *, double *, int64_t, hipStream_t);
template void launch_axpy_to_f64<double>(const double *, double *, int64_t, hipStream_t);

void launch_set_dirichlet(const fem_handle *h, double *u, const double *u0, const double *g, double lam,
                          hipStream_t s) {
    if (h->g.N == 0) return;
    hipLaunchKernelGGL(k_set_dirichlet, dim3(grid_for(h->g.N, kThreads)), dim3(kThreads), 0, s, h->g.N, h->m.mask, u,
                       u0, g, lam);
    FEM_HIP(hipGetLastError());
}

void launch_dirichlet_increment(const fem_handle *h, const double *u, const double *u0, const double *g, double lam,
                                double *delta, hipStream_t s) {
    if (h->g.N == 0) return;
    hipLaunchKernelGGL(k_dirichlet_increment, dim3(grid_for(h->g.N, kThreads)), dim3(kThreads), 0, s, h->g.N,
                       h->m.mask, u, u0, g, lam, delta);
    FEM_HIP(hipGetLastError());
}

void launch_neg_sum(const double *a, const double *b, double *out, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_neg_sum, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, s, n, a, b, out);
    FEM_HIP(hipGetLastError());
}

void launch_mask_copy(const fem_handle *h, const double *in, double *out, hipStream_t s) {
    if (h->g.N == 0) return;
    hipLaunchKernelGGL(k_mask_copy, dim3(grid_for(h->g.N, kThreads)), dim3(kThreads), 0, s, h->g.N, h->m.mask, in,
                       out);
    FEM_HIP(hipGetLastError());
}

void launch_sub(const double *a, const double *b, double *out, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_sub, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, s, n, a, b, out);
    FEM_HIP(hipGetLastError());
}

void launch_export(const fem_handle *h, int64_t *row_ptr, int32_t *col_idx, int32_t *slot, int64_t *diag,
                   int32_t *tperm, hipStream_t s) {
    const Graph &g = h->g;
    if (row_ptr) FEM_HIP(hipMemcpyAsync(row_ptr, g.row_ptr, (g.N + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    const int nd = g.nd;
    if ((col_idx || tperm) && g.nnz > 0) {
        dim3 grid(grid_for(g.nnz, kThreads));
        if (nd == 1)
            hipLaunchKernelGGL(k_export_cols<1>, grid, dim3(kThreads), 0, s, g.nnzb, g.node_ptr, g.node_nb, g.blk_row,
                               g.mirror, g.row_ptr, col_idx, tperm);
        else
            hipLaunchKernelGGL(k_export_cols<3>, grid, dim3(kThreads), 0, s, g.nnzb, g.node_ptr, g.node_nb, g.blk_row,
                               g.mirror, g.row_ptr, col_idx, tperm);
    }
    if (slot && g.Ne > 0) {
        int64_t tot = g.Ne * 64 * nd * nd;
        dim3 grid(grid_for(tot, kThreads));
        if (nd == 1)
            hipLaunchKernelGGL(k_export_slots<1>, grid, dim3(kThreads), 0, s, g.Ne, h->m.conn, g.bslot, g.node_ptr,
                               g.row_ptr, slot);
        else
            hipLaunchKernelGGL(k_export_slots<3>, grid, dim3(kThreads), 0, s, g.Ne, h->m.conn, g.bslot, g.node_ptr,
                               g.row_ptr, slot);
    }
    if (diag && g.N > 0) {
        dim3 grid(grid_for(g.N, kThreads));
        if (nd == 1)
            hipLaunchKernelGGL(k_export_diag<1>, grid, dim3(kThreads), 0, s, g.N, g.bdiag, g.node_ptr, g.row_ptr, diag);
        else
            hipLaunchKernelGGL(k_export_diag<3>, grid, dim3(kThreads), 0, s, g.N, g.bdiag, g.node_ptr, g.row_ptr, diag);
    }
    FEM_HIP(hipGetLastError());
}

}  // namespace fem

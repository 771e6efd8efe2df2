// Element-level kernels for HEX8 meshes on gfx950.
//
// Work mapping: one element per group of 8 consecutive lanes, lane a <-> local
// node a (so a 64-wide wavefront holds 8 elements and every cross-lane exchange
// stays inside a wavefront).  At each of the 2x2x2 Gauss points the lanes of an
// element build the isoparametric Jacobian and the displacement gradient by an
// 8-lane butterfly sum (every lane ends with bit-identical values), then each lane
// forms the quantities of its own node.  For the tangent, each lane accumulates the
// 3 x 24 row block of K_e that belongs to its node; the shape-gradient data of the
// other seven nodes come from LDS.
//
// Element outputs go to a per-element scratch area and are summed per node / per
// CSR block by separate gather kernels: every global entry is written exactly once,
// with no atomics on values and a fixed summation order (deterministic).
//
// Paper: element residual R_e and K_e = dr_e/dU_e (Sec. 2.2), constitutive laws
// (Sec. 2.3, Eq. (linear_elasticity), Eq. (neo-hookean)), assembly (Alg. 1).
#include <algorithm>
#include <vector>

#include "internal.h"
#include "lanes.h"

namespace fem {

namespace {

constexpr int kThreads = 256;
constexpr int kElemsPerBlock = kThreads / 8;

__device__ __forceinline__ int ref_sign(int a, int j) {
    // reference coordinates of HEX8 node a: x = (a ^ (a >> 1)) & 1, y = (a >> 1) & 1, z = (a >> 2) & 1
    int bit = (j == 0) ? ((a ^ (a >> 1)) & 1) : (j == 1 ? ((a >> 1) & 1) : ((a >> 2) & 1));
    return bit ? 1 : -1;
}

// Sum over the 8 lanes of an element (DPP butterfly; every lane gets the total).
template <typename T>
__device__ __forceinline__ T sum8(T v) {
    return lane_sum8(v);
}

template <typename T>
__device__ __forceinline__ T det3(const T A[3][3]) {
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

// B = A^{-T} (so that B g = A^{-T} g), given det(A) = d.
template <typename T>
__device__ __forceinline__ void inv_transpose3(const T A[3][3], T d, T B[3][3]) {
    T id = T(1) / d;
    B[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) * id;
    B[1][0] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
    B[2][0] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
    B[0][1] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) * id;
    B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
    B[2][1] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
    B[0][2] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) * id;
    B[1][2] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
    B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
}

__device__ __forceinline__ double modulus(const Material &m, double theta) {
    return m.pmap == FEM_THETA_SIMP ? m.simp_emin + pow(theta, m.simp_p) * (m.simp_e0 - m.simp_emin) : theta;
}

__device__ __forceinline__ double dmodulus(const Material &m, double theta) {
    return m.pmap == FEM_THETA_SIMP ? m.simp_p * pow(theta, m.simp_p - 1.0) * (m.simp_e0 - m.simp_emin) : 1.0;
}

// Per-lane geometry at Gauss point q: physical gradient g of this lane's shape
// function and the Jacobian determinant (identical in all 8 lanes).
template <typename T>
__device__ __forceinline__ T gp_geometry(int a, int q, const T X[3], T g[3]) {
    const T gq = T(0.57735026918962576451);  // 1/sqrt(3)
    T xi[3] = {(q & 1) ? gq : -gq, (q & 2) ? gq : -gq, (q & 4) ? gq : -gq};
    T l[3], s[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        s[j] = T(ref_sign(a, j));
        l[j] = T(0.5) * (T(1) + s[j] * xi[j]);
    }
    T dN[3] = {T(0.5) * s[0] * l[1] * l[2], T(0.5) * s[1] * l[0] * l[2], T(0.5) * s[2] * l[0] * l[1]};
    T J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) J[i][j] = sum8(X[i] * dN[j]);
    T d = det3(J);
    T Bt[3][3];
    inv_transpose3(J, d, Bt);
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = Bt[i][0] * dN[0] + Bt[i][1] * dN[1] + Bt[i][2] * dN[2];
    return d;
}

// Gradient of a nodal field (ND components) at the Gauss point: G[i][J] = sum_a U_a,i g_a,J.
template <int ND, typename T>
__device__ __forceinline__ void field_grad(const T U[ND], const T g[3], T G[3][3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) G[i][j] = (i < ND) ? sum8(U[i] * g[j]) : T(0);
}

// Neo-Hookean kinematic scalars at F = I + G.
template <typename T>
struct NHState {
    T F[3][3], H[3][3];  // H = F^{-T}
    T J, I1, c, alpha, beta, pcoef;
};

template <typename T>
__device__ __forceinline__ bool nh_state(const T G[3][3], T mod, T bulk_ratio, NHState<T> &s) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) s.F[i][j] = G[i][j] + (i == j ? T(1) : T(0));
    s.J = det3(s.F);
    bool ok = s.J > T(0);
    T J = ok ? s.J : T(1);
    inv_transpose3(s.F, J, s.H);
    T I1 = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) I1 += s.F[i][j] * s.F[i][j];
    s.I1 = I1;
    T kappa = bulk_ratio * mod;
    T cr = cbrt(J);
    s.c = mod / (cr * cr);  // G J^{-2/3}
    s.alpha = T(2.0 / 9.0) * s.c * I1 + kappa * (T(2) * J * J - J);
    s.beta = s.c * I1 * T(1.0 / 3.0) - kappa * (J * J - J);
    s.pcoef = kappa * J * (J - T(1)) - s.c * I1 * T(1.0 / 3.0);  // P g = c F g + pcoef H g
    return ok;
}

template <typename T>
__device__ __forceinline__ void matvec3(const T A[3][3], const T x[3], T y[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) y[i] = A[i][0] * x[0] + A[i][1] * x[1] + A[i][2] * x[2];
}

// Perfect J2 plasticity at one Gauss point (Sec. 2.3, plasticity paragraph).  hq holds
// the committed state of the point: total strain then stress, each as (xx, yy, zz, yz,
// xz, xy).  Trial stress from the strain increment sym(G) - eps, deviator s and
// s_vm = sqrt(3/2 s:s); above the yield stress the deviator is scaled back onto the
// surface (radial return).  The consistent tangent of that map, d sigma / d grad u
// (hand-derived; the paper leaves it to automatic differentiation), is
//   A = lw I(x)I + mup (delta_ik delta_jl + delta_il delta_jk) - beta s(x)s
// with kappa = lambda + 2 mu / 3; elastic: mup = mu, beta = 0; plastic:
// mup = mu sigma_y / s_vm, beta = 3 mup / s_vm^2; and lw = kappa - 2 mup / 3.
template <typename T>
struct J2State {
    T sig[6], dev[6];  // returned stress and trial deviator, (xx, yy, zz, yz, xz, xy)
    T lw, mup, beta;
};

template <typename T>
__device__ __forceinline__ void j2_state(const Material &m, T E, const T G[3][3], const double *hq, J2State<T> &s) {
    const T nu = T(m.nu);
    const T lam = E * nu / ((T(1) + nu) * (T(1) - T(2) * nu)), mu = E / (T(2) * (T(1) + nu));
    T de[6] = {G[0][0], G[1][1], G[2][2], T(0.5) * (G[1][2] + G[2][1]), T(0.5) * (G[0][2] + G[2][0]),
               T(0.5) * (G[0][1] + G[1][0])};
#pragma unroll
    for (int c = 0; c < 6; ++c) de[c] -= T(hq[c]);
    const T tr = de[0] + de[1] + de[2];
    T st[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) st[c] = T(hq[6 + c]) + T(2) * mu * de[c] + (c < 3 ? lam * tr : T(0));
    const T p = (st[0] + st[1] + st[2]) * T(1.0 / 3.0);
    T ss = T(0);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        s.dev[c] = st[c] - (c < 3 ? p : T(0));
        ss += (c < 3 ? T(1) : T(2)) * s.dev[c] * s.dev[c];
    }
    const T svm = sqrt(T(1.5) * ss), f = svm - T(m.yield_stress);
    const bool plastic = f > T(0);
    const T kappa = lam + T(2.0 / 3.0) * mu;
    s.mup = plastic ? mu * T(m.yield_stress) / svm : mu;
    s.beta = plastic ? T(3) * s.mup / (svm * svm) : T(0);
    s.lw = kappa - T(2.0 / 3.0) * s.mup;
#pragma unroll
    for (int c = 0; c < 6; ++c) s.sig[c] = plastic ? st[c] - s.dev[c] / svm * f : st[c];
}

// y = S x for a symmetric tensor stored as (xx, yy, zz, yz, xz, xy).
template <typename T>
__device__ __forceinline__ void symvec(const T S[6], const T x[3], T y[3]) {
    y[0] = S[0] * x[0] + S[5] * x[1] + S[4] * x[2];
    y[1] = S[5] * x[0] + S[1] * x[1] + S[3] * x[2];
    y[2] = S[4] * x[0] + S[3] * x[1] + S[2] * x[2];
}

// Flux applied to this lane's shape gradient: out = f(G) g (the integrand of R_e
// at one Gauss point, before the quadrature weight).  Returns false if det F <= 0.
// hq: the Gauss point's committed J2 state (unused by the other laws).
// First Piola flux P(G) as a 3x3 matrix (rows >= ND are zero): the element residual
// of node a is sum_q detJ P g_a.
template <int MODEL, typename T>
__device__ __forceinline__ bool flux_mat(const Material &m, T mod, const T G[3][3], T P[3][3], const double *hq) {
    if constexpr (MODEL == FEM_POISSON) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) P[i][j] = (i == 0) ? mod * G[0][j] : T(0);
        return true;
    } else if constexpr (MODEL == FEM_LINEAR_ELASTIC) {
        T nu = T(m.nu);
        T lam = mod * nu / ((T(1) + nu) * (T(1) - T(2) * nu)), mu = mod / (T(2) * (T(1) + nu));
        T tr = G[0][0] + G[1][1] + G[2][2];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) P[i][j] = mu * (G[i][j] + G[j][i]) + (i == j ? lam * tr : T(0));
        return true;
    } else {
        static_assert(MODEL == FEM_NEO_HOOKEAN, "the J2 law uses j2_flux_dot");
        NHState<T> s;
        bool ok = nh_state(G, mod, T(m.bulk_ratio), s);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) P[i][j] = s.c * s.F[i][j] + s.pcoef * s.H[i][j];
        return ok;
    }
}

// Directional derivative of the flux, dP = A(G) : dG, as a 3x3 matrix.
template <int MODEL, typename T>
__device__ __forceinline__ bool dflux_mat(const Material &m, T mod, const T G[3][3], const T dG[3][3], T dP[3][3],
                                          const double *hq) {
    if constexpr (MODEL == FEM_POISSON || MODEL == FEM_LINEAR_ELASTIC) {
        return flux_mat<MODEL, T>(m, mod, dG, dP, hq);  // linear laws
    } else {
        static_assert(MODEL == FEM_NEO_HOOKEAN, "the J2 law uses j2_dflux_dot");
        NHState<T> s;
        bool ok = nh_state(G, mod, T(m.bulk_ratio), s);
        T HdF = T(0), FdF = T(0);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                HdF += s.H[i][j] * dG[i][j];
                FdF += s.F[i][j] * dG[i][j];
            }
        // dF^T H, then H (dF^T H)
        T DH[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) DH[k][j] = dG[0][k] * s.H[0][j] + dG[1][k] * s.H[1][j] + dG[2][k] * s.H[2][j];
        T c23 = T(2.0 / 3.0) * s.c;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const T HDH = s.H[i][0] * DH[0][j] + s.H[i][1] * DH[1][j] + s.H[i][2] * DH[2][j];
                dP[i][j] = s.c * dG[i][j] - c23 * (s.F[i][j] * HdF + s.H[i][j] * FdF) + s.alpha * s.H[i][j] * HdF +
                           s.beta * HDH;
            }
        return ok;
    }
}

// J2 flux and its derivative applied to this lane's gradient g (the per-lane form used
// by the J2 vector kernel): out = sigma g, and out = (A : dG) g.
template <typename T>
__device__ __forceinline__ void j2_flux_dot(const Material &m, T mod, const T G[3][3], const T g[3], T out[3],
                                            const double *hq) {
    J2State<T> s;
    j2_state(m, mod, G, hq, s);
    symvec(s.sig, g, out);
}

template <typename T>
__device__ __forceinline__ void j2_dflux_dot(const Material &m, T mod, const T G[3][3], const T dG[3][3],
                                             const T g[3], T out[3], const double *hq) {
    J2State<T> s;
    j2_state(m, mod, G, hq, s);
    const T tr = dG[0][0] + dG[1][1] + dG[2][2];
    const T sd = s.dev[0] * dG[0][0] + s.dev[1] * dG[1][1] + s.dev[2] * dG[2][2] + s.dev[3] * (dG[1][2] + dG[2][1]) +
                 s.dev[4] * (dG[0][2] + dG[2][0]) + s.dev[5] * (dG[0][1] + dG[1][0]);
    T sg[3];
    symvec(s.dev, g, sg);
#pragma unroll
    for (int i = 0; i < 3; ++i)
        out[i] = s.lw * tr * g[i] +
                 s.mup * ((dG[i][0] + dG[0][i]) * g[0] + (dG[i][1] + dG[1][i]) * g[1] + (dG[i][2] + dG[2][i]) * g[2]) -
                 s.beta * sd * sg[i];
}

// Reference gradients dN_b(xi_q) of the 8 shape functions at Gauss point q.
template <typename T>
__device__ __forceinline__ void ref_grad(int b, int q, T dN[3]) {
    const T gq = T(0.57735026918962576451);  // 1/sqrt(3)
    T l[3], sg[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const T xi = ((q >> j) & 1) ? gq : -gq;
        sg[j] = T(ref_sign(b, j));
        l[j] = T(0.5) * (T(1) + sg[j] * xi);
    }
    dN[0] = T(0.5) * sg[0] * l[1] * l[2];
    dN[1] = T(0.5) * sg[1] * l[0] * l[2];
    dN[2] = T(0.5) * sg[2] * l[0] * l[1];
}

struct ElemIds {
    int64_t e;
    int a, el;
    bool valid;
};

__device__ __forceinline__ ElemIds elem_ids(int64_t Ne) {
    ElemIds id;
    id.a = threadIdx.x & 7;
    id.el = threadIdx.x >> 3;
    int64_t e = int64_t(blockIdx.x) * kElemsPerBlock + id.el;
    id.valid = e < Ne;
    id.e = id.valid ? e : Ne - 1;  // idle groups recompute the last element and store nothing
    return id;
}

// Loads this lane's node.  Coordinates (and, with rel_u, the field) are taken
// relative to local node 0 of the element, in FP64 before rounding to T: the
// gradients are unchanged (the shape-function gradients sum to zero) but the
// differences of nearby absolute values no longer cancel in T arithmetic.
template <int ND, typename T>
__device__ __forceinline__ void load_node(const double *coords, const int32_t *conn, const double *u,
                                          const uint8_t *mask, const ElemIds &id, T X[3], T U[ND], bool rel_u) {
    const int64_t n = conn[id.e * 8 + id.a];
    const int64_t n0 = conn[id.e * 8];
#pragma unroll
    for (int i = 0; i < 3; ++i) X[i] = T(coords[3 * n + i] - coords[3 * n0 + i]);
#pragma unroll
    for (int i = 0; i < ND; ++i) {
        const int64_t d = ND * n + i, d0 = ND * n0 + i;
        const double ua = (u == nullptr || (mask && mask[d])) ? 0.0 : u[d];
        const double u0 = (!rel_u || u == nullptr || (mask && mask[d0])) ? 0.0 : u[d0];
        U[i] = T(ua - u0);
    }
}

// ------------------------------------------------------------------ residual-type kernels
enum { VEC_RESIDUAL = 0, VEC_JVP = 1, VEC_VJP = 2, VEC_LIFT = 3, VEC_MASS = 4 };

// (slot s = kpos[e*8 + a]: node-major incidence order, so each node's terms are contiguous)
// VEC_RESIDUAL: scratch[s][i] = sum_q detJ f(grad u) g_a            (modulus m(theta_e))
// VEC_JVP:      scratch[s][i] = sum_q detJ (A(grad u) : grad v) g_a  (v with Dirichlet dofs zeroed)
// VEC_VJP:      g[e] = -m'(theta_e) sum_{a,i free} lam_a,i sum_q detJ f_unit(grad u) g_a
// VEC_LIFT:     as VEC_JVP but with v used on every dof (v is nonzero on Dirichlet dofs only)
//
// Two phases, 8 lanes per element.  Lane q evaluates Gauss point q: the Jacobian J_q
// from the element's node coordinates, the field gradients G = G_ref J_q^{-1}, the
// flux P (or its derivative) and M_q = detJ_q P J_q^{-T}, which it leaves in LDS.
// Lane a then sums its node's terms, sum_q M_q dN_a(xi_q) (= sum_q detJ P g_a).  The
// per-point work (Jacobian inverse, constitutive update) is done once per point
// instead of once per lane.
template <int MODEL, int ND, int MODE>
__global__ __launch_bounds__(kThreads) void k_element_vec(int64_t Ne, const double *__restrict__ coords,
                                                          const int32_t *__restrict__ conn,
                                                          const int32_t *__restrict__ kpos,
                                                          const uint8_t *__restrict__ mask, Material mat,
                                                          const double *__restrict__ theta,
                                                          const double *__restrict__ u,
                                                          const double *__restrict__ v,
                                                          const double *__restrict__ hist, double *__restrict__ out,
                                                          int *status) {
    constexpr bool kDir = MODE == VEC_JVP || MODE == VEC_LIFT;
    if constexpr (MODEL == FEM_J2_PLASTIC) {
        // J2 keeps the per-lane form (every lane walks the 8 points for its own node): the
        // loading-unloading path near the limit load has a nearly singular tangent, and
        // its Newton iterations were measured to converge with this form's rounding.
        ElemIds id = elem_ids(Ne);
        double X[3], U[ND], W[ND];
        load_node<ND, double>(coords, conn, u, nullptr, id, X, U, true);
        if (MODE != VEC_RESIDUAL)
            load_node<ND, double>(coords, conn, v, MODE == VEC_LIFT ? nullptr : mask, id, X, W, MODE != VEC_VJP);
        double th = theta[id.e];
        double mod = (MODE == VEC_VJP) ? 1.0 : modulus(mat, th);
        double acc[3] = {0, 0, 0};
        bool mesh_ok = true;
#pragma unroll 1
        for (int q = 0; q < 8; ++q) {
            double g[3];
            double dJ = gp_geometry(id.a, q, X, g);
            mesh_ok &= dJ > 0.0;
            double G[3][3], o[3];
            field_grad<ND>(U, g, G);
            const double *hq = hist + (id.e * 8 + q) * 12;
            if (kDir) {
                double dG[3][3];
                field_grad<ND>(W, g, dG);
                j2_dflux_dot<double>(mat, mod, G, dG, g, o, hq);
            } else {
                j2_flux_dot<double>(mat, mod, G, g, o, hq);
            }
#pragma unroll
            for (int i = 0; i < ND; ++i) acc[i] += dJ * o[i];
        }
        if (id.valid && id.a == 0 && !mesh_ok) atomicOr(status, ST_MESH);
        if (MODE == VEC_VJP) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < ND; ++i) s += W[i] * acc[i];
            s = sum8(s);
            if (id.valid && id.a == 0) out[id.e] = -dmodulus(mat, th) * s;
        } else if (id.valid) {
#pragma unroll
            for (int i = 0; i < ND; ++i) out[int64_t(kpos[id.e * 8 + id.a]) * ND + i] = acc[i];
        }
    } else {
    constexpr int NF = 3 + ND + (MODE == VEC_RESIDUAL ? 0 : ND);  // node values staged per lane
    __shared__ double nodes[kElemsPerBlock][8][NF];
    __shared__ double Ms[kElemsPerBlock][8][9];
    ElemIds id = elem_ids(Ne);
    double X[3], U[ND], W[ND];
    load_node<ND, double>(coords, conn, u, nullptr, id, X, U, true);
    if (MODE != VEC_RESIDUAL)
        load_node<ND, double>(coords, conn, v, MODE == VEC_LIFT ? nullptr : mask, id, X, W, MODE != VEC_VJP);
    double *mine = nodes[id.el][id.a];
#pragma unroll
    for (int i = 0; i < 3; ++i) mine[i] = X[i];
#pragma unroll
    for (int i = 0; i < ND; ++i) mine[3 + i] = U[i];
    if constexpr (MODE != VEC_RESIDUAL)
#pragma unroll
        for (int i = 0; i < ND; ++i) mine[3 + ND + i] = W[i];
    const double th = theta[id.e];
    const double mod = (MODE == VEC_VJP) ? 1.0 : modulus(mat, th);
    __syncthreads();
    // phase 1: this lane's Gauss point q = a
    bool mesh_ok, mat_ok;
    {
        const int q = id.a;
        double J[3][3] = {}, Gr[3][3] = {}, Wr[3][3] = {};  // Jacobian, reference gradients of u and v
#pragma unroll 2
        for (int b = 0; b < 8; ++b) {
            double dN[3];
            ref_grad<double>(b, q, dN);
            const double *nb = nodes[id.el][b];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    J[i][j] = fma(nb[i], dN[j], J[i][j]);
                    if (i < ND) Gr[i][j] = fma(nb[3 + i], dN[j], Gr[i][j]);
                    if (kDir && i < ND) Wr[i][j] = fma(nb[3 + ND + i], dN[j], Wr[i][j]);
                }
        }
        const double d = det3(J);
        mesh_ok = d > 0.0;
        double Bt[3][3];  // J^{-T}: g_b = Bt dN_b
        inv_transpose3(J, d, Bt);
        double G[3][3], dG[3][3], P[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                G[i][j] = Gr[i][0] * Bt[j][0] + Gr[i][1] * Bt[j][1] + Gr[i][2] * Bt[j][2];
                dG[i][j] = Wr[i][0] * Bt[j][0] + Wr[i][1] * Bt[j][1] + Wr[i][2] * Bt[j][2];
            }
        if constexpr (kDir) mat_ok = dflux_mat<MODEL, double>(mat, mod, G, dG, P, nullptr);
        else mat_ok = flux_mat<MODEL, double>(mat, mod, G, P, nullptr);
        double *mq = Ms[id.el][q];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) mq[i * 3 + k] = d * (P[i][0] * Bt[0][k] + P[i][1] * Bt[1][k] + P[i][2] * Bt[2][k]);
    }
    __syncthreads();
    // phase 2: this lane's node a
    double acc[ND];
#pragma unroll
    for (int i = 0; i < ND; ++i) acc[i] = 0.0;
#pragma unroll 2
    for (int q = 0; q < 8; ++q) {
        double dN[3];
        ref_grad<double>(id.a, q, dN);
        const double *mq = Ms[id.el][q];
#pragma unroll
        for (int i = 0; i < ND; ++i) acc[i] += mq[i * 3] * dN[0] + mq[i * 3 + 1] * dN[1] + mq[i * 3 + 2] * dN[2];
    }
    if (id.valid && (!mesh_ok || !mat_ok))
        atomicOr(status, (!mesh_ok ? ST_MESH : 0) | (!mat_ok ? ST_INVERTED : 0));
    if (MODE == VEC_VJP) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < ND; ++i) s += W[i] * acc[i];
        s = sum8(s);
        if (id.valid && id.a == 0) out[id.e] = -dmodulus(mat, th) * s;
    } else if (id.valid) {
#pragma unroll
        for (int i = 0; i < ND; ++i) out[int64_t(kpos[id.e * 8 + id.a]) * ND + i] = acc[i];
    }
    }
}

// Consistent mass product: scratch[s][i] = sum_q detJ N_a(xi_q) sum_b N_b(xi_q) x_b,i
// (the load of a nodal field x interpolated with the shape functions; Sec. 2.1,
// the body-force term of Eq. (weak)).
template <int ND>
__global__ __launch_bounds__(kThreads) void k_element_mass(int64_t Ne, const double *__restrict__ coords,
                                                           const int32_t *__restrict__ conn,
                                                           const int32_t *__restrict__ kpos,
                                                           const double *__restrict__ x, double *__restrict__ out,
                                                           int *status) {
    ElemIds id = elem_ids(Ne);
    double X[3], Xv[ND];
    load_node<ND, double>(coords, conn, x, nullptr, id, X, Xv, false);
    const double gq = 0.57735026918962576451;
    double acc[ND];
#pragma unroll
    for (int i = 0; i < ND; ++i) acc[i] = 0.0;
    bool mesh_ok = true;
#pragma unroll 1
    for (int q = 0; q < 8; ++q) {
        double g[3];
        const double dJ = gp_geometry(id.a, q, X, g);
        mesh_ok &= dJ > 0.0;
        double Na = 1.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double xi = (q >> j) & 1 ? gq : -gq;
            Na *= 0.5 * (1.0 + double(ref_sign(id.a, j)) * xi);
        }
#pragma unroll
        for (int i = 0; i < ND; ++i) acc[i] += dJ * Na * sum8(Na * Xv[i]);
    }
    if (id.valid && id.a == 0 && !mesh_ok) atomicOr(status, ST_MESH);
    if (id.valid)
#pragma unroll
        for (int i = 0; i < ND; ++i) out[int64_t(kpos[id.e * 8 + id.a]) * ND + i] = acc[i];
}

// J2 history commit after a converged load step: lane a updates Gauss point a of its
// element, eps <- sym(grad u) and sigma <- the returned stress of j2_state.  Each
// point reads and then writes only its own record, so the update is in place.
__global__ __launch_bounds__(kThreads) void k_j2_commit(int64_t Ne, const double *__restrict__ coords,
                                                       const int32_t *__restrict__ conn, Material mat,
                                                       const double *__restrict__ theta,
                                                       const double *__restrict__ u, double *__restrict__ hist) {
    ElemIds id = elem_ids(Ne);
    double X[3], U[3];
    load_node<3, double>(coords, conn, u, nullptr, id, X, U, true);
    double Gm[3][3] = {};
#pragma unroll 1
    for (int q = 0; q < 8; ++q) {
        double g[3], G[3][3];
        gp_geometry(id.a, q, X, g);
        field_grad<3>(U, g, G);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Gm[i][j] = (q == id.a) ? G[i][j] : Gm[i][j];
    }
    if (!id.valid) return;
    double *hq = hist + (id.e * 8 + id.a) * 12;
    J2State<double> st;
    j2_state(mat, modulus(mat, theta[id.e]), Gm, hq, st);
    const double eps[6] = {Gm[0][0], Gm[1][1], Gm[2][2], 0.5 * (Gm[1][2] + Gm[2][1]), 0.5 * (Gm[0][2] + Gm[2][0]),
                           0.5 * (Gm[0][1] + Gm[1][0])};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        hq[c] = eps[c];
        hq[6 + c] = st.sig[c];
    }
}

// Per-block partial sums of sum_q detJ sigma_q (6 components) and sum_q detJ over the
// committed J2 history: lane a takes Gauss point a; partials[block * 7 + c].
__global__ __launch_bounds__(kThreads) void k_j2_average(int64_t Ne, const double *__restrict__ coords,
                                                        const int32_t *__restrict__ conn,
                                                        const double *__restrict__ hist, double *partials) {
    __shared__ double red[kThreads / 64][7];
    ElemIds id = elem_ids(Ne);
    double X[3], U[1];
    load_node<1, double>(coords, conn, nullptr, nullptr, id, X, U, false);
    double w = 0.0;
#pragma unroll 1
    for (int q = 0; q < 8; ++q) {
        double g[3];
        const double dJ = gp_geometry(id.a, q, X, g);
        w = (q == id.a) ? dJ : w;
    }
    if (!id.valid) w = 0.0;
    const double *hs = hist + (id.e * 8 + id.a) * 12 + 6;
    double v[7];
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = w * hs[c];
    v[6] = w;
#pragma unroll
    for (int c = 0; c < 7; ++c) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[c] += __shfl_xor(v[c], o, 64);
    }
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int c = 0; c < 7; ++c) red[threadIdx.x >> 6][c] = v[c];
    __syncthreads();
    if (threadIdx.x < 7) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < kThreads / 64; ++k) t += red[k][threadIdx.x];
        partials[int64_t(blockIdx.x) * 7 + threadIdx.x] = t;
    }
}

// Sum element contributions per dof.
// VEC_RESIDUAL: out[d] = sum - lf * F[d], 0 on Dirichlet dofs.
// VEC_JVP:      out[d] = sum, v[d] on Dirichlet dofs.
// VEC_LIFT:     out[d] = sum, 0 on Dirichlet dofs.
template <int ND, int MODE>
__global__ __launch_bounds__(256) void k_gather_vec(int64_t N, const int64_t *__restrict__ ne_ptr,
                                                    const double *__restrict__ scratch,
                                                    const uint8_t *__restrict__ mask, const double *__restrict__ F,
                                                    double lf, const double *__restrict__ v,
                                                    double *__restrict__ out, int *status) {
    int64_t d = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (d >= N) return;
    int64_t n = d / ND;
    int i = int(d - n * ND);
    double s = 0.0;
    for (int64_t k = ne_ptr[n]; k < ne_ptr[n + 1]; ++k) s += scratch[k * ND + i];  // node n's contiguous slots
    double r;
    if (mask && mask[d]) {
        r = (MODE == VEC_JVP) ? v[d] : 0.0;
    } else {
        r = (MODE == VEC_RESIDUAL) ? s - lf * F[d] : s;
    }
    if (!isfinite(r)) atomicOr(status, ST_NAN);
    out[d] = r;
}

// ------------------------------------------------------------------ tangent kernel
// Lane a accumulates the row block K_e[(a,i), (b,k)] for all b, i, k and writes it to
// scratch[((kpos[e*8 + a])*8 + b)*ND*ND + i*ND + k]: the row blocks feeding node
// conn[e][a] are contiguous, so the gather reads each node's 8 row blocks as one run.
template <int MODEL, int ND, typename T>
__global__ __launch_bounds__(kThreads, sizeof(T) == 4 ? 3 : 2) void k_element_tangent(int64_t Ne, const double *__restrict__ coords,
                                                              const int32_t *__restrict__ conn,
                                                              const int32_t *__restrict__ kpos, Material mat,
                                                              const double *__restrict__ theta,
                                                              const double *__restrict__ u,
                                                              const double *__restrict__ hist, T *__restrict__ ke,
                                                              int *status) {
    // per-node data shared through LDS: g (all laws), F g and F^{-T} g (neo-Hookean),
    // s g with the trial deviator s (J2)
    constexpr int NV = (MODEL == FEM_NEO_HOOKEAN) ? 9 : (MODEL == FEM_J2_PLASTIC ? 6 : 3);
    constexpr int ES = 8 * NV + 1;  // padded element stride (bank spread)
    constexpr bool kNonlinear = MODEL == FEM_NEO_HOOKEAN || MODEL == FEM_J2_PLASTIC;
    __shared__ T lds[kElemsPerBlock * ES];
    ElemIds id = elem_ids(Ne);
    T X[3], U[ND];
    load_node<ND, T>(coords, conn, kNonlinear ? u : nullptr, nullptr, id, X, U, true);
    T mod = T(modulus(mat, theta[id.e]));
    T K[8][ND][ND];
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
        for (int i = 0; i < ND; ++i)
#pragma unroll
            for (int k = 0; k < ND; ++k) K[b][i][k] = T(0);
    bool mesh_ok = true, mat_ok = true;
    T *my = lds + id.el * ES + id.a * NV;
    const T *el = lds + id.el * ES;
#pragma unroll 1
    for (int q = 0; q < 8; ++q) {
        T g[3];
        T dJ = gp_geometry(id.a, q, X, g);
        mesh_ok &= dJ > T(0);
        if constexpr (MODEL == FEM_NEO_HOOKEAN) {
            T G[3][3];
            field_grad<ND>(U, g, G);
            NHState<T> s;
            mat_ok &= nh_state(G, mod, T(mat.bulk_ratio), s);
            T f[3], h[3];
            matvec3(s.F, g, f);
            matvec3(s.H, g, h);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                my[i] = g[i];
                my[3 + i] = f[i];
                my[6 + i] = h[i];
            }
            __syncthreads();
            T cw = dJ * s.c, c23 = T(2.0 / 3.0) * cw, aw = dJ * s.alpha, bw = dJ * s.beta;
            // block (a, b): aw h_i hb_k + bw hb_i h_k - c23 (f_i hb_k + h_i fb_k) + delta_ik cw g.gb,
            // grouped by the factors of this node so each entry takes three FMAs
            T P[3], Q[3], R[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                P[i] = aw * h[i] - c23 * f[i];
                Q[i] = bw * h[i];
                R[i] = -c23 * h[i];
            }
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const T *o = el + b * NV;
                T gb[3] = {o[0], o[1], o[2]}, fb[3] = {o[3], o[4], o[5]}, hb[3] = {o[6], o[7], o[8]};
                T sdot = cw * (g[0] * gb[0] + g[1] * gb[1] + g[2] * gb[2]);
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        T v = fma(P[i], hb[k], K[b][i][k]);
                        v = fma(hb[i], Q[k], v);
                        v = fma(R[i], fb[k], v);
                        if (i == k) v += sdot;
                        K[b][i][k] = v;
                    }
            }
            __syncthreads();
        } else if constexpr (MODEL == FEM_J2_PLASTIC) {
            T G[3][3];
            field_grad<ND>(U, g, G);
            J2State<T> s;
            j2_state(mat, mod, G, hist + (id.e * 8 + q) * 12, s);
            T sg[3];
            symvec(s.dev, g, sg);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                my[i] = g[i];
                my[3 + i] = sg[i];
            }
            __syncthreads();
            T lw = dJ * s.lw, mw = dJ * s.mup, bw = dJ * s.beta;
            // block (a, b): lw g_i gb_k + mw g_k gb_i - bw sg_i sb_k + delta_ik mw g.gb, three FMAs
            // per entry with this node's factors taken first
            T P[3], Q[3], R[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                P[i] = lw * g[i];
                Q[i] = mw * g[i];
                R[i] = -bw * sg[i];
            }
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const T *o = el + b * NV;
                T gb[3] = {o[0], o[1], o[2]}, sb[3] = {o[3], o[4], o[5]};
                T sdot = mw * (g[0] * gb[0] + g[1] * gb[1] + g[2] * gb[2]);
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        T v = fma(P[i], gb[k], K[b][i][k]);
                        v = fma(gb[i], Q[k], v);
                        v = fma(R[i], sb[k], v);
                        if (i == k) v += sdot;
                        K[b][i][k] = v;
                    }
            }
            __syncthreads();
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) my[i] = g[i];
            __syncthreads();
            if constexpr (MODEL == FEM_LINEAR_ELASTIC) {
                T nu = T(mat.nu);
                T lw = dJ * mod * nu / ((T(1) + nu) * (T(1) - T(2) * nu)), mw = dJ * mod / (T(2) * (T(1) + nu));
                T P[3], Q[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    P[i] = lw * g[i];
                    Q[i] = mw * g[i];
                }
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const T *o = el + b * NV;
                    T gb[3] = {o[0], o[1], o[2]};
                    T sdot = mw * (g[0] * gb[0] + g[1] * gb[1] + g[2] * gb[2]);
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            // lw g_i gb_k + mw g_k gb_i + delta_ik mw g.gb
                            T v = fma(P[i], gb[k], K[b][i][k]);
                            v = fma(gb[i], Q[k], v);
                            if (i == k) v += sdot;
                            K[b][i][k] = v;
                        }
                }
            } else {
                T w = dJ * mod;
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const T *o = el + b * NV;
                    K[b][0][0] += w * (g[0] * o[0] + g[1] * o[1] + g[2] * o[2]);
                }
            }
            __syncthreads();
        }
    }
    if (id.valid && id.a == 0 && (!mesh_ok || !mat_ok))
        atomicOr(status, (!mesh_ok ? ST_MESH : 0) | (!mat_ok ? ST_INVERTED : 0));
    if (id.valid) {
        T *dst = ke + int64_t(kpos[id.e * 8 + id.a]) * 8 * ND * ND;
#pragma unroll
        for (int b = 0; b < 8; ++b)
#pragma unroll
            for (int i = 0; i < ND; ++i)
#pragma unroll
                for (int k = 0; k < ND; ++k) dst[(b * ND + i) * ND + k] = K[b][i][k];
    }
}

// Tangent values from element blocks: thread (block kb, row component i) sums the
// contributing element blocks of node-graph block kb = (n, j-th neighbour m) in
// element order, applies the symmetric Dirichlet elimination and writes row i of
// the block once:
//   LAYOUT_CSR: values[row_ptr[ND*n+i] + ND*j + k], k < ND;
//   LAYOUT_SYM: only blocks with m >= n, block-major at values[ND*ND*(up_base[n] +
//               kb - bdiag[n]) + ND*i + k] (the lower blocks are their transposes).
template <int ND, int LAYOUT, typename T>
__global__ __launch_bounds__(256) void k_gather_values(int64_t nnzb, const int64_t *__restrict__ node_ptr,
                                                       const int32_t *__restrict__ node_nb,
                                                       const int32_t *__restrict__ blk_row,
                                                       const int64_t *__restrict__ blk_ptr,
                                                       const int32_t *__restrict__ blk_src,
                                                       const int64_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ bdiag,
                                                       const int64_t *__restrict__ up_base,
                                                       const uint8_t *__restrict__ mask, const T *__restrict__ ke,
                                                       T *__restrict__ values, int *status) {
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nnzb * ND) return;
    int64_t kb = t / ND;
    int i = int(t - kb * ND);
    int64_t n = blk_row[kb];
    int64_t m = node_nb[kb];
    if (LAYOUT == LAYOUT_SYM && m < n) return;
    T acc[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) acc[k] = T(0);
    for (int64_t s = blk_ptr[kb]; s < blk_ptr[kb + 1]; ++s) {
        const T *src = ke + int64_t(blk_src[s]) * ND * ND + i * ND;
#pragma unroll
        for (int k = 0; k < ND; ++k) acc[k] += src[k];
    }
    int64_t row = ND * n + i;
    bool bad = false;
    T *dst = (LAYOUT == LAYOUT_SYM) ? values + ND * ND * (up_base[n] + kb - bdiag[n]) + ND * i
                                    : values + row_ptr[row] + ND * (kb - node_ptr[n]);
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        int64_t col = ND * m + k;
        T v = acc[k];
        if (mask && (mask[row] || mask[col])) v = (row == col) ? T(1) : T(0);
        bad |= !isfinite(v);
        dst[k] = v;
    }
    if (bad) atomicOr(status, ST_NAN);
}

// Inverse of an ND x ND block (FP64 cofactors), written row-major to out; false when
// the block is singular or not finite.
template <int ND, typename T>
__device__ __forceinline__ bool invert_block(const double B[ND][ND], T *out) {
    if constexpr (ND == 1) {
        out[0] = T(1.0 / B[0][0]);
        return B[0][0] != 0.0 && isfinite(B[0][0]);
    } else {
        const double d = det3(B);
        double C[3][3];
        inv_transpose3(B, d, C);  // C = B^{-T}
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) out[i * 3 + c] = T(C[c][i]);
        return d != 0.0 && isfinite(d);
    }
}

// Block-Jacobi inverses read from assembled values (used when the node-centric gather
// does not apply): one thread per node.
template <int ND, int LAYOUT, typename T>
__global__ __launch_bounds__(256) void k_extract_binv(int64_t Nn, const int64_t *__restrict__ node_ptr,
                                                      const int32_t *__restrict__ bdiag,
                                                      const int64_t *__restrict__ row_ptr,
                                                      const int64_t *__restrict__ up_base,
                                                      const T *__restrict__ values, T *__restrict__ binv,
                                                      int *status) {
    const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (n >= Nn) return;
    double B[ND][ND];
#pragma unroll
    for (int i = 0; i < ND; ++i)
#pragma unroll
        for (int c = 0; c < ND; ++c)
            B[i][c] = (LAYOUT == LAYOUT_SYM)
                          ? double(values[int64_t(ND) * ND * up_base[n] + i * ND + c])
                          : double(values[row_ptr[ND * n + i] + ND * (bdiag[n] - node_ptr[n]) + c]);
    if (!invert_block<ND>(B, binv + int64_t(ND) * ND * n)) atomicOr(status, ST_NAN);
}

// Node-centric gather (one wavefront per node, for node degrees up to
// kGatherMaxDeg): the node's element row blocks are one contiguous run of slots
// ne_ptr[n] .. ne_ptr[n+1]-1 (element ascending); each slot's 8 column blocks are
// added into an LDS image of the node's rows at the positions tgt gives, one slot at
// a time (so every entry sums its contributions in element order, and no two lanes
// touch the same entry in a step).  The rows are then written once, coalesced, with
// the symmetric Dirichlet elimination applied, and the Jacobi inverse diagonal of the
// node is taken from the same image.
constexpr int kGatherMaxDeg = 32;
constexpr int kGatherSlots = 8;  // slots preloaded per pass

// Hand-off of LDS data between lanes of one wavefront: a wavefront's LDS operations are
// performed in program order, so a lane reads what other lanes of its wavefront wrote
// before this point; the fence (wavefront scope) and the wave barrier keep the compiler
// from moving LDS accesses across it.  Neither emits an instruction.
__device__ __forceinline__ void wave_lds_handoff() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int ND, int LAYOUT, typename T>
__global__ __launch_bounds__(256) void k_gather_node(int64_t Nn, const int64_t *__restrict__ node_ptr,
                                                     const uint8_t *__restrict__ nb_bits,
                                                     const int64_t *__restrict__ ne_ptr,
                                                     const uint8_t *__restrict__ tgt,
                                                     const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ bdiag,
                                                     const int64_t *__restrict__ up_base,
                                                     const uint8_t *__restrict__ mask, const T *__restrict__ ke,
                                                     T *__restrict__ values, T *__restrict__ dinv, int bj,
                                                     int *status) {
    constexpr int BS = ND * ND;
    constexpr int W = 64;
    constexpr int PER = (8 * BS + W - 1) / W;  // values of one slot per lane
    __shared__ T img[256 / W][kGatherMaxDeg * BS];
    __shared__ uint8_t nbm[256 / W][kGatherMaxDeg];  // Dirichlet bits of each neighbour's dofs
    // wavefront index made explicitly uniform, so node and slot indices live in scalar
    // registers and their loads go through the scalar cache
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / W), lane = threadIdx.x % W;
    T *a = img[wave];
    // Each wavefront walks nodes with a grid stride (a few resident blocks per CU;
    // one short-lived workgroup per node would be bound by the dispatch rate).  The
    // loop trip count is uniform per wavefront and the kernel has no block barriers.
    for (int64_t n = int64_t(blockIdx.x) * (256 / W) + wave; n < Nn; n += int64_t(gridDim.x) * (256 / W)) {
        const int64_t nb0 = node_ptr[n];
        const int deg = int(node_ptr[n + 1] - nb0);
        // Dirichlet bits of the node's own dofs and of its neighbours', fetched up front so
        // their latency overlaps the value loads
        int rowbits = 0;
        if (mask)
#pragma unroll
            for (int c = 0; c < ND; ++c) rowbits |= int(mask[ND * n + c] != 0) << c;
        if (lane < deg) nbm[wave][lane] = nb_bits[nb0 + lane];
        for (int l = lane; l < deg * BS; l += W) a[l] = T(0);
        wave_lds_handoff();  // the zeroed image and the neighbour bits, to every lane
        const int64_t k1 = ne_ptr[n + 1];
        for (int64_t k0 = ne_ptr[n]; k0 < k1; k0 += kGatherSlots) {
            T val[kGatherSlots][PER];
            int pos[kGatherSlots][PER];
#pragma unroll
            for (int kk = 0; kk < kGatherSlots; ++kk) {
                // the slot index is uniform across the wavefront, so its 8 targets come in
                // one scalar load; the value loads are unconditional (clamped indices) so
                // no load sits behind a branch that would wait for everything in flight
                const bool slot_ok = k0 + kk < k1;
                const int64_t k = slot_ok ? k0 + kk : k0;
                const uint64_t tw = *reinterpret_cast<const uint64_t *>(tgt + k * 8);
#pragma unroll
                for (int t = 0; t < PER; ++t) {
                    const int l = lane + W * t;
                    const bool ok = slot_ok && l < 8 * BS;
                    const int lc = l < 8 * BS ? l : 0;
                    const int b = lc / BS;
                    val[kk][t] = ke[(k * 8) * BS + lc];
                    const int j = int((tw >> (8 * b)) & 0xff);
                    pos[kk][t] = ok ? j * BS + (lc - b * BS) : -1;
                }
            }
            // slot by slot: within a slot no two lanes touch one entry; a later slot's
            // read-modify-write of an entry follows the earlier slot's
#pragma unroll
            for (int kk = 0; kk < kGatherSlots; ++kk) {
#pragma unroll
                for (int t = 0; t < PER; ++t)
                    if (pos[kk][t] >= 0) a[pos[kk][t]] += val[kk][t];
                wave_lds_handoff();
            }
        }
        // rows of the node, CSR (or upper blocks only), with the Dirichlet elimination
        const int jd = int(bdiag[n] - nb0);
        wave_lds_handoff();
        bool bad = false;
#pragma unroll
        for (int i = 0; i < ND; ++i) {
            const int64_t rbase = (LAYOUT == LAYOUT_SYM) ? 0 : row_ptr[ND * n + i];
            const bool rm = (rowbits >> i) & 1;
            for (int r = lane; r < ND * deg; r += W) {
                const int j = r / ND, c = r - j * ND;
                T v = a[j * BS + i * ND + c];
                if (rm || ((nbm[wave][j] >> c) & 1)) v = (j == jd && c == i) ? T(1) : T(0);
                bad |= !isfinite(v);
                if (LAYOUT == LAYOUT_SYM) {
                    if (j >= jd) values[int64_t(BS) * (up_base[n] + j - jd) + i * ND + c] = v;
                } else {
                    values[rbase + r] = v;
                }
            }
        }
        if (dinv && !bj && lane < ND) {
            T v = ((rowbits >> lane) & 1) ? T(1) : a[jd * BS + lane * ND + lane];
            bad |= !(v != T(0)) || !isfinite(v);
            dinv[ND * n + lane] = T(1) / v;
        }
        if (dinv && bj && lane == 0) {
            double B[ND][ND];
#pragma unroll
            for (int i = 0; i < ND; ++i)
#pragma unroll
                for (int c = 0; c < ND; ++c)
                    B[i][c] = (((rowbits >> i) | (rowbits >> c)) & 1) ? (i == c ? 1.0 : 0.0) : double(a[jd * BS + i * ND + c]);
            bad |= !invert_block<ND>(B, dinv + int64_t(BS) * n);
        }
        if (bad) atomicOr(status, ST_NAN);
        wave_lds_handoff();  // the next node reuses the image
    }
}

template <int ND, int LAYOUT, typename T>
__global__ __launch_bounds__(256) void k_extract_dinv(int64_t N, const int64_t *__restrict__ node_ptr,
                                                      const int32_t *__restrict__ bdiag,
                                                      const int64_t *__restrict__ row_ptr,
                                                      const int64_t *__restrict__ up_base,
                                                      const T *__restrict__ values, T *__restrict__ dinv,
                                                      int *status) {
    int64_t d = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (d >= N) return;
    int64_t n = d / ND;
    int i = int(d - n * ND);
    T v = (LAYOUT == LAYOUT_SYM) ? values[ND * ND * up_base[n] + (ND + 1) * i]
                                 : values[row_ptr[d] + ND * (bdiag[n] - node_ptr[n]) + i];
    if (!(v != T(0)) || !isfinite(v)) atomicOr(status, ST_NAN);
    dinv[d] = T(1) / v;
}

inline unsigned grid_for(int64_t n, int threads) { return unsigned((n + threads - 1) / threads); }

// Resident grid of the node-centric gather: 8 blocks of 4 wavefronts per CU.
inline unsigned gather_grid(const fem_handle *h) {
    return unsigned(std::min<int64_t>(int64_t(8) * h->num_cus, (h->g.Nn + 3) / 4));
}

}  // namespace

// ------------------------------------------------------------------ launchers
#define FEM_DISPATCH_MODEL(h, CALL)                                                                  \
    switch ((h)->mat.model) {                                                                        \
    case FEM_POISSON: { constexpr int MODEL = FEM_POISSON; constexpr int ND = 1; CALL; break; }      \
    case FEM_LINEAR_ELASTIC: { constexpr int MODEL = FEM_LINEAR_ELASTIC; constexpr int ND = 3; CALL; break; } \
    case FEM_J2_PLASTIC: { constexpr int MODEL = FEM_J2_PLASTIC; constexpr int ND = 3; CALL; break; }        \
    default: { constexpr int MODEL = FEM_NEO_HOOKEAN; constexpr int ND = 3; CALL; break; }          \
    }

void launch_residual(const fem_handle *h, const double *u, const double *theta, double lf, double *scratch,
                     double *r, hipStream_t s) {
    const Graph &g = h->g;
    if (g.Ne == 0) {
        FEM_HIP(hipMemsetAsync(r, 0, g.N * sizeof(double), s));
        return;
    }
    unsigned gridE = grid_for(g.Ne, kElemsPerBlock);
    FEM_DISPATCH_MODEL(h, {
        hipLaunchKernelGGL((k_element_vec<MODEL, ND, VEC_RESIDUAL>), dim3(gridE), dim3(kThreads), 0, s, g.Ne,
                           h->m.coords, h->m.conn, g.kpos, h->m.mask, h->mat, theta, u, nullptr, h->hist, scratch,
                           h->status);
        hipLaunchKernelGGL((k_gather_vec<ND, VEC_RESIDUAL>), dim3(grid_for(g.N, 256)), dim3(256), 0, s, g.N,
                           g.ne_ptr, scratch, h->m.mask, h->m.fext, lf, nullptr, r, h->status);
    });
    FEM_HIP(hipGetLastError());
}

void launch_apply_tangent(const fem_handle *h, const double *u, const double *theta, const double *v,
                          double *scratch, double *y, hipStream_t s) {
    const Graph &g = h->g;
    if (g.Ne == 0) {
        FEM_HIP(hipMemcpyAsync(y, v, g.N * sizeof(double), hipMemcpyDeviceToDevice, s));
        return;
    }
    unsigned gridE = grid_for(g.Ne, kElemsPerBlock);
    FEM_DISPATCH_MODEL(h, {
        hipLaunchKernelGGL((k_element_vec<MODEL, ND, VEC_JVP>), dim3(gridE), dim3(kThreads), 0, s, g.Ne, h->m.coords,
                           h->m.conn, g.kpos, h->m.mask, h->mat, theta, u, v, h->hist, scratch, h->status);
        hipLaunchKernelGGL((k_gather_vec<ND, VEC_JVP>), dim3(grid_for(g.N, 256)), dim3(256), 0, s, g.N, g.ne_ptr,
                           scratch, h->m.mask, nullptr, 0.0, v, y, h->status);
    });
    FEM_HIP(hipGetLastError());
}

void launch_lift(const fem_handle *h, const double *u, const double *theta, const double *v, double *scratch,
                 double *y, hipStream_t s) {
    const Graph &g = h->g;
    if (g.Ne == 0) return;
    unsigned gridE = grid_for(g.Ne, kElemsPerBlock);
    FEM_DISPATCH_MODEL(h, {
        hipLaunchKernelGGL((k_element_vec<MODEL, ND, VEC_LIFT>), dim3(gridE), dim3(kThreads), 0, s, g.Ne,
                           h->m.coords, h->m.conn, g.kpos, h->m.mask, h->mat, theta, u, v, h->hist, scratch, h->status);
        hipLaunchKernelGGL((k_gather_vec<ND, VEC_LIFT>), dim3(grid_for(g.N, 256)), dim3(256), 0, s, g.N, g.ne_ptr,
                           scratch, h->m.mask, nullptr, 0.0, v, y, h->status);
    });
    FEM_HIP(hipGetLastError());
}

void launch_mass(const fem_handle *h, const double *x, double *scratch, double *y, hipStream_t s) {
    const Graph &g = h->g;
    if (g.Ne == 0) {
        FEM_HIP(hipMemsetAsync(y, 0, g.N * sizeof(double), s));
        return;
    }
    unsigned gridE = grid_for(g.Ne, kElemsPerBlock);
    if (g.nd == 1) {
        hipLaunchKernelGGL((k_element_mass<1>), dim3(gridE), dim3(kThreads), 0, s, g.Ne, h->m.coords, h->m.conn,
                           g.kpos, x, scratch, h->status);
        hipLaunchKernelGGL((k_gather_vec<1, VEC_MASS>), dim3(grid_for(g.N, 256)), dim3(256), 0, s, g.N, g.ne_ptr,
                           scratch, nullptr, nullptr, 0.0, nullptr, y, h->status);
    } else {
        hipLaunchKernelGGL((k_element_mass<3>), dim3(gridE), dim3(kThreads), 0, s, g.Ne, h->m.coords, h->m.conn,
                           g.kpos, x, scratch, h->status);
        hipLaunchKernelGGL((k_gather_vec<3, VEC_MASS>), dim3(grid_for(g.N, 256)), dim3(256), 0, s, g.N, g.ne_ptr,
                           scratch, nullptr, nullptr, 0.0, nullptr, y, h->status);
    }
    FEM_HIP(hipGetLastError());
}

void launch_j2_commit(const fem_handle *h, const double *u, const double *theta, hipStream_t s) {
    const Graph &g = h->g;
    if (g.Ne == 0 || h->mat.model != FEM_J2_PLASTIC) return;
    hipLaunchKernelGGL(k_j2_commit, dim3(grid_for(g.Ne, kElemsPerBlock)), dim3(kThreads), 0, s, g.Ne, h->m.coords,
                       h->m.conn, h->mat, theta, u, h->hist);
    FEM_HIP(hipGetLastError());
}

size_t j2_partials_count(int64_t n_elems) { return size_t(grid_for(n_elems, kElemsPerBlock)) * 7; }

void j2_average_stress(fem_handle *h, double out[6], hipStream_t s) {
    const Graph &g = h->g;
    for (int c = 0; c < 6; ++c) out[c] = 0.0;
    if (g.Ne == 0) return;
    const unsigned grid = grid_for(g.Ne, kElemsPerBlock);
    hipLaunchKernelGGL(k_j2_average, dim3(grid), dim3(kThreads), 0, s, g.Ne, h->m.coords, h->m.conn, h->hist,
                       h->hist_partials);
    FEM_HIP(hipGetLastError());
    std::vector<double> hp(size_t(grid) * 7);
    FEM_HIP(hipMemcpyAsync(hp.data(), h->hist_partials, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    double t[7] = {0, 0, 0, 0, 0, 0, 0};
    for (unsigned b = 0; b < grid; ++b)
        for (int c = 0; c < 7; ++c) t[c] += hp[size_t(b) * 7 + c];
    for (int c = 0; c < 6; ++c) out[c] = t[c] / t[6];
}

void launch_vjp(const fem_handle *h, const double *u, const double *theta, const double *lam, double *gout,
                hipStream_t s) {
    const Graph &g = h->g;
    if (g.Ne == 0) return;
    if (h->mat.model == FEM_J2_PLASTIC) throw Error(FEM_EINVAL, "the parameter VJP is not defined for FEM_J2_PLASTIC");
    unsigned gridE = grid_for(g.Ne, kElemsPerBlock);
    FEM_DISPATCH_MODEL(h, {
        hipLaunchKernelGGL((k_element_vec<MODEL, ND, VEC_VJP>), dim3(gridE), dim3(kThreads), 0, s, g.Ne, h->m.coords,
                           h->m.conn, g.kpos, h->m.mask, h->mat, theta, u, lam, nullptr, gout, h->status);
    });
    FEM_HIP(hipGetLastError());
}

template <typename T>
void launch_tangent(const fem_handle *h, const double *u, const double *theta, T *ke, T *values, T *dinv,
                    hipStream_t s, int layout, int precond) {
    const int bj = precond == FEM_PRECOND_BLOCK_JACOBI;
    const Graph &g = h->g;
    if (g.Ne == 0) return;
    unsigned gridE = grid_for(g.Ne, kElemsPerBlock);
    const bool node_gather = g.tgt != nullptr && g.max_deg <= kGatherMaxDeg;
    FEM_DISPATCH_MODEL(h, {
        hipLaunchKernelGGL((k_element_tangent<MODEL, ND, T>), dim3(gridE), dim3(kThreads), 0, s, g.Ne, h->m.coords,
                           h->m.conn, g.kpos, h->mat, theta, u, h->hist, ke, h->status);
        if (node_gather) {
            if (layout == LAYOUT_SYM)
                hipLaunchKernelGGL((k_gather_node<ND, LAYOUT_SYM, T>), dim3(gather_grid(h)), dim3(256), 0, s,
                                   g.Nn, g.node_ptr, g.nb_bits, g.ne_ptr, g.tgt, g.row_ptr, g.bdiag, g.up_base,
                                   h->m.mask, ke, values, dinv, bj, h->status);
            else
                hipLaunchKernelGGL((k_gather_node<ND, LAYOUT_CSR, T>), dim3(gather_grid(h)), dim3(256), 0, s,
                                   g.Nn, g.node_ptr, g.nb_bits, g.ne_ptr, g.tgt, g.row_ptr, g.bdiag, g.up_base,
                                   h->m.mask, ke, values, dinv, bj, h->status);
        } else {
            if (layout == LAYOUT_SYM)
                hipLaunchKernelGGL((k_gather_values<ND, LAYOUT_SYM, T>), dim3(grid_for(g.nnzb * ND, 256)), dim3(256),
                                   0, s, g.nnzb, g.node_ptr, g.node_nb, g.blk_row, g.blk_ptr, g.blk_src, g.row_ptr,
                                   g.bdiag, g.up_base, h->m.mask, ke, values, h->status);
            else
                hipLaunchKernelGGL((k_gather_values<ND, LAYOUT_CSR, T>), dim3(grid_for(g.nnzb * ND, 256)), dim3(256),
                                   0, s, g.nnzb, g.node_ptr, g.node_nb, g.blk_row, g.blk_ptr, g.blk_src, g.row_ptr,
                                   g.bdiag, g.up_base, h->m.mask, ke, values, h->status);
        }
    });
    FEM_HIP(hipGetLastError());
    if (dinv && !node_gather) {
        if (!bj) {
            launch_extract_dinv<T>(h, values, dinv, s, layout);
        } else {
#define FEM_BINV(ND, LY)                                                                                           \
    hipLaunchKernelGGL((k_extract_binv<ND, LY, T>), dim3(grid_for(g.Nn, 256)), dim3(256), 0, s, g.Nn, g.node_ptr, \
                       g.bdiag, g.row_ptr, g.up_base, values, dinv, h->status)
            if (g.nd == 1) {
                if (layout == LAYOUT_SYM) FEM_BINV(1, LAYOUT_SYM);
                else FEM_BINV(1, LAYOUT_CSR);
            } else {
                if (layout == LAYOUT_SYM) FEM_BINV(3, LAYOUT_SYM);
                else FEM_BINV(3, LAYOUT_CSR);
            }
#undef FEM_BINV
            FEM_HIP(hipGetLastError());
        }
    }
}

template <typename T>
void launch_extract_dinv(const fem_handle *h, const T *values, T *dinv, hipStream_t s, int layout) {
    const Graph &g = h->g;
    if (g.N == 0) return;
#define FEM_DINV(ND, LY)                                                                                         \
    hipLaunchKernelGGL((k_extract_dinv<ND, LY, T>), dim3(grid_for(g.N, 256)), dim3(256), 0, s, g.N, g.node_ptr,  \
                       g.bdiag, g.row_ptr, g.up_base, values, dinv, h->status)
    if (g.nd == 1) {
        if (layout == LAYOUT_SYM) FEM_DINV(1, LAYOUT_SYM);
        else FEM_DINV(1, LAYOUT_CSR);
    } else {
        if (layout == LAYOUT_SYM) FEM_DINV(3, LAYOUT_SYM);
        else FEM_DINV(3, LAYOUT_CSR);
    }
#undef FEM_DINV
    FEM_HIP(hipGetLastError());
}

template void launch_tangent<float>(const fem_handle *, const double *, const double *, float *, float *, float *,
                                    hipStream_t, int, int);
template void launch_tangent<double>(const fem_handle *, const double *, const double *, double *, double *,
                                     double *, hipStream_t, int, int);
template void launch_extract_dinv<float>(const fem_handle *, const float *, float *, hipStream_t, int);
template void launch_extract_dinv<double>(const fem_handle *, const double *, double *, hipStream_t, int);

}  // namespace fem

/*
 * CPU FP64 oracle for the HEX8 finite-element hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so and is
 * used exclusively by the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark.  The GPU library shares no code with it.
 *
 * It is deliberately plain: sequential loops over elements (Alg. 1 of the
 * paper, "conceptual process of matrix assembly"), dense element matrices,
 * explicit Gauss-point loops, textbook Krylov methods.  No blocking, fusion or
 * reordering.  Everything is double precision.
 *
 * Paper passages followed:
 *   strong / weak form ........................ Sec. 2.1, Eq. (strong), Eq. (weak)
 *   Newton linearisation, tangent C_ijkl ...... Sec. 2.1, Eq. (newton), Eq. (linearization)
 *   element residual R_e and K_e = dr_e/dU_e .. Sec. 2.2 (automatic differentiation paragraph)
 *   assembly loop ............................. Sec. 2.2, Alg. 1
 *   linear elasticity ......................... Sec. 2.3, Eq. (linear_elasticity)
 *   compressible neo-Hookean .................. Sec. 2.3, Eq. (neo-hookean)
 *   Jacobi-preconditioned BiCGSTAB ............ Sec. 5 (conclusions, item 2), van der Vorst 1992
 *   adjoint gradient -lambda^T dC/dtheta ...... Sec. 3, Eq. (adjoint_PDE), Eq. (adjoint_chain_simp)
 *   perfect J2 plasticity (return map) ........ Sec. 2.3, Eq. (plasticity_strong) and the update
 *                                               equations that follow it
 *
 * Readings where the paper is silent (HEX8 node order, 2x2x2 Gauss rule,
 * interpolated nodal source, symmetric Dirichlet elimination, CSR layout) are
 * the ones documented with the build; they are restated at each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_POISSON 0
#define ORC_ELASTIC 1
#define ORC_NEOHOOKE 2
#define ORC_J2 3

#define ORC_OK 0
#define ORC_EMESH (-4)      /* det(dx/dxi) <= 0 at a Gauss point */
#define ORC_EINVERTED (-5)  /* det(F) <= 0 at a Gauss point (neo-Hookean) */
#define ORC_EMAXITER (-8)
#define ORC_EBREAKDOWN (-7)

/* Worker threads of the loops marked ORC_PAR below.  1, the default, runs every loop
 * in plain sequential order, and the parity tests use the oracle that way.  More
 * threads serve only to time the oracle on all host cores and to finish large
 * reference solves: row loops are split by rows, inner products reduce per thread
 * (so their rounding order differs), and the element loop of the assembly goes
 * colour by colour (no two elements of one colour share a node, so their additions
 * never touch the same entry).  Without OpenMP the pragmas are ignored. */
static int orc_threads = 1;
void orc_set_threads(int n) { orc_threads = n < 1 ? 1 : n; }
int orc_get_threads(void) { return orc_threads; }
#define ORC_PAR _Pragma("omp parallel for schedule(static) num_threads(orc_threads) if (orc_threads > 1)")

typedef struct {
    int32_t model;     /* ORC_POISSON / ORC_ELASTIC / ORC_NEOHOOKE */
    int32_t pmap;      /* 0: modulus = theta ; 1: modulus = emin + theta^p (e0 - emin) */
    double nu;         /* Poisson ratio (linear elasticity) */
    double bulk_ratio; /* kappa = bulk_ratio * G (neo-Hookean) */
    double simp_p, simp_emin, simp_e0;
    double yield_stress; /* sigma_yield (J2 plasticity) */
} orc_material;

/* Reference coordinates of the eight HEX8 nodes (bottom face counter-clockwise, then top). */
static const double REF[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                 {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

/* ------------------------------------------------------------------ shape functions */

/* Trilinear shape functions N_a = 1/8 (1 + xi_a xi)(1 + eta_a eta)(1 + zeta_a zeta) and
 * their derivatives with respect to the reference coordinates. */
void orc_shape(const double xi[3], double N[8], double dN[8][3]) {
    for (int a = 0; a < 8; ++a) {
        double f0 = 1.0 + REF[a][0] * xi[0];
        double f1 = 1.0 + REF[a][1] * xi[1];
        double f2 = 1.0 + REF[a][2] * xi[2];
        N[a] = 0.125 * f0 * f1 * f2;
        dN[a][0] = 0.125 * REF[a][0] * f1 * f2;
        dN[a][1] = 0.125 * f0 * REF[a][1] * f2;
        dN[a][2] = 0.125 * f0 * f1 * REF[a][2];
    }
}

/* 2x2x2 Gauss-Legendre point q (xi fastest, then eta, then zeta); all weights are 1. */
void orc_gauss_point(int q, double xi[3]) {
    double g = 1.0 / sqrt(3.0);
    xi[0] = (q & 1) ? g : -g;
    xi[1] = (q & 2) ? g : -g;
    xi[2] = (q & 4) ? g : -g;
}

static double det3(const double A[3][3]) {
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
           A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

/* Inverse of a 3x3 matrix by cofactors; returns the determinant. */
static double inv3(const double A[3][3], double B[3][3]) {
    double d = det3(A);
    B[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / d;
    B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / d;
    B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / d;
    B[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / d;
    B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / d;
    B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / d;
    B[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / d;
    B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / d;
    B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / d;
    return d;
}

/* Isoparametric geometry at reference point xi: Jacobian J_ij = sum_a X_a,i dN_a/dxi_j,
 * physical gradients dN_a/dx_i = sum_j (J^-1)_ji dN_a/dxi_j.  Returns ORC_EMESH if det J <= 0. */
int orc_geometry(const double X[8][3], const double xi[3], double N[8], double gradN[8][3], double *detJ) {
    double dN[8][3], J[3][3], Ji[3][3];
    orc_shape(xi, N, dN);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int a = 0; a < 8; ++a) s += X[a][i] * dN[a][j];
            J[i][j] = s;
        }
    double d = det3(J);
    *detJ = d;
    if (!(d > 0.0)) return ORC_EMESH;
    inv3(J, Ji);
    for (int a = 0; a < 8; ++a)
        for (int i = 0; i < 3; ++i) {
            double s = 0.0;
            for (int j = 0; j < 3; ++j) s += Ji[j][i] * dN[a][j];
            gradN[a][i] = s;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------ constitutive laws */

/* Material modulus as a function of the per-element parameter theta. */
double orc_modulus(const orc_material *m, double theta) {
    if (m->pmap == 1) return m->simp_emin + pow(theta, m->simp_p) * (m->simp_e0 - m->simp_emin);
    return theta;
}

double orc_dmodulus(const orc_material *m, double theta) {
    if (m->pmap == 1) return m->simp_p * pow(theta, m->simp_p - 1.0) * (m->simp_e0 - m->simp_emin);
    return 1.0;
}

/* Neo-Hookean strain energy W(F) = G/2 (J^{-2/3} I1 - 3) + kappa/2 (J - 1)^2, I1 = tr(F^T F),
 * with G = mod, kappa = bulk_ratio * mod (Eq. neo-hookean).  Used only to pin P = dW/dF. */
double orc_nh_energy(const orc_material *m, double mod, const double F[3][3]) {
    double G = mod, kappa = m->bulk_ratio * mod;
    double J = det3(F), I1 = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) I1 += F[i][j] * F[i][j];
    return 0.5 * G * (pow(J, -2.0 / 3.0) * I1 - 3.0) + 0.5 * kappa * (J - 1.0) * (J - 1.0);
}

/* Flux f(grad u) of the strong form (Eq. strong) at a Gauss point.
 *   Poisson:     f = mod * grad u                            (row 0 of Gu / P)
 *   elasticity:  f = sigma = lambda tr(eps) I + 2 mu eps, eps = sym(grad u), E = mod
 *   neo-Hookean: f = P = dW/dF = G J^{-2/3} (F - I1/3 F^{-T}) + kappa J (J - 1) F^{-T}
 * Returns ORC_EINVERTED if det F <= 0 for the neo-Hookean law. */
int orc_flux(const orc_material *m, double mod, const double Gu[3][3], double P[3][3]) {
    memset(P, 0, 9 * sizeof(double));
    if (m->model == ORC_POISSON) {
        for (int j = 0; j < 3; ++j) P[0][j] = mod * Gu[0][j];
        return ORC_OK;
    }
    if (m->model == ORC_ELASTIC) {
        double E = mod, nu = m->nu;
        double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = E / (2.0 * (1.0 + nu));
        double eps[3][3], tr = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) eps[i][j] = 0.5 * (Gu[i][j] + Gu[j][i]);
        for (int i = 0; i < 3; ++i) tr += eps[i][i];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) P[i][j] = 2.0 * mu * eps[i][j] + (i == j ? lam * tr : 0.0);
        return ORC_OK;
    }
    /* neo-Hookean */
    double G = mod, kappa = m->bulk_ratio * mod;
    double F[3][3], Fi[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) F[i][j] = Gu[i][j] + (i == j ? 1.0 : 0.0);
    double J = det3(F);
    if (!(J > 0.0)) return ORC_EINVERTED;
    inv3(F, Fi);
    double I1 = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) I1 += F[i][j] * F[i][j];
    double c = G * pow(J, -2.0 / 3.0);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double H = Fi[j][i]; /* (F^{-T})_ij */
            P[i][j] = c * (F[i][j] - I1 / 3.0 * H) + kappa * J * (J - 1.0) * H;
        }
    return ORC_OK;
}

/* Fourth-order tangent A_iJkL = d f_iJ / d (grad u)_kL (Eq. linearization, C_ijkl = f_ij,kl),
 * derived by hand for each law.  Layout A[i][J][k][L]. */
int orc_tangent(const orc_material *m, double mod, const double Gu[3][3], double A[3][3][3][3]) {
    memset(A, 0, 81 * sizeof(double));
    if (m->model == ORC_POISSON) {
        for (int j = 0; j < 3; ++j) A[0][j][0][j] = mod;
        return ORC_OK;
    }
    if (m->model == ORC_ELASTIC) {
        double E = mod, nu = m->nu;
        double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = E / (2.0 * (1.0 + nu));
        for (int i = 0; i < 3; ++i)
            for (int J = 0; J < 3; ++J)
                for (int k = 0; k < 3; ++k)
                    for (int L = 0; L < 3; ++L)
                        A[i][J][k][L] = lam * (i == J) * (k == L) + mu * ((i == k) * (J == L) + (i == L) * (J == k));
        return ORC_OK;
    }
    double G = mod, kappa = m->bulk_ratio * mod;
    double F[3][3], Fi[3][3], H[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) F[i][j] = Gu[i][j] + (i == j ? 1.0 : 0.0);
    double J = det3(F);
    if (!(J > 0.0)) return ORC_EINVERTED;
    inv3(F, Fi);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) H[i][j] = Fi[j][i];
    double I1 = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) I1 += F[i][j] * F[i][j];
    double c = G * pow(J, -2.0 / 3.0);
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 3; ++a)
            for (int k = 0; k < 3; ++k)
                for (int b = 0; b < 3; ++b) {
                    /* a = J index, b = L index */
                    double v = c * (i == k) * (a == b);
                    v -= 2.0 / 3.0 * c * (F[i][a] * H[k][b] + H[i][a] * F[k][b]);
                    v += 2.0 / 9.0 * c * I1 * H[i][a] * H[k][b];
                    v += c * I1 / 3.0 * H[i][b] * H[k][a];
                    v += kappa * (2.0 * J * J - J) * H[i][a] * H[k][b];
                    v -= kappa * (J * J - J) * H[i][b] * H[k][a];
                    A[i][a][k][b] = v;
                }
    return ORC_OK;
}

/* ------------------------------------------------------------------ element routines */

static void gather_element(const double *coords, const int32_t *conn, int64_t e, int ndpn, const double *u,
                           double X[8][3], double Ue[24]) {
    for (int a = 0; a < 8; ++a) {
        int64_t n = conn[8 * e + a];
        for (int i = 0; i < 3; ++i) X[a][i] = coords[3 * n + i];
        if (u)
            for (int i = 0; i < ndpn; ++i) Ue[ndpn * a + i] = u[(int64_t)ndpn * n + i];
    }
}

/* grad u at a Gauss point: (grad u)_iJ = sum_a U_a,i dN_a/dX_J (rows >= ndpn stay 0). */
static void grad_u(int ndpn, const double Ue[24], const double gradN[8][3], double Gu[3][3]) {
    memset(Gu, 0, 9 * sizeof(double));
    for (int i = 0; i < ndpn; ++i)
        for (int J = 0; J < 3; ++J) {
            double s = 0.0;
            for (int a = 0; a < 8; ++a) s += Ue[ndpn * a + i] * gradN[a][J];
            Gu[i][J] = s;
        }
}

/* Element internal residual R_e[(a,i)] = int_{Omega_e} f(grad u_h) : grad phi_(a,i)
 *                                      = sum_q detJ_q sum_J f_iJ dN_a/dX_J   (2x2x2 Gauss, w = 1). */
int orc_element_residual(const orc_material *m, double mod, int ndpn, const double X[8][3], const double Ue[24],
                         double *re) {
    memset(re, 0, (size_t)(8 * ndpn) * sizeof(double));
    for (int q = 0; q < 8; ++q) {
        double xi[3], N[8], gradN[8][3], detJ, Gu[3][3], P[3][3];
        orc_gauss_point(q, xi);
        int rc = orc_geometry(X, xi, N, gradN, &detJ);
        if (rc) return rc;
        grad_u(ndpn, Ue, gradN, Gu);
        rc = orc_flux(m, mod, Gu, P);
        if (rc) return rc;
        for (int a = 0; a < 8; ++a)
            for (int i = 0; i < ndpn; ++i) {
                double s = 0.0;
                for (int J = 0; J < 3; ++J) s += P[i][J] * gradN[a][J];
                re[ndpn * a + i] += detJ * s;
            }
    }
    return ORC_OK;
}

/* Element tangent K_e[(a,i),(b,k)] = dR_e[(a,i)]/dU_e[(b,k)]
 *   = sum_q detJ_q sum_{J,L} dN_a/dX_J A_iJkL dN_b/dX_L.  Row-major [Nd][Nd], Nd = 8*ndpn. */
int orc_element_stiffness(const orc_material *m, double mod, int ndpn, const double X[8][3], const double Ue[24],
                          double *Ke) {
    int Nd = 8 * ndpn;
    memset(Ke, 0, (size_t)Nd * Nd * sizeof(double));
    for (int q = 0; q < 8; ++q) {
        double xi[3], N[8], gradN[8][3], detJ, Gu[3][3], A[3][3][3][3];
        orc_gauss_point(q, xi);
        int rc = orc_geometry(X, xi, N, gradN, &detJ);
        if (rc) return rc;
        grad_u(ndpn, Ue, gradN, Gu);
        rc = orc_tangent(m, mod, Gu, A);
        if (rc) return rc;
        for (int a = 0; a < 8; ++a)
            for (int i = 0; i < ndpn; ++i)
                for (int b = 0; b < 8; ++b)
                    for (int k = 0; k < ndpn; ++k) {
                        double s = 0.0;
                        for (int J = 0; J < 3; ++J)
                            for (int L = 0; L < 3; ++L) s += gradN[a][J] * A[i][J][k][L] * gradN[b][L];
                        Ke[(ndpn * a + i) * Nd + ndpn * b + k] += detJ * s;
                    }
    }
    return ORC_OK;
}

/* Body source load f_e[(a,i)] = int_{Omega_e} b_i N_a with b interpolated from nodal values:
 * b_h = sum_b N_b s_b  (the weak form's last term, Eq. weak). */
int orc_element_source(int ndpn, const double X[8][3], const double *se, double *fe) {
    memset(fe, 0, (size_t)(8 * ndpn) * sizeof(double));
    for (int q = 0; q < 8; ++q) {
        double xi[3], N[8], gradN[8][3], detJ;
        orc_gauss_point(q, xi);
        int rc = orc_geometry(X, xi, N, gradN, &detJ);
        if (rc) return rc;
        for (int i = 0; i < ndpn; ++i) {
            double bq = 0.0;
            for (int b = 0; b < 8; ++b) bq += N[b] * se[ndpn * b + i];
            for (int a = 0; a < 8; ++a) fe[ndpn * a + i] += detJ * N[a] * bq;
        }
    }
    return ORC_OK;
}

/* Surface load of a constant traction t on local face f = 2*axis + side of an element:
 * f_e[(a,i)] = int_{face} t_i N_a dGamma, 2x2 Gauss on the face, dGamma = |dx/ds x dx/dt| ds dt
 * (the weak form's Neumann term, Eq. weak). */
int orc_face_traction(int ndpn, const double X[8][3], int face, const double *t, double *fe) {
    memset(fe, 0, (size_t)(8 * ndpn) * sizeof(double));
    int axis = face / 2, side = face % 2;
    int s1 = (axis + 1) % 3, s2 = (axis + 2) % 3;
    double g = 1.0 / sqrt(3.0);
    for (int q = 0; q < 4; ++q) {
        double xi[3], N[8], dN[8][3], t1[3], t2[3], n[3];
        xi[axis] = side ? 1.0 : -1.0;
        xi[s1] = (q & 1) ? g : -g;
        xi[s2] = (q & 2) ? g : -g;
        orc_shape(xi, N, dN);
        for (int i = 0; i < 3; ++i) {
            t1[i] = 0.0;
            t2[i] = 0.0;
            for (int a = 0; a < 8; ++a) {
                t1[i] += X[a][i] * dN[a][s1];
                t2[i] += X[a][i] * dN[a][s2];
            }
        }
        n[0] = t1[1] * t2[2] - t1[2] * t2[1];
        n[1] = t1[2] * t2[0] - t1[0] * t2[2];
        n[2] = t1[0] * t2[1] - t1[1] * t2[0];
        double dA = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int a = 0; a < 8; ++a)
            for (int i = 0; i < ndpn; ++i) fe[ndpn * a + i] += t[i] * N[a] * dA;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ global loads */

/* External load vector F = (nodal loads) + (traction faces) + (interpolated body source). */
int orc_load_vector(int64_t n_nodes, int64_t n_elems, int ndpn, const double *coords, const int32_t *conn,
                    const double *source_nodal, int64_t n_faces, const int32_t *faces, const double *traction,
                    const double *f_nodal, double *F) {
    int64_t N = n_nodes * ndpn;
    for (int64_t d = 0; d < N; ++d) F[d] = f_nodal ? f_nodal[d] : 0.0;
    double X[8][3], se[24], fe[24];
    if (source_nodal) {
        for (int64_t e = 0; e < n_elems; ++e) {
            gather_element(coords, conn, e, ndpn, source_nodal, X, se);
            int rc = orc_element_source(ndpn, X, se, fe);
            if (rc) return rc;
            for (int a = 0; a < 8; ++a)
                for (int i = 0; i < ndpn; ++i) F[(int64_t)ndpn * conn[8 * e + a] + i] += fe[ndpn * a + i];
        }
    }
    for (int64_t f = 0; f < n_faces; ++f) {
        int64_t e = faces[2 * f];
        gather_element(coords, conn, e, ndpn, NULL, X, NULL);
        orc_face_traction(ndpn, X, faces[2 * f + 1], traction + ndpn * f, fe);
        for (int a = 0; a < 8; ++a)
            for (int i = 0; i < ndpn; ++i) F[(int64_t)ndpn * conn[8 * e + a] + i] += fe[ndpn * a + i];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ sparsity pattern */

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Sorted, duplicate-free set of nodes sharing at least one element with each node.
 * Returns arrays (caller frees) nb_ptr[n_nodes+1], nb[...]. */
static int node_neighbours(int64_t n_nodes, int64_t n_elems, const int32_t *conn, int64_t **nb_ptr_out,
                           int32_t **nb_out) {
    int64_t *ecount = calloc(n_nodes + 1, sizeof(int64_t));
    for (int64_t e = 0; e < n_elems; ++e)
        for (int a = 0; a < 8; ++a) ecount[conn[8 * e + a] + 1]++;
    for (int64_t n = 0; n < n_nodes; ++n) ecount[n + 1] += ecount[n];
    int64_t *fill = malloc(n_nodes * sizeof(int64_t));
    int32_t *elist = malloc((ecount[n_nodes] + 1) * sizeof(int32_t));
    for (int64_t n = 0; n < n_nodes; ++n) fill[n] = ecount[n];
    for (int64_t e = 0; e < n_elems; ++e)
        for (int a = 0; a < 8; ++a) elist[fill[conn[8 * e + a]]++] = (int32_t)e;
    int64_t *nb_ptr = malloc((n_nodes + 1) * sizeof(int64_t));
    int64_t cap = 0;
    for (int64_t n = 0; n < n_nodes; ++n) cap += 8 * (ecount[n + 1] - ecount[n]);
    int32_t *nb = malloc((cap + 1) * sizeof(int32_t));
    int64_t pos = 0;
    int32_t *tmp = NULL;
    int64_t tmpcap = 0;
    nb_ptr[0] = 0;
    for (int64_t n = 0; n < n_nodes; ++n) {
        int64_t k = 0, ne = ecount[n + 1] - ecount[n];
        if (8 * ne > tmpcap) {
            tmpcap = 8 * ne;
            tmp = realloc(tmp, tmpcap * sizeof(int32_t));
        }
        for (int64_t j = ecount[n]; j < ecount[n + 1]; ++j)
            for (int a = 0; a < 8; ++a) tmp[k++] = conn[8 * (int64_t)elist[j] + a];
        qsort(tmp, k, sizeof(int32_t), cmp_i32);
        for (int64_t j = 0; j < k; ++j)
            if (j == 0 || tmp[j] != tmp[j - 1]) nb[pos++] = tmp[j];
        nb_ptr[n + 1] = pos;
    }
    free(tmp);
    free(ecount);
    free(fill);
    free(elist);
    *nb_ptr_out = nb_ptr;
    *nb_out = nb;
    return 0;
}

/* CSR row pointers of the DOF graph: row d = ndpn*n + c holds every dof ndpn*m + c'
 * with m a neighbour of n.  Returns nnz.  (Alg. 1's sparse K, all N rows kept.) */
int64_t orc_pattern_rows(int64_t n_nodes, int64_t n_elems, int ndpn, const int32_t *conn, int64_t *row_ptr) {
    int64_t *nb_ptr;
    int32_t *nb;
    node_neighbours(n_nodes, n_elems, conn, &nb_ptr, &nb);
    row_ptr[0] = 0;
    for (int64_t n = 0; n < n_nodes; ++n)
        for (int c = 0; c < ndpn; ++c) {
            int64_t d = (int64_t)ndpn * n + c;
            row_ptr[d + 1] = row_ptr[d] + ndpn * (nb_ptr[n + 1] - nb_ptr[n]);
        }
    int64_t nnz = row_ptr[n_nodes * ndpn];
    free(nb_ptr);
    free(nb);
    return nnz;
}

/* Column indices, ascending within each row. */
int orc_pattern_cols(int64_t n_nodes, int64_t n_elems, int ndpn, const int32_t *conn, const int64_t *row_ptr,
                     int32_t *col_idx) {
    int64_t *nb_ptr;
    int32_t *nb;
    node_neighbours(n_nodes, n_elems, conn, &nb_ptr, &nb);
    for (int64_t n = 0; n < n_nodes; ++n)
        for (int c = 0; c < ndpn; ++c) {
            int64_t k = row_ptr[(int64_t)ndpn * n + c];
            for (int64_t j = nb_ptr[n]; j < nb_ptr[n + 1]; ++j)
                for (int c2 = 0; c2 < ndpn; ++c2) col_idx[k++] = ndpn * nb[j] + c2;
        }
    free(nb_ptr);
    free(nb);
    return 0;
}

/* Position of column `col` in row `row` (binary search); -1 if absent. */
static int64_t csr_find(const int64_t *row_ptr, const int32_t *col_idx, int64_t row, int32_t col) {
    int64_t lo = row_ptr[row], hi = row_ptr[row + 1] - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col_idx[mid] == col) return mid;
        if (col_idx[mid] < col) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

/* Slot map: slot[e][p][q] = CSR position of (dof(e,p), dof(e,q)), p,q = ndpn*a + i.
 * Implements "Add K_e to K" of Alg. 1 as values[slot[e,p,q]] += K_e[p,q]. */
int orc_slot_map(int64_t n_elems, int ndpn, const int32_t *conn, const int64_t *row_ptr, const int32_t *col_idx,
                 int32_t *slot) {
    int Nd = 8 * ndpn;
    for (int64_t e = 0; e < n_elems; ++e)
        for (int p = 0; p < Nd; ++p)
            for (int q = 0; q < Nd; ++q) {
                int64_t row = (int64_t)ndpn * conn[8 * e + p / ndpn] + p % ndpn;
                int32_t col = ndpn * conn[8 * e + q / ndpn] + q % ndpn;
                int64_t s = csr_find(row_ptr, col_idx, row, col);
                if (s < 0) return -1;
                slot[(e * Nd + p) * Nd + q] = (int32_t)s;
            }
    return 0;
}

int orc_diag_slot(int64_t n_dofs, const int64_t *row_ptr, const int32_t *col_idx, int64_t *diag) {
    for (int64_t d = 0; d < n_dofs; ++d) {
        diag[d] = csr_find(row_ptr, col_idx, d, (int32_t)d);
        if (diag[d] < 0) return -1;
    }
    return 0;
}

/* tperm[k] = CSR position of the transposed entry (col_k, row_k). */
int orc_transpose_perm(int64_t n_dofs, const int64_t *row_ptr, const int32_t *col_idx, int32_t *tperm) {
    for (int64_t r = 0; r < n_dofs; ++r)
        for (int64_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
            int64_t s = csr_find(row_ptr, col_idx, col_idx[k], (int32_t)r);
            if (s < 0) return -1;
            tperm[k] = (int32_t)s;
        }
    return 0;
}

/* ------------------------------------------------------------------ assembly (Alg. 1) */

/* Greedy colouring of the elements: element e takes the smallest colour that no
 * earlier element sharing a node with it has taken.  Writes the elements of colour c,
 * ascending, to elems[ptr[c] .. ptr[c+1]) and returns the number of colours, or -1
 * when 64 colours do not suffice. */
int orc_element_colours(int64_t n_nodes, int64_t n_elems, const int32_t *conn, int64_t ptr[65], int64_t *elems) {
    uint64_t *used = calloc(n_nodes > 0 ? n_nodes : 1, sizeof(uint64_t));
    uint8_t *colour = malloc(n_elems > 0 ? n_elems : 1);
    int nc = 0;
    for (int64_t e = 0; e < n_elems; ++e) {
        uint64_t taken = 0;
        for (int a = 0; a < 8; ++a) taken |= used[conn[8 * e + a]];
        if (taken == ~(uint64_t)0) {
            free(used);
            free(colour);
            return -1;
        }
        int c = 0;
        while (taken & ((uint64_t)1 << c)) ++c;
        colour[e] = (uint8_t)c;
        for (int a = 0; a < 8; ++a) used[conn[8 * e + a]] |= (uint64_t)1 << c;
        if (c + 1 > nc) nc = c + 1;
    }
    for (int c = 0; c <= 64; ++c) ptr[c] = 0;
    for (int64_t e = 0; e < n_elems; ++e) ptr[colour[e] + 1]++;
    for (int c = 0; c < 64; ++c) ptr[c + 1] += ptr[c];
    int64_t fill[64];
    for (int c = 0; c < 64; ++c) fill[c] = ptr[c];
    for (int64_t e = 0; e < n_elems; ++e) elems[fill[colour[e]]++] = e;
    free(used);
    free(colour);
    return nc;
}

/* One pass of Alg. 1's loop body for element e: r_e into r, K_e into the CSR values
 * through the slot map (either output may be NULL).  Ke is scratch of Nd*Nd doubles. */
static int assemble_element(int64_t e, int ndpn, const double *coords, const int32_t *conn, const orc_material *m,
                            const double *theta, const double *u, const int32_t *slot, double *r, double *values,
                            double *Ke) {
    int Nd = 8 * ndpn;
    double X[8][3], Ue[24], re[24];
    double mod = orc_modulus(m, theta[e]);
    gather_element(coords, conn, e, ndpn, u, X, Ue);
    if (r) {
        int rc = orc_element_residual(m, mod, ndpn, X, Ue, re);
        if (rc) return rc;
        for (int p = 0; p < Nd; ++p) r[(int64_t)ndpn * conn[8 * e + p / ndpn] + p % ndpn] += re[p];
    }
    if (values) {
        int rc = orc_element_stiffness(m, mod, ndpn, X, Ue, Ke);
        if (rc) return rc;
        for (int p = 0; p < Nd; ++p)
            for (int q = 0; q < Nd; ++q) values[slot[((int64_t)e * Nd + p) * Nd + q]] += Ke[p * Nd + q];
    }
    return ORC_OK;
}

/* Residual r = R_int(u; theta) - F and (optionally) tangent values in CSR order,
 * literally as Alg. 1: loop over elements, form r_e and K_e, add them into the
 * globals through the slot map.  Then Dirichlet rows/columns are eliminated
 * symmetrically: r_d = 0 and row/column d of K replaced by the unit vector. */
int orc_assemble(int64_t n_nodes, int64_t n_elems, int ndpn, const double *coords, const int32_t *conn,
                 const orc_material *m, const double *theta, const double *u, const uint8_t *mask, const double *F,
                 const int64_t *row_ptr, const int32_t *col_idx, const int32_t *slot, double *r, double *values) {
    int64_t N = n_nodes * ndpn;
    int Nd = 8 * ndpn;
    if (r)
        for (int64_t d = 0; d < N; ++d) r[d] = 0.0;
    if (values) memset(values, 0, (size_t)row_ptr[N] * sizeof(double));
    int rc = ORC_OK;
    if (orc_threads <= 1) {
        double *Ke = malloc((size_t)Nd * Nd * sizeof(double));
        for (int64_t e = 0; e < n_elems && rc == ORC_OK; ++e)
            rc = assemble_element(e, ndpn, coords, conn, m, theta, u, slot, r, values, Ke);
        free(Ke);
    } else {
        int64_t ptr[65];
        int64_t *elems = malloc((n_elems > 0 ? n_elems : 1) * sizeof(int64_t));
        int nc = orc_element_colours(n_nodes, n_elems, conn, ptr, elems);
        if (nc < 0) rc = ORC_EMAXITER;
        for (int c = 0; c < nc && rc == ORC_OK; ++c) {
#pragma omp parallel num_threads(orc_threads)
            {
                double *Ke = malloc((size_t)Nd * Nd * sizeof(double));
                int rc_t = ORC_OK;
#pragma omp for schedule(static)
                for (int64_t j = ptr[c]; j < ptr[c + 1]; ++j)
                    if (rc_t == ORC_OK)
                        rc_t = assemble_element(elems[j], ndpn, coords, conn, m, theta, u, slot, r, values, Ke);
                free(Ke);
                if (rc_t != ORC_OK) {
#pragma omp critical
                    rc = rc_t;
                }
            }
        }
        free(elems);
    }
    if (rc) return rc;
    if (r)
        for (int64_t d = 0; d < N; ++d) {
            if (F) r[d] -= F[d];
            if (mask && mask[d]) r[d] = 0.0;
        }
    if (values && mask) {
        ORC_PAR
        for (int64_t i = 0; i < N; ++i)
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                int64_t j = col_idx[k];
                if (mask[i] || mask[j]) values[k] = (i == j) ? 1.0 : 0.0;
            }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ sparse linear algebra */

void orc_spmv(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *values, const double *x,
              double *y) {
    ORC_PAR
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += values[k] * x[col_idx[k]];
        y[i] = s;
    }
}

static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : s) num_threads(orc_threads) if (orc_threads > 1)
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Jacobi-preconditioned conjugate gradients for SPD K: stops when
 * ||b - K x||_2 <= rtol ||b||_2 (recursively updated residual). */
int orc_pcg(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *values, const double *b,
            double *x, double rtol, int maxit, int *its_out, double *relres_out) {
    double *r = malloc(n * sizeof(double)), *z = malloc(n * sizeof(double)), *p = malloc(n * sizeof(double)),
           *q = malloc(n * sizeof(double)), *dinv = malloc(n * sizeof(double));
    ORC_PAR
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = csr_find(row_ptr, col_idx, i, (int32_t)i);
        dinv[i] = 1.0 / values[k];
    }
    orc_spmv(n, row_ptr, col_idx, values, x, q);
    ORC_PAR
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    double bn = sqrt(dot(n, b, b));
    if (bn == 0.0) bn = 1.0;
    ORC_PAR
    for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
    memcpy(p, z, n * sizeof(double));
    double rz = dot(n, r, z), rn = sqrt(dot(n, r, r));
    int it = 0, rc = ORC_OK;
    while (rn > rtol * bn) {
        if (it >= maxit) {
            rc = ORC_EMAXITER;
            break;
        }
        orc_spmv(n, row_ptr, col_idx, values, p, q);
        double alpha = rz / dot(n, p, q);
        ORC_PAR
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        ORC_PAR
        for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
        double rz_new = dot(n, r, z);
        double beta = rz_new / rz;
        rz = rz_new;
        ORC_PAR
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rn = sqrt(dot(n, r, r));
        ++it;
    }
    *its_out = it;
    *relres_out = rn / bn;
    free(r);
    free(z);
    free(p);
    free(q);
    free(dinv);
    return rc;
}

/* BiCGSTAB (van der Vorst 1992) with right Jacobi preconditioning M = diag(K):
 *   r = b - Kx, rhat = r; rho = alpha = omega = 1; v = p = 0
 *   loop: rho' = (rhat, r); beta = (rho'/rho)(alpha/omega); p = r + beta (p - omega v)
 *         phat = M^-1 p; v = K phat; alpha = rho' / (rhat, v); s = r - alpha v
 *         shat = M^-1 s; t = K shat; omega = (t, s)/(t, t)
 *         x += alpha phat + omega shat; r = s - omega t
 * Stops when ||r||_2 <= rtol ||b||_2. */
int orc_bicgstab(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *values, const double *b,
                 double *x, double rtol, int maxit, int *its_out, double *relres_out) {
    double *r = malloc(n * sizeof(double)), *rh = malloc(n * sizeof(double)), *p = calloc(n, sizeof(double)),
           *v = calloc(n, sizeof(double)), *ph = malloc(n * sizeof(double)), *s = malloc(n * sizeof(double)),
           *sh = malloc(n * sizeof(double)), *t = malloc(n * sizeof(double)), *dinv = malloc(n * sizeof(double));
    ORC_PAR
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = csr_find(row_ptr, col_idx, i, (int32_t)i);
        dinv[i] = 1.0 / values[k];
    }
    orc_spmv(n, row_ptr, col_idx, values, x, t);
    ORC_PAR
    for (int64_t i = 0; i < n; ++i) {
        r[i] = b[i] - t[i];
        rh[i] = r[i];
    }
    double bn = sqrt(dot(n, b, b));
    if (bn == 0.0) bn = 1.0;
    double rho = 1.0, alpha = 1.0, omega = 1.0, rn = sqrt(dot(n, r, r));
    int it = 0, rc = ORC_OK;
    while (rn > rtol * bn) {
        if (it >= maxit) {
            rc = ORC_EMAXITER;
            break;
        }
        double rho_new = dot(n, rh, r);
        if (fabs(rho_new) < 1e-300) {
            rc = ORC_EBREAKDOWN;
            break;
        }
        double beta = (rho_new / rho) * (alpha / omega);
        rho = rho_new;
        ORC_PAR
        for (int64_t i = 0; i < n; ++i) {
            p[i] = r[i] + beta * (p[i] - omega * v[i]);
            ph[i] = dinv[i] * p[i];
        }
        orc_spmv(n, row_ptr, col_idx, values, ph, v);
        alpha = rho / dot(n, rh, v);
        ORC_PAR
        for (int64_t i = 0; i < n; ++i) {
            s[i] = r[i] - alpha * v[i];
            sh[i] = dinv[i] * s[i];
        }
        orc_spmv(n, row_ptr, col_idx, values, sh, t);
        double tt = dot(n, t, t);
        omega = tt > 0.0 ? dot(n, t, s) / tt : 0.0;
        ORC_PAR
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * ph[i] + omega * sh[i];
            r[i] = s[i] - omega * t[i];
        }
        rn = sqrt(dot(n, r, r));
        ++it;
        if (omega == 0.0 && rn > rtol * bn) {
            rc = ORC_EBREAKDOWN;
            break;
        }
    }
    *its_out = it;
    *relres_out = rn / bn;
    free(r);
    free(rh);
    free(p);
    free(v);
    free(ph);
    free(s);
    free(sh);
    free(t);
    free(dinv);
    return rc;
}

/* ------------------------------------------------------------------ adjoint VJP */

/* g_e = -lambda^T dC/dtheta_e (Eq. adjoint_chain_simp, first term).  Only element e's
 * internal residual depends on theta_e, and every law here is linear in its modulus,
 * so dr_e/dtheta_e = modulus'(theta_e) * r_e(U_e; modulus = 1).  Dirichlet rows of C
 * do not depend on theta, so they are skipped. */
int orc_vjp_theta(int64_t n_elems, int ndpn, const double *coords, const int32_t *conn, const orc_material *m,
                  const double *theta, const double *u, const double *lam, const uint8_t *mask, double *g) {
    int rc_all = ORC_OK;
    ORC_PAR
    for (int64_t e = 0; e < n_elems; ++e) {
        double X[8][3], Ue[24], re[24];
        gather_element(coords, conn, e, ndpn, u, X, Ue);
        int rc = orc_element_residual(m, 1.0, ndpn, X, Ue, re);
        if (rc) {
#pragma omp critical
            rc_all = rc;
            continue;
        }
        double s = 0.0;
        for (int p = 0; p < 8 * ndpn; ++p) {
            int64_t d = (int64_t)ndpn * conn[8 * e + p / ndpn] + p % ndpn;
            if (mask && mask[d]) continue;
            s += lam[d] * re[p];
        }
        g[e] = -orc_dmodulus(m, theta[e]) * s;
    }
    return rc_all;
}

/* Per-element residual and stiffness for a list of elements (used to check sampled
 * rows of very large systems without assembling them whole). */
int orc_elements_dense(int64_t n_sel, const int64_t *sel, int ndpn, const double *coords, const int32_t *conn,
                       const orc_material *m, const double *theta, const double *u, double *re_out, double *Ke_out) {
    int Nd = 8 * ndpn;
    int rc_all = ORC_OK;
    ORC_PAR
    for (int64_t s = 0; s < n_sel; ++s) {
        double X[8][3], Ue[24];
        int64_t e = sel[s];
        double mod = orc_modulus(m, theta[e]);
        gather_element(coords, conn, e, ndpn, u, X, Ue);
        int rc = ORC_OK;
        if (re_out) rc = orc_element_residual(m, mod, ndpn, X, Ue, re_out + s * Nd);
        if (!rc && Ke_out) rc = orc_element_stiffness(m, mod, ndpn, X, Ue, Ke_out + s * Nd * Nd);
        if (rc) {
#pragma omp critical
            rc_all = rc;
        }
    }
    return rc_all;
}

/* ------------------------------------------------------------------ perfect J2 plasticity
 * Small-strain perfect J2 plasticity in the form the paper states (Sec. 2.3, the
 * plasticity paragraph): with the total strain eps^{k-1} and the stress sigma^{k-1}
 * of the previous load step,
 *   d_eps = sym(grad u^k) - eps^{k-1}
 *   sigma_trial = sigma^{k-1} + lambda tr(d_eps) I + 2 mu d_eps
 *   s = dev(sigma_trial),  |s|_vm = sqrt(3/2 s:s),  f = |s|_vm - sigma_yield
 *   sigma^k = sigma_trial - (s / |s|_vm) <f>_+
 * E = mod (per element), nu from the material.  History per Gauss point: 12 values,
 * eps^{k-1} then sigma^{k-1}, each symmetric tensor as (xx, yy, zz, yz, xz, xy). */

static void sym_from6(const double v[6], double T[3][3]) {
    T[0][0] = v[0]; T[1][1] = v[1]; T[2][2] = v[2];
    T[1][2] = T[2][1] = v[3];
    T[0][2] = T[2][0] = v[4];
    T[0][1] = T[1][0] = v[5];
}

static void sym_to6(const double T[3][3], double v[6]) {
    v[0] = T[0][0]; v[1] = T[1][1]; v[2] = T[2][2];
    v[3] = T[1][2]; v[4] = T[0][2]; v[5] = T[0][1];
}

int orc_j2_stress(const orc_material *m, double E, const double Gu[3][3], const double hist[12], double sig[3][3],
                  int *yielding) {
    double nu = m->nu;
    double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = E / (2.0 * (1.0 + nu));
    double ep[3][3], sp[3][3], de[3][3], st[3][3], dev[3][3];
    sym_from6(hist, ep);
    sym_from6(hist + 6, sp);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) de[i][j] = 0.5 * (Gu[i][j] + Gu[j][i]) - ep[i][j];
    double tr = de[0][0] + de[1][1] + de[2][2];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) st[i][j] = sp[i][j] + 2.0 * mu * de[i][j] + (i == j ? lam * tr : 0.0);
    double p = (st[0][0] + st[1][1] + st[2][2]) / 3.0, ss = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            dev[i][j] = st[i][j] - (i == j ? p : 0.0);
            ss += dev[i][j] * dev[i][j];
        }
    double svm = sqrt(1.5 * ss), f = svm - m->yield_stress;
    double ramp = 0.5 * (f + fabs(f));
    if (yielding) *yielding = f > 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) sig[i][j] = st[i][j] - (ramp > 0.0 ? dev[i][j] / svm * ramp : 0.0);
    return ORC_OK;
}

/* d sigma^k / d grad u^k (consistent tangent of the return map above; the paper obtains
 * it by automatic differentiation).  Elastic: lambda I(x)I + 2 mu I_sym.  Yielding:
 * kappa I(x)I + 2 mu (sigma_y / |s|_vm) (I_sym - I(x)I / 3 - 3/2 s(x)s / |s|_vm^2) with
 * kappa = lambda + 2 mu / 3 (the trial deviator s).  Layout A[i][J][k][L]. */
int orc_j2_tangent(const orc_material *m, double E, const double Gu[3][3], const double hist[12],
                   double A[3][3][3][3]) {
    double nu = m->nu;
    double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = E / (2.0 * (1.0 + nu));
    double ep[3][3], sp[3][3], de[3][3], st[3][3], dev[3][3];
    sym_from6(hist, ep);
    sym_from6(hist + 6, sp);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) de[i][j] = 0.5 * (Gu[i][j] + Gu[j][i]) - ep[i][j];
    double tr = de[0][0] + de[1][1] + de[2][2];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) st[i][j] = sp[i][j] + 2.0 * mu * de[i][j] + (i == j ? lam * tr : 0.0);
    double p = (st[0][0] + st[1][1] + st[2][2]) / 3.0, ss = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            dev[i][j] = st[i][j] - (i == j ? p : 0.0);
            ss += dev[i][j] * dev[i][j];
        }
    double svm = sqrt(1.5 * ss);
    int plastic = svm - m->yield_stress > 0.0;
    double kappa = lam + 2.0 * mu / 3.0;
    double mup = plastic ? mu * m->yield_stress / svm : mu;
    double beta = plastic ? 3.0 * mup / (svm * svm) : 0.0;
    for (int i = 0; i < 3; ++i)
        for (int J = 0; J < 3; ++J)
            for (int k = 0; k < 3; ++k)
                for (int L = 0; L < 3; ++L)
                    A[i][J][k][L] = (kappa - 2.0 * mup / 3.0) * (i == J) * (k == L) +
                                    mup * ((i == k) * (J == L) + (i == L) * (J == k)) - beta * dev[i][J] * dev[k][L];
    return ORC_OK;
}

/* Element residual and tangent of the J2 law (history hist_e[q*12 .. q*12+11] per Gauss
 * point); Ke may be NULL. */
static int j2_element(const orc_material *m, double E, const double X[8][3], const double Ue[24],
                      const double *hist_e, double *re, double *Ke) {
    memset(re, 0, 24 * sizeof(double));
    if (Ke) memset(Ke, 0, 24 * 24 * sizeof(double));
    for (int q = 0; q < 8; ++q) {
        double xi[3], N[8], gradN[8][3], detJ, Gu[3][3], S[3][3], A[3][3][3][3];
        orc_gauss_point(q, xi);
        int rc = orc_geometry(X, xi, N, gradN, &detJ);
        if (rc) return rc;
        grad_u(3, Ue, gradN, Gu);
        orc_j2_stress(m, E, Gu, hist_e + 12 * q, S, NULL);
        for (int a = 0; a < 8; ++a)
            for (int i = 0; i < 3; ++i) {
                double s = 0.0;
                for (int J = 0; J < 3; ++J) s += S[i][J] * gradN[a][J];
                re[3 * a + i] += detJ * s;
            }
        if (!Ke) continue;
        orc_j2_tangent(m, E, Gu, hist_e + 12 * q, A);
        for (int a = 0; a < 8; ++a)
            for (int i = 0; i < 3; ++i)
                for (int b = 0; b < 8; ++b)
                    for (int k = 0; k < 3; ++k) {
                        double s = 0.0;
                        for (int J = 0; J < 3; ++J)
                            for (int L = 0; L < 3; ++L) s += gradN[a][J] * A[i][J][k][L] * gradN[b][L];
                        Ke[(3 * a + i) * 24 + 3 * b + k] += detJ * s;
                    }
    }
    return ORC_OK;
}

/* Alg. 1 for the J2 law: residual R_int(u; history) - F and the tangent, with the same
 * symmetric Dirichlet elimination as orc_assemble.  hist [n_elems * 8 * 12]. */
int orc_j2_assemble(int64_t n_nodes, int64_t n_elems, const double *coords, const int32_t *conn,
                    const orc_material *m, const double *theta, const double *hist, const double *u,
                    const uint8_t *mask, const double *F, const int64_t *row_ptr, const int32_t *col_idx,
                    const int32_t *slot, double *r, double *values) {
    int64_t N = n_nodes * 3;
    if (r)
        for (int64_t d = 0; d < N; ++d) r[d] = 0.0;
    if (values) memset(values, 0, (size_t)row_ptr[N] * sizeof(double));
    double X[8][3], Ue[24], re[24];
    double *Ke = values ? malloc(24 * 24 * sizeof(double)) : NULL;
    for (int64_t e = 0; e < n_elems; ++e) {
        gather_element(coords, conn, e, 3, u, X, Ue);
        int rc = j2_element(m, orc_modulus(m, theta[e]), X, Ue, hist + 96 * e, re, Ke);
        if (rc) {
            free(Ke);
            return rc;
        }
        if (r)
            for (int p = 0; p < 24; ++p) r[3 * (int64_t)conn[8 * e + p / 3] + p % 3] += re[p];
        if (values)
            for (int p = 0; p < 24; ++p)
                for (int q = 0; q < 24; ++q) values[slot[((int64_t)e * 24 + p) * 24 + q]] += Ke[p * 24 + q];
    }
    free(Ke);
    if (r)
        for (int64_t d = 0; d < N; ++d) {
            if (F) r[d] -= F[d];
            if (mask && mask[d]) r[d] = 0.0;
        }
    if (values && mask)
        for (int64_t i = 0; i < N; ++i)
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                int64_t j = col_idx[k];
                if (mask[i] || mask[j]) values[k] = (i == j) ? 1.0 : 0.0;
            }
    return ORC_OK;
}

/* New history after a converged load step: eps^k = sym(grad u^k), sigma^k from the
 * return map, at every Gauss point.  hist_out may alias hist_in. */
int orc_j2_update_history(int64_t n_elems, const double *coords, const int32_t *conn, const orc_material *m,
                          const double *theta, const double *u, const double *hist_in, double *hist_out) {
    double X[8][3], Ue[24];
    for (int64_t e = 0; e < n_elems; ++e) {
        gather_element(coords, conn, e, 3, u, X, Ue);
        double E = orc_modulus(m, theta[e]);
        for (int q = 0; q < 8; ++q) {
            double xi[3], N[8], gradN[8][3], detJ, Gu[3][3], S[3][3], eps[3][3];
            orc_gauss_point(q, xi);
            int rc = orc_geometry(X, xi, N, gradN, &detJ);
            if (rc) return rc;
            grad_u(3, Ue, gradN, Gu);
            orc_j2_stress(m, E, Gu, hist_in + 96 * e + 12 * q, S, NULL);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) eps[i][j] = 0.5 * (Gu[i][j] + Gu[j][i]);
            sym_to6(eps, hist_out + 96 * e + 12 * q);
            sym_to6(S, hist_out + 96 * e + 12 * q + 6);
        }
    }
    return ORC_OK;
}

/* Volume average of the stress history (xx, yy, zz, yz, xz, xy). */
int orc_j2_average_stress(int64_t n_elems, const double *coords, const int32_t *conn, const double *hist,
                          double out[6]) {
    double X[8][3], vol = 0.0;
    memset(out, 0, 6 * sizeof(double));
    for (int64_t e = 0; e < n_elems; ++e) {
        gather_element(coords, conn, e, 3, NULL, X, NULL);
        for (int q = 0; q < 8; ++q) {
            double xi[3], N[8], gradN[8][3], detJ;
            orc_gauss_point(q, xi);
            int rc = orc_geometry(X, xi, N, gradN, &detJ);
            if (rc) return rc;
            vol += detJ;
            for (int c = 0; c < 6; ++c) out[c] += detJ * hist[96 * e + 12 * q + 6 + c];
        }
    }
    for (int c = 0; c < 6; ++c) out[c] /= vol;
    return ORC_OK;
}

"""CPU oracle of the SIMP compliance optimisation loop — TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may import
this module.  Plain numpy / scipy, FP64.

Paper, Sec. 3.2 (topology optimisation): compliance minimisation under the SIMP law of
Eq. (top_strong)/(top_weak) with the objective of Eq. (top_inverse), a 50 % material
constraint, a convolution filter that blurs the sensitivities, and the method of
moving asymptotes (Svanberg 1987) as the optimiser.  The paper gives no further
detail; the readings taken here (shared by the GPU path) are:

* sensitivity filter (Sigmund 1998): weights H_ef = max(0, r_min - |c_e - c_f|) over
  element centroids c; filtered dC/dtheta_e = sum_f H_ef theta_f dC_f /
  (max(gamma, theta_e) sum_f H_ef) with gamma = 1e-3;
* volume constraint f1(theta) = sum_e v_e theta_e / sum_e v_e - vfrac <= 0 (element
  volumes v_e from the 2x2x2 Gauss rule);
* MMA with one constraint: moving asymptotes (initial distance 0.5 of the box,
  contracted by 0.7 where the iterate oscillates, widened by 1.2 where it does not,
  kept between 0.01 and 10 box widths from the iterate), move limits 0.1 of the
  distance to the asymptote and 0.5 of the box, the convex separable approximations
  with the small regularisation (0.001 / 1.001 weights and 1e-5 / box) of Svanberg's
  later description of the method, and the one-dimensional dual solved by bisection
  on the multiplier (no artificial variables).  When the approximated constraint
  cannot be met inside the move limits even as the multiplier grows (the doubling
  reaches 2^200), the step takes that multiplier, i.e. the point of the move box that
  minimises the constraint approximation.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

from . import oracle as orc

GAMMA = 1e-3          # lower bound of theta in the sensitivity filter's denominator
ASY_INIT, ASY_DECR, ASY_INCR = 0.5, 0.7, 1.2
ALBEFA, MOVE, RAA0 = 0.1, 0.5, 1e-5
BISECT_ITERS = 100
MAX_DOUBLINGS = 200


def element_centroids(prob) -> np.ndarray:
    """Mean of the element's 8 node coordinates."""
    return prob.coords[prob.conn].mean(axis=1)


def element_volumes(prob) -> np.ndarray:
    """sum_q w_q det J_q (2x2x2 Gauss, weights 1) per element."""
    v = np.empty(prob.n_elems)
    for e in range(prob.n_elems):
        X = prob.coords[prob.conn[e]]
        v[e] = sum(orc.geometry(X, orc.gauss_point(q))[2] for q in range(8))
    return v


def filter_matrix(prob, rmin: float) -> sp.csr_matrix:
    """H_ef = max(0, rmin - |c_e - c_f|) for all element pairs closer than rmin."""
    c = element_centroids(prob)
    tree = cKDTree(c)
    pairs = tree.query_pairs(rmin, output_type="ndarray")
    rows = np.concatenate([np.arange(len(c)), pairs[:, 0], pairs[:, 1]])
    cols = np.concatenate([np.arange(len(c)), pairs[:, 1], pairs[:, 0]])
    d = np.linalg.norm(c[rows] - c[cols], axis=1)
    w = np.maximum(0.0, rmin - d)
    H = sp.csr_matrix((w, (rows, cols)), shape=(len(c), len(c)))
    H.eliminate_zeros()
    return H


def sensitivity_filter(H: sp.csr_matrix, theta: np.ndarray, dc: np.ndarray) -> np.ndarray:
    return (H @ (theta * dc)) / (np.maximum(GAMMA, theta) * np.asarray(H.sum(axis=1)).ravel())


def density_filter(H: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    return (H @ x) / np.asarray(H.sum(axis=1)).ravel()


def mma_asymptotes(it, x, xold1, xold2, low, upp, xmin=0.0, xmax=1.0):
    """Asymptotes of iteration `it` (0-based)."""
    box = xmax - xmin
    if it < 2:
        return x - ASY_INIT * box, x + ASY_INIT * box
    osc = (x - xold1) * (xold1 - xold2)
    factor = np.ones_like(x)
    factor[osc > 0] = ASY_INCR
    factor[osc < 0] = ASY_DECR
    low = x - factor * (xold1 - low)
    upp = x + factor * (upp - xold1)
    low = np.clip(low, x - 10.0 * box, x - 0.01 * box)
    upp = np.clip(upp, x + 0.01 * box, x + 10.0 * box)
    return low, upp


def mma_step(it, x, xold1, xold2, df0, f1, df1, low, upp, xmin=0.0, xmax=1.0):
    """One MMA iteration for min f0 s.t. f1 <= 0 on [xmin, xmax]^n.

    df0, df1: gradients at x; f1: constraint value at x.  Returns (xnew, low, upp, lam).
    """
    box = xmax - xmin
    low, upp = mma_asymptotes(it, x, xold1, xold2, low, upp, xmin, xmax)
    alpha = np.maximum.reduce([np.full_like(x, xmin), low + ALBEFA * (x - low), x - MOVE * box])
    beta = np.minimum.reduce([np.full_like(x, xmax), upp - ALBEFA * (upp - x), x + MOVE * box])
    ux2, xl2 = (upp - x) ** 2, (x - low) ** 2
    reg = RAA0 / box
    p0 = ux2 * (1.001 * np.maximum(df0, 0) + 0.001 * np.maximum(-df0, 0) + reg)
    q0 = xl2 * (0.001 * np.maximum(df0, 0) + 1.001 * np.maximum(-df0, 0) + reg)
    p1 = ux2 * (1.001 * np.maximum(df1, 0) + 0.001 * np.maximum(-df1, 0) + reg)
    q1 = xl2 * (0.001 * np.maximum(df1, 0) + 1.001 * np.maximum(-df1, 0) + reg)
    r1 = f1 - np.sum(p1 / (upp - x) + q1 / (x - low))

    def x_of(lam):
        P, Q = p0 + lam * p1, q0 + lam * q1
        sp_, sq = np.sqrt(P), np.sqrt(Q)
        return np.clip((low * sp_ + upp * sq) / (sp_ + sq), alpha, beta)

    def g(lam):  # derivative of the dual = approximated constraint at x(lam)
        xl = x_of(lam)
        return r1 + np.sum(p1 / (upp - xl) + q1 / (xl - low))

    lam_lo, lam_hi = 0.0, 1.0
    if g(0.0) <= 0.0:
        lam = 0.0
    else:
        doublings = 0
        while g(lam_hi) > 0.0 and doublings < MAX_DOUBLINGS:
            lam_lo, lam_hi = lam_hi, 2.0 * lam_hi
            doublings += 1
        if g(lam_hi) > 0.0:  # not satisfiable inside the move limits
            lam = lam_hi
        else:
            for _ in range(BISECT_ITERS):
                mid = 0.5 * (lam_lo + lam_hi)
                if g(mid) > 0.0:
                    lam_lo = mid
                else:
                    lam_hi = mid
            lam = 0.5 * (lam_lo + lam_hi)
    return x_of(lam), low, upp, lam


def compliance_loop(prob, n_iter: int, rmin: float, vfrac: float = 0.5, linear: str = "direct"):
    """The SIMP compliance loop: solve, C = F.U, dC/dtheta by the adjoint (lambda = U
    for this self-adjoint objective), sensitivity filter, MMA step.  Returns the
    density history and the compliance history."""
    H = filter_matrix(prob, rmin)
    v = element_volumes(prob)
    F = orc.load_vector(prob)
    x = prob.theta.copy()
    xold1, xold2 = x.copy(), x.copy()
    low, upp = np.zeros_like(x), np.ones_like(x)
    hist_x, hist_c = [x.copy()], []
    for it in range(n_iter):
        u = orc.newton_solve(prob, theta=x, linear=linear, rtol=1e-12)
        c = float(F @ u)
        dc = orc.vjp_theta(prob, u, u, theta=x)
        dcf = sensitivity_filter(H, x, dc)
        f1 = float(v @ x) / v.sum() - vfrac
        df1 = v / v.sum()
        xnew, low, upp, _ = mma_step(it, x, xold1, xold2, dcf, f1, df1, low, upp)
        xold2, xold1, x = xold1, x, xnew
        hist_x.append(x.copy())
        hist_c.append(c)
    return hist_x, hist_c

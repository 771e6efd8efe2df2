"""CPU oracle of the two-level aggregation preconditioner — TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may import
this module.  Plain numpy / scipy, FP64.

The paper names the Jacobi-preconditioned linear solver as the bottleneck of its
method (Sec. 5, item 2) and prescribes nothing stronger; this is the multilevel
preconditioner the build adds on that basis.  Definition (every choice below is a
reading, taken identically by the GPU path):

* Aggregation of the node graph (nodes sharing an element), in node order: a node
  whose neighbours (itself included) are all unaggregated founds an aggregate made of
  exactly that neighbourhood; afterwards every leftover node joins the aggregate of its
  first aggregated neighbour in ascending neighbour order, or founds a singleton.
* Coarse space: per aggregate the 6 rigid-body modes of elasticity (3 translations and
  the rotations (-y, x, 0), (0, -z, y), (z, 0, -x) about the aggregate's node
  centroid; for ndpn = 1 the constant), with Dirichlet dofs zeroed, orthonormalised by
  modified Gram-Schmidt in that column order; a column whose norm after projection
  falls below 1e-10 of its original norm is dropped (set to zero).  P holds the
  columns (6 per aggregate), so A_c = P^T A P, with a unit diagonal entry for every
  dropped column.
* Chebyshev iteration on D^{-1} A (Saad, "Iterative Methods for Sparse Linear
  Systems", 2nd ed., Alg. 12.1) on the interval [lmax / 30, lmax].  On the fine level
  lmax is the Gershgorin bound max_i sum_j |A_ij| / |A_ii|, an upper bound of the
  spectrum: an interval that misses the top of the spectrum amplifies those modes and
  makes the preconditioner indefinite.  On the coarse level, whose polynomial has a
  higher degree and is hurt more by a loose interval, lmax is 1.2 times the power
  estimate ||D^{-1} A x|| / ||x|| after 12 normalised steps from x_i = sin(1 + i),
  capped by the coarse operator's Gershgorin bound.
* One application z = M r: pre-smoothing (`smooth_degree` Chebyshev steps from 0),
  the residual r - A z restricted by P^T, the coarse correction (`coarse_degree`
  Chebyshev steps from 0 on A_c), prolongation by P, and post-smoothing
  (`smooth_degree` Chebyshev steps continuing from z).  The pre and post smoothers
  are the same polynomial, so M is symmetric; the CG that uses it is the plain
  preconditioned CG.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

POWER_STEPS = 12
LMAX_SAFETY = 1.2
CHEB_RATIO = 30.0
DROP_TOL = 1e-10


def node_graph(pat, ndpn: int):
    """Node adjacency (CSR over nodes, neighbours ascending) from the dof pattern."""
    A = sp.csr_matrix((np.ones(pat.nnz), pat.col_idx, pat.row_ptr), shape=(pat.n, pat.n))
    rows = np.repeat(np.arange(pat.n), np.diff(pat.row_ptr)) // ndpn
    G = sp.csr_matrix((np.ones(A.nnz), (rows, A.indices // ndpn)), shape=(pat.n // ndpn, pat.n // ndpn))
    G.sum_duplicates()
    G.sort_indices()
    return G.indptr.astype(np.int64), G.indices.astype(np.int64)


def aggregate(ptr, nb):
    """Aggregate index of every node (rule in the module docstring)."""
    n = ptr.size - 1
    agg = np.full(n, -1, dtype=np.int64)
    na = 0
    for i in range(n):
        if agg[i] >= 0:
            continue
        nbr = nb[ptr[i]:ptr[i + 1]]
        if np.all(agg[nbr] < 0):
            agg[nbr] = na
            na += 1
    for i in range(n):
        if agg[i] >= 0:
            continue
        nbr = nb[ptr[i]:ptr[i + 1]]
        owners = agg[nbr][agg[nbr] >= 0]
        if owners.size:
            agg[i] = owners[0]
        else:
            agg[i] = na
            na += 1
    return agg, na


def rigid_modes(xyz_rel: np.ndarray, ndpn: int) -> np.ndarray:
    """Near-null-space columns of one node (ndpn x 6, or 1 x 1 for scalar problems)."""
    if ndpn == 1:
        return np.ones((1, 1))
    x, y, z = xyz_rel
    B = np.zeros((3, 6))
    B[:, :3] = np.eye(3)
    B[:, 3] = (-y, x, 0.0)
    B[:, 4] = (0.0, -z, y)
    B[:, 5] = (z, 0.0, -x)
    return B


def prolongator(prob, agg, na):
    """P (N x nc*na, nc = 6 or 1) and the list of dropped coarse columns."""
    nd = prob.ndpn
    nc = 6 if nd == 3 else 1
    mask = prob.dirichlet_mask.astype(bool)
    rows, cols, vals = [], [], []
    dropped = []
    for a in range(na):
        nodes = np.flatnonzero(agg == a)
        c = prob.coords[nodes].mean(axis=0)
        B = np.vstack([rigid_modes(prob.coords[k] - c, nd) for k in nodes])
        dofs = (nd * nodes[:, None] + np.arange(nd)).ravel()
        B[mask[dofs]] = 0.0
        Q = np.zeros_like(B)
        for j in range(nc):  # modified Gram-Schmidt, columns in order
            v = B[:, j].copy()
            n0 = np.linalg.norm(v)
            for k in range(j):
                v -= (Q[:, k] @ v) * Q[:, k]
            nv = np.linalg.norm(v)
            if n0 > 0.0 and nv > DROP_TOL * n0:
                Q[:, j] = v / nv
            else:
                dropped.append(nc * a + j)
        for j in range(nc):
            rows += list(dofs)
            cols += [nc * a + j] * dofs.size
            vals += list(Q[:, j])
    P = sp.csr_matrix((vals, (rows, cols)), shape=(prob.n_dofs, nc * na))
    P.eliminate_zeros()
    return P, np.array(dropped, dtype=np.int64)


def coarse_operator(A, P, dropped):
    Ac = (P.T @ A @ P).tolil()
    for j in dropped:
        Ac[j, j] = 1.0
    return Ac.tocsr()


def gershgorin_bound(A, dinv):
    """max_i |dinv_i| sum_j |A_ij|: the row-sum norm of D^{-1} A, which bounds its spectrum."""
    return float(np.max(np.asarray(abs(A).sum(axis=1)).ravel() * np.abs(dinv)))


def lmax_estimate(A, dinv):
    x = np.sin(1.0 + np.arange(A.shape[0], dtype=np.float64))
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(POWER_STEPS):
        y = dinv * (A @ x)
        lam = np.linalg.norm(y)  # ||x|| = 1
        x = y / lam
    return min(LMAX_SAFETY * lam, gershgorin_bound(A, dinv))


def chebyshev(A, dinv, r, lmax, degree, z=None):
    """`degree` Chebyshev steps for A z = r on [lmax / 30, lmax] of D^{-1} A, from z (or 0)."""
    a, b = lmax / CHEB_RATIO, lmax
    theta, delta = 0.5 * (b + a), 0.5 * (b - a)
    sigma = theta / delta
    rho = 1.0 / sigma
    if z is None:
        z = np.zeros_like(r)
        rc = r.copy()
    else:
        z = z.copy()
        rc = r - A @ z
    d = dinv * rc / theta
    z += d
    for _ in range(1, degree):
        rc -= A @ d
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * rc)
        z += d
        rho = rho_new
    return z


class TwoLevel:
    """The preconditioner for one assembled (Dirichlet-eliminated) matrix A."""

    def __init__(self, prob, pat, A, smooth_degree: int = 1, coarse_degree: int = 16):
        self.A = sp.csr_matrix(A)
        ptr, nb = node_graph(pat, prob.ndpn)
        self.agg, self.na = aggregate(ptr, nb)
        self.P, self.dropped = prolongator(prob, self.agg, self.na)
        self.Ac = coarse_operator(self.A, self.P, self.dropped)
        self.dinv = 1.0 / self.A.diagonal()
        self.dcinv = 1.0 / self.Ac.diagonal()
        self.lmax = gershgorin_bound(self.A, self.dinv)
        self.lmax_c = lmax_estimate(self.Ac, self.dcinv)
        self.s, self.m = smooth_degree, coarse_degree

    def apply(self, r):
        z = chebyshev(self.A, self.dinv, r, self.lmax, self.s)
        rc = self.P.T @ (r - self.A @ z)
        ec = chebyshev(self.Ac, self.dcinv, rc, self.lmax_c, self.m)
        z = z + self.P @ ec
        return chebyshev(self.A, self.dinv, r, self.lmax, self.s, z)


def pcg(A, b, apply, rtol: float, max_it: int = 5000):
    """Preconditioned CG from x = 0 to ||b - A x|| <= rtol ||b||; returns (x, iterations)."""
    x = np.zeros_like(b)
    r = b.copy()
    z = apply(r)
    p = z.copy()
    rz = r @ z
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0
    for it in range(max_it):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) <= rtol * bn:
            return x, it + 1
        z = apply(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, max_it

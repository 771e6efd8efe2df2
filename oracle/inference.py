"""CPU oracle of the full-field inference loop — TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may import
this module.  Plain numpy / scipy, FP64.

Paper, Sec. 3.1 (full-field inference from sparse observations): the linear Poisson
problem -alpha Lap u = b with u = 0 on the boundary, Eq. (full_field_forward) /
Eq. (full_field_weak); the parameter theta is the discretised source b (nodal values,
interpolated with the shape functions, so F(theta) = M theta with the consistent mass
matrix M); the objective of Eq. (full_field_inverse), J = sum over the observed dofs
of (U[i] - U_obs,i)^2; the gradient by the adjoint (Sec. 3, Eq. (adjoint_PDE)):
K lambda = dJ/dU with lambda_D = 0, dJ/dtheta = -lambda^T dC/dtheta = M lambda since
C = K U - M theta; the optimiser is limited-memory BFGS.  Readings (the paper uses
SciPy's L-BFGS-B and states nothing more): memory 10, two-loop recursion with the
initial scaling s^T y / y^T y (identity at the first iteration), first trial step
1 / ||g|| then 1, backtracking Armijo line search (c1 = 1e-4, halving, at most 40
trials), pairs with s^T y <= 1e-16 s^T s skipped.
"""
from __future__ import annotations

import numpy as np

from . import oracle as orc

MEMORY = 10
C1 = 1e-4
MAX_HALVINGS = 40


def mass_apply(prob, x_nodal: np.ndarray) -> np.ndarray:
    """M x: the consistent load of the nodal source x (shape functions, 2x2x2 Gauss)."""
    q = _source_only(prob, x_nodal)
    return orc.load_vector(q)


def _source_only(prob, src):
    import copy
    q = copy.copy(prob)
    q.source_nodal = np.asarray(src, dtype=np.float64).reshape(prob.n_nodes * prob.ndpn)
    q.traction_faces, q.traction, q.f_nodal = None, None, None
    return q


class Inference:
    """Forward map theta -> U, objective and gradient, with the stiffness factorised once."""

    def __init__(self, prob, obs_idx: np.ndarray, obs_val: np.ndarray):
        self.prob = prob
        self.obs_idx = np.asarray(obs_idx)
        self.obs_val = np.asarray(obs_val, dtype=np.float64)
        pat = orc.Pattern(prob)
        _, vals = orc.assemble(prob, pat, np.zeros(prob.n_dofs), residual=False, matrix=True)
        import scipy.sparse.linalg as spla
        self.lu = spla.splu(pat.matrix(vals).tocsc())
        self.mask = prob.dirichlet_mask.astype(bool)
        self.n_solves = 0

    def solve(self, theta: np.ndarray) -> np.ndarray:
        F = mass_apply(self.prob, theta)
        F[self.mask] = 0.0  # u = 0 on the boundary (eliminated rows)
        self.n_solves += 1
        return self.lu.solve(F)

    def value(self, theta) -> float:
        u = self.solve(theta)
        r = u[self.obs_idx] - self.obs_val
        return float(r @ r)

    def value_and_grad(self, theta):
        u = self.solve(theta)
        r = u[self.obs_idx] - self.obs_val
        dJdu = np.zeros(self.prob.n_dofs)
        dJdu[self.obs_idx] = 2.0 * r
        dJdu[self.mask] = 0.0
        lam = self.lu.solve(dJdu)  # K is symmetric after the symmetric elimination
        lam[self.mask] = 0.0
        return float(r @ r), mass_apply(self.prob, lam)


def lbfgs(fun, theta0: np.ndarray, n_iter: int):
    """Minimise with L-BFGS (readings above).  Returns (theta history, J history)."""
    x = np.array(theta0, dtype=np.float64)
    J, g = fun.value_and_grad(x)
    S, Y = [], []
    hist_x, hist_J = [x.copy()], [J]
    for k in range(n_iter):
        # two-loop recursion: d = -H g
        q = g.copy()
        alphas = []
        for s, y in reversed(list(zip(S, Y))):
            a = (s @ q) / (y @ s)
            alphas.append(a)
            q -= a * y
        gamma = (S[-1] @ Y[-1]) / (Y[-1] @ Y[-1]) if S else 1.0
        r = gamma * q
        for (s, y), a in zip(zip(S, Y), reversed(alphas)):
            b = (y @ r) / (y @ s)
            r += (a - b) * s
        d = -r
        gd = g @ d
        t = 1.0 / np.linalg.norm(g) if k == 0 else 1.0
        for _ in range(MAX_HALVINGS):
            Jt = fun.value(x + t * d)
            if Jt <= J + C1 * t * gd:
                break
            t *= 0.5
        xn = x + t * d
        Jn, gn = fun.value_and_grad(xn)
        s, y = xn - x, gn - g
        if s @ y > 1e-16 * (s @ s):
            S.append(s)
            Y.append(y)
            if len(S) > MEMORY:
                S.pop(0)
                Y.pop(0)
        x, J, g = xn, Jn, gn
        hist_x.append(x.copy())
        hist_J.append(J)
    return hist_x, hist_J

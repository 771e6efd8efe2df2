"""Full-field inference from sparse observations on the GPU (Sec. 3.1 of the paper).

The parameter theta is the nodal source of the Poisson problem -alpha Lap u = b with
u = 0 on the boundary.  One evaluation: F = M theta (fem_mass_apply), fem_set_load,
the forward solve (fem_newton_solve; linear, so one correction plus its check), the
misfit J = sum over the observed dofs of (U[i] - U_obs,i)^2 and dJ/dU
(fem_obs_misfit); the gradient adds the adjoint solve K lambda = dJ/dU
(fem_adjoint_vjp) and dJ/dtheta = M lambda (fem_mass_apply).  The optimiser is
limited-memory BFGS: memory 10, two-loop recursion with the initial scaling
s^T y / y^T y (identity first), first trial step 1 / ||g|| then 1, backtracking Armijo
search (c1 = 1e-4, halving, at most 40 trials), pairs with s^T y <= 1e-16 s^T s
skipped.  All vector arithmetic goes through fem_dot / fem_axpby; this module keeps
buffers and scalars.
"""
from __future__ import annotations

import math
from typing import List, Optional

import torch

from . import fem

MEMORY = 10
C1 = 1e-4
MAX_HALVINGS = 40


class SourceInference:
    def __init__(self, prob: fem.Problem, obs_idx, obs_val, solve_opts: Optional[fem.SolveOpts] = None):
        self.prob = prob
        dev = prob.device
        self.idx = torch.as_tensor(obs_idx, dtype=torch.int64, device=dev).contiguous()
        self.obs = torch.as_tensor(obs_val, dtype=torch.float64, device=dev).contiguous()
        self.opts = solve_opts if solve_opts is not None else prob.opts(
            precision=fem.PREC_FP64, krylov=fem.CG, n_load_steps=1, newton_rtol=1e-12, krylov_rtol=1e-10,
            adjoint_rtol=1e-12)
        n = prob.n_dofs
        self.F = torch.empty(n, dtype=torch.float64, device=dev)
        self.dJdu = torch.empty(n, dtype=torch.float64, device=dev)
        self.g_elem = torch.empty(prob.n_elems, dtype=torch.float64, device=dev)
        self.ws = fem._vector_workspace(max(n, self.idx.numel()), dev)
        self.n_solves = 0

    def solve(self, theta: torch.Tensor) -> torch.Tensor:
        p = self.prob
        p.mass_apply(theta, out=self.F)
        p.set_load(self.F)
        u, _ = p.newton_solve(opts=self.opts)
        self.n_solves += 1
        return u

    def value(self, theta: torch.Tensor) -> float:
        u = self.solve(theta)
        return fem.obs_misfit(u, self.idx, self.obs, self.dJdu, self.ws)

    def value_and_grad(self, theta: torch.Tensor):
        u = self.solve(theta)
        J = fem.obs_misfit(u, self.idx, self.obs, self.dJdu, self.ws)
        _, lam, _ = self.prob.adjoint_vjp(u, self.dJdu, opts=self.opts)
        self.n_solves += 1
        return J, self.prob.mass_apply(lam)


def lbfgs(fun: SourceInference, theta0: torch.Tensor, n_iter: int):
    """L-BFGS (readings in the module docstring).  Returns (theta history, J history)."""
    dot, axpby = fem.dot, fem.axpby
    ws = fun.ws
    x = theta0.clone()
    J, g = fun.value_and_grad(x)
    S: List[torch.Tensor] = []
    Y: List[torch.Tensor] = []
    hist_x, hist_J = [x.clone()], [J]
    for k in range(n_iter):
        q = g.clone()
        alphas = []
        for s, y in reversed(list(zip(S, Y))):
            a = dot(s, q, ws) / dot(y, s, ws)
            alphas.append(a)
            axpby(-a, y, 1.0, q)
        gamma = dot(S[-1], Y[-1], ws) / dot(Y[-1], Y[-1], ws) if S else 1.0
        r = axpby(gamma, q, 0.0, torch.empty_like(q))
        for (s, y), a in zip(zip(S, Y), reversed(alphas)):
            b = dot(y, r, ws) / dot(y, s, ws)
            axpby(a - b, s, 1.0, r)
        d = axpby(-1.0, r, 0.0, r)  # d = -r (in place)
        gd = dot(g, d, ws)
        t = 1.0 / math.sqrt(dot(g, g, ws)) if k == 0 else 1.0
        xt = torch.empty_like(x)
        for _ in range(MAX_HALVINGS):
            axpby(1.0, x, 0.0, xt)
            axpby(t, d, 1.0, xt)
            if fun.value(xt) <= J + C1 * t * gd:
                break
            t *= 0.5
        xn = axpby(1.0, x, 0.0, torch.empty_like(x))
        axpby(t, d, 1.0, xn)
        Jn, gn = fun.value_and_grad(xn)
        s = axpby(1.0, xn, 0.0, torch.empty_like(x))
        axpby(-1.0, x, 1.0, s)
        y = axpby(1.0, gn, 0.0, torch.empty_like(x))
        axpby(-1.0, g, 1.0, y)
        if dot(s, y, ws) > 1e-16 * dot(s, s, ws):
            S.append(s)
            Y.append(y)
            if len(S) > MEMORY:
                S.pop(0)
                Y.pop(0)
        x, J, g = xn, Jn, gn
        hist_x.append(x.clone())
        hist_J.append(J)
    return hist_x, hist_J

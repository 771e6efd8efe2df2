"""SIMP compliance minimisation on the GPU (Sec. 3.2 of the paper).

Each iteration: solve the SIMP elasticity problem (fem_newton_solve; linear, so one
correction plus its check), the compliance C = F_ext . u (fem_dot), dC/dtheta by the
adjoint with lambda = u (the objective is self-adjoint; fem_param_vjp), the
sensitivity filter (fem_filter_apply), and one MMA step under the material-fraction
constraint sum_e v_e theta_e / sum_e v_e <= vfrac (fem_mma_update).  Every step runs
in libfem; this class only keeps the buffers and the iteration count.
"""
from __future__ import annotations

from typing import List, Optional

import torch

from . import fem


class SimpCompliance:
    def __init__(self, prob: fem.Problem, rmin: float, vfrac: float = 0.5, theta0=None,
                 solve_opts: Optional[fem.SolveOpts] = None, mma_opts: Optional[fem.MmaOpts] = None):
        self.prob = prob
        self.vfrac = float(vfrac)
        self.opts = solve_opts if solve_opts is not None else prob.opts(
            precision=fem.PREC_FP64, krylov=fem.CG, n_load_steps=1, newton_rtol=1e-12, krylov_rtol=1e-10)
        self.mma_opts = mma_opts if mma_opts is not None else fem.mma_default_opts()
        prob.filter_setup(rmin)
        n = prob.n_elems
        self.dvol = prob.element_volumes(normalized=True)  # gradient of the material fraction
        self.F = prob.load_vector()
        x = prob.theta if theta0 is None else prob._f64(theta0, n)
        self.x = x.clone()
        self.xold1 = x.clone()
        self.xold2 = x.clone()
        self.low = torch.zeros_like(self.x)
        self.upp = torch.ones_like(self.x)
        self.ws = fem._vector_workspace(max(n, prob.n_dofs), self.x.device)
        self.it = 0
        self.u = None
        self.compliance: List[float] = []
        self.volume: List[float] = []
        self.stats = []

    def step(self) -> float:
        """One optimisation iteration; returns the compliance at the incoming design."""
        p = self.prob
        u, st = p.newton_solve(theta=self.x, opts=self.opts)
        c = fem.dot(self.F, u, self.ws)
        dc = p.param_vjp(u, u, theta=self.x)
        dcf = p.filter_apply(dc, fem.FILTER_SENSITIVITY, theta=self.x)
        frac = fem.dot(self.dvol, self.x, self.ws)
        xnew, _ = fem.mma_update(self.it, self.x, self.xold1, self.xold2, dcf, frac - self.vfrac, self.dvol,
                                 self.low, self.upp, self.mma_opts, self.ws)
        self.xold2, self.xold1, self.x = self.xold1, self.x, xnew
        self.it += 1
        self.u = u
        self.compliance.append(c)
        self.volume.append(frac)
        self.stats.append(st)
        return c

    def run(self, n_iter: int) -> List[float]:
        for _ in range(n_iter):
            self.step()
        return self.compliance

"""CPU oracle of perfect J2 plasticity over a loading path — TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may import
this module.  Wraps the C routines orc_j2_* (the return map of Sec. 2.3, plasticity
paragraph, and its consistent tangent) and adds the load-step loop: per load step,
Newton's method with the history of the previous step fixed (lifted first iteration
as in oracle.newton_solve), then the history update eps^k = sym(grad u^k),
sigma^k = return map.
"""
from __future__ import annotations

import ctypes
from typing import List

import numpy as np

from . import oracle as orc
from .oracle import OracleError, Pattern, _c, _ptr, lib, material, spmv, linear_solve


def j2_stress(prob, E: float, Gu, hist):
    S = np.zeros((3, 3))
    y = ctypes.c_int(0)
    lib().orc_j2_stress(ctypes.byref(material(prob)), E, _c(Gu, np.float64), _c(hist, np.float64), S,
                        ctypes.byref(y))
    return S, bool(y.value)


def j2_tangent(prob, E: float, Gu, hist):
    A = np.zeros((3, 3, 3, 3))
    lib().orc_j2_tangent(ctypes.byref(material(prob)), E, _c(Gu, np.float64), _c(hist, np.float64), A)
    return A


def new_history(prob) -> np.ndarray:
    return np.zeros(prob.n_elems * 96)


def assemble(prob, pat: Pattern, u, hist, F=None, residual=True, matrix=True, eliminate=True):
    r = np.zeros(prob.n_dofs) if residual else None
    vals = np.zeros(pat.nnz) if matrix else None
    mask = _c(prob.dirichlet_mask, np.uint8) if eliminate else None
    slot = pat.slot if pat.slot is not None else np.zeros(1, dtype=np.int32)
    rc = lib().orc_j2_assemble(prob.n_nodes, prob.n_elems, _c(prob.coords, np.float64), _c(prob.conn, np.int32),
                               ctypes.byref(material(prob)), _c(prob.theta, np.float64), _c(hist, np.float64),
                               _c(u, np.float64), _ptr(mask), _ptr(_c(F, np.float64)), pat.row_ptr, pat.col_idx,
                               slot, _ptr(r), _ptr(vals))
    if rc:
        raise OracleError(rc, "j2 assemble")
    return r, vals


def update_history(prob, u, hist) -> np.ndarray:
    out = np.zeros_like(hist)
    rc = lib().orc_j2_update_history(prob.n_elems, _c(prob.coords, np.float64), _c(prob.conn, np.int32),
                                     ctypes.byref(material(prob)), _c(prob.theta, np.float64), _c(u, np.float64),
                                     _c(hist, np.float64), out)
    if rc:
        raise OracleError(rc, "j2 history")
    return out


def average_stress(prob, hist) -> np.ndarray:
    out = np.zeros(6)
    rc = lib().orc_j2_average_stress(prob.n_elems, _c(prob.coords, np.float64), _c(prob.conn, np.int32),
                                     _c(hist, np.float64), out)
    if rc:
        raise OracleError(rc, "j2 average stress")
    return out


def solve_path(prob, targets: List[np.ndarray], n_steps: int, rtol: float = 1e-12, max_it: int = 25,
               hist=None, u0=None):
    """Follows the Dirichlet values through `targets` (each reached in n_steps linear load
    steps from the previous one); returns (u, history, list of (u, average stress) after
    every load step)."""
    pat = Pattern(prob)
    mask = prob.dirichlet_mask.astype(bool)
    u = np.zeros(prob.n_dofs) if u0 is None else np.array(u0, dtype=np.float64)
    hist = new_history(prob) if hist is None else hist.copy()
    record = []
    for g_full in targets:
        uD0 = u[mask].copy()
        g = np.asarray(g_full)[mask]
        for k in range(1, n_steps + 1):
            lam = k / n_steps
            D = np.zeros(prob.n_dofs)
            D[mask] = uD0 + lam * (g - uD0) - u[mask]
            r, _ = assemble(prob, pat, u, hist, None, residual=True, matrix=False)
            _, Kfull = assemble(prob, pat, u, hist, None, residual=False, eliminate=False)
            rhs = -r - spmv(pat, Kfull, D)
            rhs[mask] = 0.0
            ref = np.linalg.norm(rhs)
            if ref > 0.0:
                _, vals = assemble(prob, pat, u, hist, None, residual=False, matrix=True)
                u += linear_solve(pat, vals, rhs, "direct")
            u += D
            r, _ = assemble(prob, pat, u, hist, None, residual=True, matrix=False)
            for it in range(max_it + 1):
                rn = np.linalg.norm(r)
                if rn <= rtol * ref or rn == 0.0:
                    break
                if it == max_it:
                    raise OracleError(-8, f"j2 newton (|r|={rn:.3e}, ref={ref:.3e})")
                _, vals = assemble(prob, pat, u, hist, None, residual=False, matrix=True)
                u += linear_solve(pat, vals, -r, "direct")
                r, _ = assemble(prob, pat, u, hist, None, residual=True, matrix=False)
            hist = update_history(prob, u, hist)
            record.append((u.copy(), average_stress(prob, hist)))
    return u, hist, record

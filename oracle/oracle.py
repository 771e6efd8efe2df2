"""CPU FP64 oracle for the HEX8 finite-element path — TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It wraps ``liboracle.so`` (plain C, built from
``oracle.c`` by ``oracle/build.py``) with numpy arrays and adds the outer loops
of the method in plain Python:

* Newton's method with incremental loading (Sec. 2.1, Eq. (newton) and
  Eq. (galerkin); load steps as in Sec. 2.3);
* the adjoint gradient (Sec. 3, Eq. (adjoint_PDE) then Eq. (adjoint_chain_simp));
* dense "Alg. 1" assembly for tiny meshes (Sec. 2.2, Alg. 1, with a dense K).

The linear solves inside Newton use either a sparse direct factorisation
(``scipy.sparse.linalg.splu``, a library primitive: exact up to rounding) or
the C Jacobi-preconditioned CG/BiCGSTAB, the paper's own solver family.
"""
from __future__ import annotations

import ctypes
import os
import pathlib
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_HERE = pathlib.Path(__file__).resolve().parent
_LIB_PATH = pathlib.Path(os.environ.get("ORACLE_LIB", str(_HERE / "liboracle.so")))

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int

EMESH, EINVERTED = -4, -5


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


class Material(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("pmap", ctypes.c_int32), ("nu", ctypes.c_double),
                ("bulk_ratio", ctypes.c_double), ("simp_p", ctypes.c_double), ("simp_emin", ctypes.c_double),
                ("simp_e0", ctypes.c_double), ("yield_stress", ctypes.c_double)]


def _load():
    if not _LIB_PATH.exists():
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(str(_LIB_PATH))
    M = ctypes.POINTER(Material)
    sig = {
        "orc_shape": (None, [_dp, _dp, _dp]),
        "orc_gauss_point": (None, [_int, _dp]),
        "orc_geometry": (_int, [_dp, _dp, _dp, _dp, _dp]),
        "orc_modulus": (ctypes.c_double, [M, ctypes.c_double]),
        "orc_dmodulus": (ctypes.c_double, [M, ctypes.c_double]),
        "orc_nh_energy": (ctypes.c_double, [M, ctypes.c_double, _dp]),
        "orc_flux": (_int, [M, ctypes.c_double, _dp, _dp]),
        "orc_tangent": (_int, [M, ctypes.c_double, _dp, _dp]),
        "orc_element_residual": (_int, [M, ctypes.c_double, _int, _dp, _dp, _dp]),
        "orc_element_stiffness": (_int, [M, ctypes.c_double, _int, _dp, _dp, _dp]),
        "orc_element_source": (_int, [_int, _dp, _dp, _dp]),
        "orc_face_traction": (_int, [_int, _dp, _int, _dp, _dp]),
        "orc_load_vector": (_int, [_i64, _i64, _int, _dp, _i32p, _vp, _i64, _vp, _vp, _vp, _dp]),
        "orc_pattern_rows": (_i64, [_i64, _i64, _int, _i32p, _i64p]),
        "orc_pattern_cols": (_int, [_i64, _i64, _int, _i32p, _i64p, _i32p]),
        "orc_slot_map": (_int, [_i64, _int, _i32p, _i64p, _i32p, _i32p]),
        "orc_diag_slot": (_int, [_i64, _i64p, _i32p, _i64p]),
        "orc_transpose_perm": (_int, [_i64, _i64p, _i32p, _i32p]),
        "orc_assemble": (_int, [_i64, _i64, _int, _dp, _i32p, M, _dp, _dp, _vp, _vp, _i64p, _i32p, _i32p, _vp,
                                _vp]),
        "orc_spmv": (None, [_i64, _i64p, _i32p, _dp, _dp, _dp]),
        "orc_pcg": (_int, [_i64, _i64p, _i32p, _dp, _dp, _dp, ctypes.c_double, _int, ctypes.POINTER(_int),
                           ctypes.POINTER(ctypes.c_double)]),
        "orc_bicgstab": (_int, [_i64, _i64p, _i32p, _dp, _dp, _dp, ctypes.c_double, _int, ctypes.POINTER(_int),
                                ctypes.POINTER(ctypes.c_double)]),
        "orc_vjp_theta": (_int, [_i64, _int, _dp, _i32p, M, _dp, _dp, _dp, _vp, _dp]),
        "orc_elements_dense": (_int, [_i64, _i64p, _int, _dp, _i32p, M, _dp, _vp, _vp, _vp]),
        "orc_set_threads": (None, [_int]),
        "orc_get_threads": (_int, []),
        "orc_element_colours": (_int, [_i64, _i64, _i32p, _i64p, _i64p]),
        "orc_j2_stress": (_int, [M, ctypes.c_double, _dp, _dp, _dp, ctypes.POINTER(_int)]),
        "orc_j2_tangent": (_int, [M, ctypes.c_double, _dp, _dp, _dp]),
        "orc_j2_assemble": (_int, [_i64, _i64, _dp, _i32p, M, _dp, _dp, _dp, _vp, _vp, _i64p, _i32p, _i32p, _vp,
                                   _vp]),
        "orc_j2_update_history": (_int, [_i64, _dp, _i32p, M, _dp, _dp, _dp, _dp]),
        "orc_j2_average_stress": (_int, [_i64, _dp, _i32p, _dp, _dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = _load()
    return _lib


class threads:
    """Runs the oracle's loops on n host threads inside the block (1 outside it: the
    sequential oracle).  Assembly then adds elements colour by colour and inner
    products reduce per thread, so results agree with the sequential ones to rounding."""

    def __init__(self, n: int):
        self.n = max(1, int(n))

    def __enter__(self):
        self.prev = lib().orc_get_threads()
        lib().orc_set_threads(self.n)
        return self

    def __exit__(self, *exc):
        lib().orc_set_threads(self.prev)


def element_colours(prob):
    """Greedy element colouring used by the threaded assembly: (ptr[65], elems)."""
    ptr = np.zeros(65, dtype=np.int64)
    elems = np.zeros(max(prob.n_elems, 1), dtype=np.int64)
    nc = lib().orc_element_colours(prob.n_nodes, prob.n_elems, _c(prob.conn, np.int32), ptr, elems)
    if nc < 0:
        raise OracleError(nc, "element colouring (more than 64 colours)")
    return ptr[:nc + 1].copy(), elems[:prob.n_elems]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def material(prob) -> Material:
    return Material(prob.model, prob.pmap, prob.nu, prob.bulk_ratio, prob.simp_p, prob.simp_emin, prob.simp_e0,
                    getattr(prob, "yield_stress", 0.0))


# ----------------------------------------------------------------------------- element level

def shape(xi):
    N = np.zeros(8)
    dN = np.zeros((8, 3))
    lib().orc_shape(np.asarray(xi, dtype=np.float64), N, dN)
    return N, dN


def gauss_point(q):
    xi = np.zeros(3)
    lib().orc_gauss_point(q, xi)
    return xi


def geometry(X, xi):
    N = np.zeros(8)
    gN = np.zeros((8, 3))
    detJ = np.zeros(1)
    rc = lib().orc_geometry(_c(X, np.float64), np.asarray(xi, dtype=np.float64), N, gN, detJ)
    if rc:
        raise OracleError(rc, "geometry")
    return N, gN, float(detJ[0])


def flux(mat: Material, mod: float, Gu):
    P = np.zeros((3, 3))
    rc = lib().orc_flux(ctypes.byref(mat), mod, _c(Gu, np.float64), P)
    if rc:
        raise OracleError(rc, "flux")
    return P


def tangent(mat: Material, mod: float, Gu):
    A = np.zeros((3, 3, 3, 3))
    rc = lib().orc_tangent(ctypes.byref(mat), mod, _c(Gu, np.float64), A)
    if rc:
        raise OracleError(rc, "tangent")
    return A


def nh_energy(mat: Material, mod: float, F) -> float:
    return lib().orc_nh_energy(ctypes.byref(mat), mod, _c(F, np.float64))


def element_residual(mat, mod, ndpn, X, Ue):
    re = np.zeros(24)
    Ue24 = np.zeros(24)
    Ue24[:8 * ndpn] = np.ravel(Ue)
    rc = lib().orc_element_residual(ctypes.byref(mat), mod, ndpn, _c(X, np.float64), Ue24, re)
    if rc:
        raise OracleError(rc, "element residual")
    return re[:8 * ndpn]


def element_stiffness(mat, mod, ndpn, X, Ue):
    Nd = 8 * ndpn
    Ke = np.zeros(Nd * Nd)
    Ue24 = np.zeros(24)
    Ue24[:Nd] = np.ravel(Ue)
    rc = lib().orc_element_stiffness(ctypes.byref(mat), mod, ndpn, _c(X, np.float64), Ue24, Ke)
    if rc:
        raise OracleError(rc, "element stiffness")
    return Ke.reshape(Nd, Nd)


def face_traction(ndpn, X, face, t):
    fe = np.zeros(24)
    lib().orc_face_traction(ndpn, _c(X, np.float64), face, np.asarray(t, dtype=np.float64), fe)
    return fe[:8 * ndpn]


# ----------------------------------------------------------------------------- pattern

class Pattern:
    """CSR pattern of the DOF graph plus the slot map (all host arrays)."""

    def __init__(self, prob, with_slot: bool = True, with_transpose: bool = False):
        L = lib()
        conn = _c(prob.conn, np.int32)
        N = prob.n_dofs
        self.n = N
        self.row_ptr = np.zeros(N + 1, dtype=np.int64)
        self.nnz = int(L.orc_pattern_rows(prob.n_nodes, prob.n_elems, prob.ndpn, conn, self.row_ptr))
        self.col_idx = np.zeros(self.nnz, dtype=np.int32)
        L.orc_pattern_cols(prob.n_nodes, prob.n_elems, prob.ndpn, conn, self.row_ptr, self.col_idx)
        self.diag_slot = np.zeros(N, dtype=np.int64)
        if L.orc_diag_slot(N, self.row_ptr, self.col_idx, self.diag_slot):
            raise OracleError(-1, "diag slot")
        Nd = 8 * prob.ndpn
        self.slot = None
        if with_slot:
            self.slot = np.zeros(prob.n_elems * Nd * Nd, dtype=np.int32)
            if L.orc_slot_map(prob.n_elems, prob.ndpn, conn, self.row_ptr, self.col_idx, self.slot):
                raise OracleError(-1, "slot map")
            self.slot = self.slot.reshape(prob.n_elems, Nd, Nd)
        self.tperm = None
        if with_transpose:
            self.tperm = np.zeros(self.nnz, dtype=np.int32)
            if L.orc_transpose_perm(N, self.row_ptr, self.col_idx, self.tperm):
                raise OracleError(-1, "transpose perm")

    def matrix(self, values):
        return sp.csr_matrix((values, self.col_idx, self.row_ptr), shape=(self.n, self.n))


# ----------------------------------------------------------------------------- global operations

def load_vector(prob) -> np.ndarray:
    F = np.zeros(prob.n_dofs)
    src = _c(prob.source_nodal, np.float64)
    faces = _c(prob.traction_faces, np.int32)
    trac = _c(prob.traction, np.float64)
    fn = _c(prob.f_nodal, np.float64)
    nf = 0 if faces is None else faces.shape[0]
    rc = lib().orc_load_vector(prob.n_nodes, prob.n_elems, prob.ndpn, _c(prob.coords, np.float64),
                               _c(prob.conn, np.int32), _ptr(src), nf, _ptr(faces), _ptr(trac), _ptr(fn), F)
    if rc:
        raise OracleError(rc, "load vector")
    return F


def assemble(prob, pat: Pattern, u, theta=None, F=None, residual=True, matrix=True, eliminate=True):
    """Returns (r, values): r = R_int(u) - F with Dirichlet rows zeroed; values = K in CSR order."""
    theta = prob.theta if theta is None else theta
    u = _c(u, np.float64)
    r = np.zeros(prob.n_dofs) if residual else None
    vals = np.zeros(pat.nnz) if matrix else None
    if matrix and pat.slot is None:
        raise ValueError("pattern built without slot map")
    mask = _c(prob.dirichlet_mask, np.uint8) if eliminate else None
    slot = pat.slot if pat.slot is not None else np.zeros(1, dtype=np.int32)
    mat = material(prob)
    rc = lib().orc_assemble(prob.n_nodes, prob.n_elems, prob.ndpn, _c(prob.coords, np.float64),
                            _c(prob.conn, np.int32), ctypes.byref(mat), _c(theta, np.float64), u, _ptr(mask),
                            _ptr(_c(F, np.float64)), pat.row_ptr, pat.col_idx, slot, _ptr(r), _ptr(vals))
    if rc:
        raise OracleError(rc, "assemble")
    return r, vals


def residual(prob, pat, u, theta=None, F=None):
    return assemble(prob, pat, u, theta, F, residual=True, matrix=False)[0]


def spmv(pat: Pattern, values, x):
    y = np.zeros(pat.n)
    lib().orc_spmv(pat.n, pat.row_ptr, pat.col_idx, _c(values, np.float64), _c(x, np.float64), y)
    return y


def krylov(pat: Pattern, values, b, method: str = "cg", rtol: float = 1e-13, maxit: int = 100000, x0=None):
    x = np.zeros(pat.n) if x0 is None else np.array(x0, dtype=np.float64)
    its = _int(0)
    rel = ctypes.c_double(0.0)
    f = lib().orc_pcg if method == "cg" else lib().orc_bicgstab
    rc = f(pat.n, pat.row_ptr, pat.col_idx, _c(values, np.float64), _c(b, np.float64), x, rtol, maxit,
           ctypes.byref(its), ctypes.byref(rel))
    if rc:
        raise OracleError(rc, f"{method} (its={its.value}, relres={rel.value:.3e})")
    return x, its.value, rel.value


def linear_solve(pat: Pattern, values, b, method: str = "direct", rtol: float = 1e-13, transpose: bool = False):
    if method == "direct":
        K = pat.matrix(values)
        if transpose:
            K = K.T
        return spla.splu(K.tocsc()).solve(b)
    if transpose:
        K = pat.matrix(values).T.tocsr()
        K.sort_indices()
        vals = K.data
        assert np.array_equal(K.indices, pat.col_idx) and np.array_equal(K.indptr, pat.row_ptr)
        values = vals
    return krylov(pat, values, b, "cg" if method == "cg" else "bicgstab", rtol=rtol)[0]


def newton_solve(prob, theta=None, linear: str = "direct", rtol: float = 1e-12, max_it: int = 25,
                 u0: Optional[np.ndarray] = None, pat: Optional[Pattern] = None, krylov_rtol: float = 1e-13,
                 history: Optional[list] = None):
    """Newton's method with incremental loading.

    Load step k of n scales the external load by k/n and moves the Dirichlet values
    linearly from their initial to their final values.  The first Newton iteration of
    a step carries the Dirichlet increment D through the tangent at the previous
    state (du = D on Dirichlet dofs, K_ff du_f = -r_f - K_fD D); later iterations
    solve K(u) du = -r(u) (Eq. newton) with Dirichlet rows and columns eliminated.
    A step stops when ||r|| <= rtol * max(||first right-hand side||, ||F_k||).
    """
    theta = prob.theta if theta is None else theta
    pat = Pattern(prob) if pat is None else pat
    F = load_vector(prob)
    mask = prob.dirichlet_mask.astype(bool)
    u = np.zeros(prob.n_dofs) if u0 is None else np.array(u0, dtype=np.float64)
    uD0 = u[mask].copy()
    g = prob.dirichlet_values[mask]
    n_steps = max(1, prob.n_load_steps)
    for k in range(1, n_steps + 1):
        lam = k / n_steps
        D = np.zeros(prob.n_dofs)
        D[mask] = uD0 + lam * (g - uD0) - u[mask]
        Fk = lam * F
        r = residual(prob, pat, u, theta, Fk)
        _, Kfull = assemble(prob, pat, u, theta, Fk, residual=False, eliminate=False)
        rhs = -r - spmv(pat, Kfull, D)
        rhs[mask] = 0.0
        ref = max(np.linalg.norm(rhs), np.linalg.norm(Fk))
        steps = [np.linalg.norm(rhs)]
        if steps[0] > rtol * ref:
            _, vals = assemble(prob, pat, u, theta, Fk, residual=False, matrix=True)
            u += linear_solve(pat, vals, rhs, linear, rtol=krylov_rtol)
        u += D
        r = residual(prob, pat, u, theta, Fk)
        for it in range(max_it + 1):
            rn = np.linalg.norm(r)
            steps.append(rn)
            if rn <= rtol * ref or rn == 0.0:
                break
            if it == max_it:
                raise OracleError(-8, f"newton load step {k} (|r|={rn:.3e}, ref={ref:.3e})")
            _, vals = assemble(prob, pat, u, theta, Fk, residual=False, matrix=True)
            u += linear_solve(pat, vals, -r, linear, rtol=krylov_rtol)
            r = residual(prob, pat, u, theta, Fk)
        if history is not None:
            history.append(steps)
    return u


def vjp_theta(prob, u, lam, theta=None):
    theta = prob.theta if theta is None else theta
    g = np.zeros(prob.n_elems)
    mat = material(prob)
    rc = lib().orc_vjp_theta(prob.n_elems, prob.ndpn, _c(prob.coords, np.float64), _c(prob.conn, np.int32),
                             ctypes.byref(mat), _c(theta, np.float64), _c(u, np.float64), _c(lam, np.float64),
                             _ptr(_c(prob.dirichlet_mask, np.uint8)), g)
    if rc:
        raise OracleError(rc, "vjp")
    return g


def adjoint_vjp(prob, u, dJdu, theta=None, linear: str = "direct", pat: Optional[Pattern] = None,
                krylov_rtol: float = 1e-13):
    """-lambda^T dC/dtheta with (dC/dU)^T lambda = (dJ/dU)^T (Eq. adjoint_PDE, Eq. adjoint_chain_simp).
    Returns (vjp, lambda)."""
    theta = prob.theta if theta is None else theta
    pat = Pattern(prob) if pat is None else pat
    _, vals = assemble(prob, pat, u, theta, None, residual=False, matrix=True)
    rhs = np.array(dJdu, dtype=np.float64)
    rhs[prob.dirichlet_mask.astype(bool)] = 0.0
    lam = linear_solve(pat, vals, rhs, linear, rtol=krylov_rtol, transpose=True)
    return vjp_theta(prob, u, lam, theta), lam


def elements_dense(prob, sel, u, theta=None, residual=True, stiffness=True):
    """Element residuals [n_sel, Nd] and stiffness matrices [n_sel, Nd, Nd] of the selected elements."""
    theta = prob.theta if theta is None else theta
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    Nd = 8 * prob.ndpn
    re = np.zeros((sel.size, Nd)) if residual else None
    Ke = np.zeros((sel.size, Nd, Nd)) if stiffness else None
    mat = material(prob)
    rc = lib().orc_elements_dense(sel.size, sel, prob.ndpn, _c(prob.coords, np.float64), _c(prob.conn, np.int32),
                                  ctypes.byref(mat), _c(theta, np.float64), _ptr(_c(u, np.float64)), _ptr(re),
                                  _ptr(Ke))
    if rc:
        raise OracleError(rc, "elements")
    return re, Ke


def element_dofs(prob, e):
    nd = prob.ndpn
    return (nd * prob.conn[e][:, None].astype(np.int64) + np.arange(nd)[None, :]).ravel()


def dense_system(prob, u, theta=None, eliminate=True):
    """Dense K and internal-force vector by Alg. 1 with a dense global matrix (tiny meshes only)."""
    theta = prob.theta if theta is None else theta
    N = prob.n_dofs
    K = np.zeros((N, N))
    R = np.zeros(N)
    re, Ke = elements_dense(prob, np.arange(prob.n_elems), u, theta)
    for e in range(prob.n_elems):
        d = element_dofs(prob, e)
        K[np.ix_(d, d)] += Ke[e]
        R[d] += re[e]
    if eliminate:
        m = prob.dirichlet_mask.astype(bool)
        K[m, :] = 0.0
        K[:, m] = 0.0
        K[m, m] = 1.0
    return K, R


def rows_of_K(prob, u, rows, theta=None, pat: Optional[Pattern] = None):
    """Sampled rows of the eliminated tangent, each summed directly from the elements
    that contain the row's node.  Returns {row: (cols sorted, values)}."""
    theta = prob.theta if theta is None else theta
    nd = prob.ndpn
    mask = prob.dirichlet_mask.astype(bool)
    nodes = np.unique(np.asarray(rows) // nd)
    # elements touching each sampled node
    hit = np.isin(prob.conn, nodes)
    elems = np.nonzero(hit.any(axis=1))[0]
    _, Ke = elements_dense(prob, elems, u, theta, residual=False)
    out = {}
    for row in rows:
        acc = {}
        if mask[row]:
            out[int(row)] = (np.array([row]), np.array([1.0]))
            continue
        n = row // nd
        for j, e in enumerate(elems):
            loc = np.nonzero(prob.conn[e] == n)[0]
            if loc.size == 0:
                continue
            p = nd * loc[0] + row % nd
            d = element_dofs(prob, e)
            for q, col in enumerate(d):
                acc[int(col)] = acc.get(int(col), 0.0) + Ke[j, p, q]
        cols = np.array(sorted(acc))
        vals = np.array([0.0 if mask[c] else acc[c] for c in cols])
        out[int(row)] = (cols, vals)
    return out

"""Thin Python binding of libfem (ctypes).

Only argument marshalling happens here: device memory comes from torch tensors,
the stream is torch's current stream, and every step of the computation runs in
the library's HIP kernels.  If libfem.so is not built the binding raises; there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import pathlib
from typing import Optional

import numpy as np
import torch

from . import inputs

_LIB_PATH = pathlib.Path(os.environ.get("FEM_LIBRARY") or pathlib.Path(__file__).resolve().parent / "libfem.so")

FEM_OK = 0
ERRORS = {-1: "FEM_EINVAL", -2: "FEM_ERANGE", -3: "FEM_EHIP", -4: "FEM_EMESH", -5: "FEM_EINVERTED",
          -6: "FEM_ENAN", -7: "FEM_EBREAKDOWN", -8: "FEM_EMAXITER", -9: "FEM_EDIVERGED", -10: "FEM_ENOMEM"}
F32, F64 = 0, 1
LAYOUT_CSR, LAYOUT_SYM_BLOCK = 0, 1
PREC_FP64, PREC_MIXED, PREC_MIXED_V64 = 0, 1, 2
CG, BICGSTAB = 0, 1
PRECOND_JACOBI, PRECOND_BLOCK_JACOBI, PRECOND_AMG = 0, 1, 2
FILTER_DENSITY, FILTER_SENSITIVITY = 0, 1
MAX_HIST = 64


class FemLibraryMissing(RuntimeError):
    pass


class FemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_elems", ctypes.c_int64), ("ndpn", ctypes.c_int32),
                ("model", ctypes.c_int32), ("pmap", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("nu", ctypes.c_double), ("bulk_ratio", ctypes.c_double), ("simp_p", ctypes.c_double),
                ("simp_emin", ctypes.c_double), ("simp_e0", ctypes.c_double), ("coords", ctypes.c_void_p),
                ("conn", ctypes.c_void_p), ("dirichlet_mask", ctypes.c_void_p), ("f_nodal", ctypes.c_void_p),
                ("source_nodal", ctypes.c_void_p), ("n_traction_faces", ctypes.c_int64),
                ("traction_faces", ctypes.c_void_p), ("traction", ctypes.c_void_p), ("yield_stress", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("krylov", ctypes.c_int32), ("n_load_steps", ctypes.c_int32),
                ("newton_max_it", ctypes.c_int32), ("newton_rtol", ctypes.c_double),
                ("newton_atol", ctypes.c_double), ("krylov_rtol", ctypes.c_double),
                ("krylov_max_it", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("adjoint_rtol", ctypes.c_double), ("adjoint_max_refine", ctypes.c_int32),
                ("profile_spmv", ctypes.c_int32), ("newton_fixed_its", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("amg_smooth_degree", ctypes.c_int32), ("amg_coarse_degree", ctypes.c_int32),
                ("max_bisections", ctypes.c_int32), ("reserved_opts", ctypes.c_int32), ("refine_rtol", ctypes.c_double)]


class SolveStats(ctypes.Structure):
    _fields_ = [("newton_its", ctypes.c_int32), ("load_steps", ctypes.c_int32), ("krylov_its_total", ctypes.c_int32),
                ("n_hist", ctypes.c_int32), ("initial_residual", ctypes.c_double),
                ("final_residual", ctypes.c_double), ("ms_residual", ctypes.c_double),
                ("ms_assemble", ctypes.c_double), ("ms_krylov", ctypes.c_double), ("ms_vjp", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("spmv_calls", ctypes.c_int32), ("krylov_unconverged", ctypes.c_int32),
                ("spmv_ms_total", ctypes.c_double), ("krylov_its", ctypes.c_int32 * MAX_HIST),
                ("residual_hist", ctypes.c_double * MAX_HIST), ("krylov_relres", ctypes.c_double * MAX_HIST),
                ("bisections", ctypes.c_int32), ("reserved_stats", ctypes.c_int32),
                ("iter_ms", ctypes.c_double * MAX_HIST)]

    def as_dict(self) -> dict:
        arrays = ("krylov_its", "residual_hist", "krylov_relres", "iter_ms")
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in arrays}
        for k in arrays:
            d[k] = list(getattr(self, k)[:self.n_hist])
        return d


class MmaOpts(ctypes.Structure):
    _fields_ = [("xmin", ctypes.c_double), ("xmax", ctypes.c_double), ("move", ctypes.c_double),
                ("asy_init", ctypes.c_double), ("asy_decr", ctypes.c_double), ("asy_incr", ctypes.c_double),
                ("albefa", ctypes.c_double), ("raa0", ctypes.c_double), ("bisect_iters", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


# Names, in the order the header declares them (checked by the CPU test-suite).
EXPORTS = ["fem_last_error", "fem_default_opts", "fem_build_pattern", "fem_pattern_host", "fem_destroy", "fem_pattern_export",
           "fem_values_count", "fem_load_vector", "fem_workspace_bytes", "fem_assemble", "fem_residual_noalloc", "fem_check", "fem_spmv",
           "fem_apply_tangent", "fem_newton_solve", "fem_adjoint_vjp", "fem_history_copy", "fem_average_stress",
           "fem_amg_setup", "fem_amg_sizes", "fem_amg_export", "fem_amg_apply", "fem_param_vjp", "fem_element_volumes",
           "fem_filter_setup", "fem_filter_apply", "fem_vector_workspace_bytes", "fem_dot", "fem_mma_default_opts",
           "fem_mma_update", "fem_mass_apply", "fem_set_load", "fem_axpby", "fem_obs_misfit"]

_lib = None


def library_path() -> pathlib.Path:
    return _LIB_PATH


def lib():
    """Loads libfem.so; raises FemLibraryMissing if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not _LIB_PATH.exists():
        raise FemLibraryMissing(f"{_LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    L = ctypes.CDLL(str(_LIB_PATH))
    vp, i64, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "fem_last_error": (ctypes.c_char_p, []),
        "fem_default_opts": (ctypes.c_int, [P(SolveOpts)]),
        "fem_build_pattern": (ctypes.c_int, [P(MeshDesc), P(vp), P(i64), P(i64)]),
        "fem_pattern_host": (ctypes.c_int, [P(MeshDesc), P(i64), P(i64), vp, vp, vp]),
        "fem_destroy": (None, [vp]),
        "fem_pattern_export": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
        "fem_values_count": (ctypes.c_int, [vp, i32, P(i64)]),
        "fem_load_vector": (ctypes.c_int, [vp, vp, vp]),
        "fem_workspace_bytes": (ctypes.c_int, [vp, P(SolveOpts), P(sz)]),
        "fem_assemble": (ctypes.c_int, [vp, vp, vp, vp, vp, i32, i32, vp, sz, vp]),
        "fem_residual_noalloc": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "fem_check": (ctypes.c_int, [vp, vp]),
        "fem_spmv": (ctypes.c_int, [vp, vp, i32, i32, i32, vp, vp, dbl, dbl, vp]),
        "fem_apply_tangent": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, sz, vp]),
        "fem_newton_solve": (ctypes.c_int, [vp, vp, vp, vp, P(SolveOpts), P(SolveStats), vp, sz, vp]),
        "fem_adjoint_vjp": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, P(SolveOpts), P(SolveStats), vp, sz, vp]),
        "fem_history_copy": (ctypes.c_int, [vp, vp, i32, vp]),
        "fem_average_stress": (ctypes.c_int, [vp, P(dbl), vp]),
        "fem_amg_setup": (ctypes.c_int, [vp]),
        "fem_amg_sizes": (ctypes.c_int, [vp, P(i64), P(i64)]),
        "fem_amg_export": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "fem_amg_apply": (ctypes.c_int, [vp, vp, vp, vp, vp, P(SolveOpts), P(dbl), vp, vp, sz, vp]),
        "fem_param_vjp": (ctypes.c_int, [vp, vp, vp, vp, vp, vp]),
        "fem_element_volumes": (ctypes.c_int, [vp, vp, i32, vp]),
        "fem_filter_setup": (ctypes.c_int, [vp, dbl]),
        "fem_filter_apply": (ctypes.c_int, [vp, i32, vp, vp, vp, vp]),
        "fem_vector_workspace_bytes": (sz, [i64]),
        "fem_dot": (ctypes.c_int, [vp, vp, i64, P(dbl), vp, sz, vp]),
        "fem_mma_default_opts": (ctypes.c_int, [P(MmaOpts)]),
        "fem_mma_update": (ctypes.c_int, [i64, i32, vp, vp, vp, vp, dbl, vp, vp, vp, vp, P(dbl), P(MmaOpts), vp, sz,
                                          vp]),
        "fem_mass_apply": (ctypes.c_int, [vp, vp, vp, vp, sz, vp]),
        "fem_set_load": (ctypes.c_int, [vp, vp, vp]),
        "fem_axpby": (ctypes.c_int, [i64, dbl, vp, dbl, vp, vp]),
        "fem_obs_misfit": (ctypes.c_int, [i64, i64, vp, vp, vp, vp, P(dbl), vp, sz, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc: int, stats=None):
    if rc != FEM_OK:
        e = FemError(rc, lib().fem_last_error().decode())
        e.stats = stats
        raise e


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    _check(lib().fem_default_opts(ctypes.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def mma_default_opts(**kw) -> MmaOpts:
    o = MmaOpts()
    _check(lib().fem_mma_default_opts(ctypes.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _vector_workspace(n: int, device) -> torch.Tensor:
    return torch.empty(max(int(lib().fem_vector_workspace_bytes(n)), 256), dtype=torch.uint8, device=device)


def dot(a: torch.Tensor, b: torch.Tensor, workspace: Optional[torch.Tensor] = None) -> float:
    """Deterministic FP64 dot product of two device vectors (fem_dot)."""
    if a.dtype != torch.float64 or b.dtype != torch.float64 or a.numel() != b.numel():
        raise ValueError("dot needs two float64 vectors of equal length")
    a, b = a.contiguous(), b.contiguous()
    ws = _vector_workspace(a.numel(), a.device) if workspace is None else workspace
    out = ctypes.c_double()
    _check(lib().fem_dot(_ptr(a), _ptr(b), a.numel(), ctypes.byref(out), _ptr(ws), ws.numel(), _stream()))
    return out.value


def mma_update(it: int, x, xold1, xold2, df0, f1: float, df1, low, upp, opts: Optional[MmaOpts] = None,
               workspace: Optional[torch.Tensor] = None):
    """One MMA iteration (fem_mma_update).  low/upp are updated in place; returns
    (xnew, lambda)."""
    n = x.numel()
    opts = mma_default_opts() if opts is None else opts
    ws = _vector_workspace(n, x.device) if workspace is None else workspace
    xnew = torch.empty_like(x)
    lam = ctypes.c_double()
    _check(lib().fem_mma_update(n, it, _ptr(x), _ptr(xold1), _ptr(xold2), _ptr(df0), float(f1), _ptr(df1),
                                _ptr(low), _ptr(upp), _ptr(xnew), ctypes.byref(lam), ctypes.byref(opts), _ptr(ws),
                                ws.numel(), _stream()))
    return xnew, lam.value


def axpby(a: float, x: torch.Tensor, b: float, y: torch.Tensor) -> torch.Tensor:
    """y = a x + b y in place on float64 device vectors (fem_axpby); returns y."""
    if x.dtype != torch.float64 or y.dtype != torch.float64 or x.numel() != y.numel():
        raise ValueError("axpby needs two float64 vectors of equal length")
    _check(lib().fem_axpby(x.numel(), float(a), _ptr(x), float(b), _ptr(y), _stream()))
    return y


def obs_misfit(u: torch.Tensor, idx: torch.Tensor, obs: torch.Tensor, dJdu: torch.Tensor,
               workspace: Optional[torch.Tensor] = None) -> float:
    """J = sum_k (u[idx_k] - obs_k)^2 and dJdu (fem_obs_misfit)."""
    ws = _vector_workspace(idx.numel(), u.device) if workspace is None else workspace
    J = ctypes.c_double()
    _check(lib().fem_obs_misfit(u.numel(), idx.numel(), _ptr(idx), _ptr(obs), _ptr(u), _ptr(dJdu), ctypes.byref(J),
                                _ptr(ws), ws.numel(), _stream()))
    return J.value


def _host(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def _keep_arrays(prob: inputs.Problem) -> dict:
    return dict(coords=_host(prob.coords, np.float64), conn=_host(prob.conn, np.int32),
                mask=_host(prob.dirichlet_mask, np.uint8), f=_host(prob.f_nodal, np.float64),
                src=_host(prob.source_nodal, np.float64), faces=_host(prob.traction_faces, np.int32),
                trac=_host(prob.traction, np.float64))


def _mesh_desc(prob: inputs.Problem, k: dict) -> MeshDesc:
    """fem_mesh_desc over the host arrays in k (which must outlive its use)."""
    def p(a):
        return None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    return MeshDesc(prob.n_nodes, prob.n_elems, prob.ndpn, prob.model, prob.pmap, 0, prob.nu, prob.bulk_ratio,
                    prob.simp_p, prob.simp_emin, prob.simp_e0, p(k["coords"]), p(k["conn"]), p(k["mask"]),
                    p(k["f"]), p(k["src"]), 0 if k["faces"] is None else k["faces"].shape[0], p(k["faces"]),
                    p(k["trac"]), float(getattr(prob, "yield_stress", 0.0)))


def pattern_host(prob: inputs.Problem):
    """(row_ptr, col_idx, f_ext) built on the host by fem_pattern_host (no GPU)."""
    k = _keep_arrays(prob)
    d = _mesh_desc(prob, k)
    n, nnz = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().fem_pattern_host(ctypes.byref(d), ctypes.byref(n), ctypes.byref(nnz), None, None, None))
    row_ptr = np.empty(n.value + 1, dtype=np.int64)
    col_idx = np.empty(max(nnz.value, 1), dtype=np.int32)
    f = np.empty(max(n.value, 1), dtype=np.float64)
    _check(lib().fem_pattern_host(ctypes.byref(d), ctypes.byref(n), ctypes.byref(nnz),
                                  row_ptr.ctypes.data_as(ctypes.c_void_p), col_idx.ctypes.data_as(ctypes.c_void_p),
                                  f.ctypes.data_as(ctypes.c_void_p)))
    return row_ptr, col_idx[:nnz.value], f[:n.value]


class Problem:
    """A mesh + material + loads bound to a libfem handle on the current GPU."""

    def __init__(self, prob: inputs.Problem, device: str = "cuda"):
        L = lib()
        self.spec = prob
        self.device = torch.device(device)
        self._keep = _keep_arrays(prob)
        d = _mesh_desc(prob, self._keep)
        h = ctypes.c_void_p()
        n, nnz = ctypes.c_int64(), ctypes.c_int64()
        with torch.cuda.device(self.device):
            _check(L.fem_build_pattern(ctypes.byref(d), ctypes.byref(h), ctypes.byref(n), ctypes.byref(nnz)))
        self.handle = h
        self.n_dofs = n.value
        self.nnz = nnz.value
        self.n_elems = prob.n_elems
        self._ws = None
        self.mask = torch.as_tensor(prob.dirichlet_mask.astype(bool), device=self.device)
        self.dirichlet_values = torch.as_tensor(prob.dirichlet_values, dtype=torch.float64, device=self.device)
        self.theta = torch.as_tensor(prob.theta, dtype=torch.float64, device=self.device)

    # ------------------------------------------------------------------ lifetime
    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().fem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ helpers
    def workspace_bytes(self, opts: Optional[SolveOpts] = None) -> int:
        b = ctypes.c_size_t()
        _check(lib().fem_workspace_bytes(self.handle, None if opts is None else ctypes.byref(opts), ctypes.byref(b)))
        return b.value

    def workspace(self, opts: Optional[SolveOpts] = None) -> torch.Tensor:
        need = self.workspace_bytes(opts)
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def _f64(self, t, n=None):
        if t is None:
            return None
        t = torch.as_tensor(t, dtype=torch.float64, device=self.device).contiguous()
        if n is not None and t.numel() != n:
            raise ValueError(f"expected {n} entries, got {t.numel()}")
        return t

    # ------------------------------------------------------------------ entry points
    def export_pattern(self, slot_map: bool = True, transpose: bool = True) -> dict:
        N, nnz = self.n_dofs, self.nnz
        nd = self.spec.ndpn
        Nd = 8 * nd
        out = dict(row_ptr=torch.empty(N + 1, dtype=torch.int64, device=self.device),
                   col_idx=torch.empty(nnz, dtype=torch.int32, device=self.device),
                   diag_slot=torch.empty(N, dtype=torch.int64, device=self.device))
        out["slot_map"] = (torch.empty(self.n_elems * Nd * Nd, dtype=torch.int32, device=self.device)
                           if slot_map else None)
        out["transpose_perm"] = torch.empty(nnz, dtype=torch.int32, device=self.device) if transpose else None
        _check(lib().fem_pattern_export(self.handle, _ptr(out["row_ptr"]), _ptr(out["col_idx"]),
                                        _ptr(out["slot_map"]), _ptr(out["diag_slot"]),
                                        _ptr(out["transpose_perm"]), _stream()))
        return out

    def load_vector(self) -> torch.Tensor:
        f = torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        _check(lib().fem_load_vector(self.handle, _ptr(f), _stream()))
        return f

    def values_count(self, layout: int = LAYOUT_CSR) -> int:
        c = ctypes.c_int64()
        _check(lib().fem_values_count(self.handle, layout, ctypes.byref(c)))
        return c.value

    def assemble(self, u, theta=None, residual: bool = True, values_dtype: Optional[torch.dtype] = torch.float64,
                 layout: int = LAYOUT_CSR, check: bool = True):
        u = self._f64(u, self.n_dofs)
        theta = self.theta if theta is None else self._f64(theta, self.n_elems)
        r = torch.empty(self.n_dofs, dtype=torch.float64, device=self.device) if residual else None
        vals = None
        dt = F64
        if values_dtype is not None:
            dt = F32 if values_dtype == torch.float32 else F64
            vals = torch.empty(self.values_count(layout), dtype=values_dtype, device=self.device)
        ws = self.workspace(None)
        _check(lib().fem_assemble(self.handle, _ptr(u), _ptr(theta), _ptr(r), _ptr(vals), dt, layout, _ptr(ws),
                                  ws.numel(), _stream()))
        if check:
            self.check()
        return r, vals

    def residual_noalloc(self, u, theta=None, out: Optional[torch.Tensor] = None, check: bool = True):
        """The FP64 residual through fem_residual_noalloc (static device scratch, no
        workspace; meshes up to the library's limit)."""
        u = self._f64(u, self.n_dofs)
        theta = self.theta if theta is None else self._f64(theta, self.n_elems)
        r = torch.empty(self.n_dofs, dtype=torch.float64, device=self.device) if out is None else out
        _check(lib().fem_residual_noalloc(self.handle, _ptr(u), _ptr(theta), _ptr(r), _stream()))
        if check:
            self.check()
        return r

    def check(self):
        """Waits for the stream and raises what the enqueue-only kernels found (fem_check)."""
        _check(lib().fem_check(self.handle, _stream()))

    def spmv(self, values: torch.Tensor, x: torch.Tensor, transpose: bool = False, alpha: float = 1.0,
             beta: float = 0.0, y: Optional[torch.Tensor] = None, layout: int = LAYOUT_CSR) -> torch.Tensor:
        dt = F32 if values.dtype == torch.float32 else F64
        if values.numel() != self.values_count(layout) or x.numel() != self.n_dofs or x.dtype != values.dtype:
            raise ValueError("spmv operand shapes/dtypes do not match the pattern")
        if y is None:
            y = torch.empty_like(x)
        _check(lib().fem_spmv(self.handle, _ptr(values), dt, layout, int(transpose), _ptr(x), _ptr(y), alpha, beta,
                              _stream()))
        return y

    def apply_tangent(self, u, v, theta=None) -> torch.Tensor:
        u = self._f64(u, self.n_dofs)
        v = self._f64(v, self.n_dofs)
        theta = self.theta if theta is None else self._f64(theta, self.n_elems)
        y = torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        ws = self.workspace(None)
        _check(lib().fem_apply_tangent(self.handle, _ptr(u), _ptr(theta), _ptr(v), _ptr(y), _ptr(ws), ws.numel(),
                                       _stream()))
        return y

    def mass_apply(self, x, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """M x for a nodal field x (fem_mass_apply)."""
        x = self._f64(x, self.n_dofs)
        y = torch.empty_like(x) if out is None else out
        ws = self.workspace(None)
        _check(lib().fem_mass_apply(self.handle, _ptr(x), _ptr(y), _ptr(ws), ws.numel(), _stream()))
        return y

    def set_load(self, f):
        """Replaces the external load vector (fem_set_load)."""
        f = self._f64(f, self.n_dofs)
        _check(lib().fem_set_load(self.handle, _ptr(f), _stream()))

    def history(self) -> torch.Tensor:
        """The J2 history [n_elems, 8, 12] (strain then stress per Gauss point; fem_history_copy)."""
        buf = torch.empty(self.n_elems * 96, dtype=torch.float64, device=self.device)
        _check(lib().fem_history_copy(self.handle, _ptr(buf), 0, _stream()))
        return buf.view(self.n_elems, 8, 12)

    def set_history(self, hist):
        """Replaces the J2 history (fem_history_copy into the handle)."""
        h = self._f64(hist, self.n_elems * 96)
        _check(lib().fem_history_copy(self.handle, _ptr(h), 1, _stream()))

    def average_stress(self):
        """Volume-averaged committed stress (xx, yy, zz, yz, xz, xy) (fem_average_stress)."""
        out = (ctypes.c_double * 6)()
        _check(lib().fem_average_stress(self.handle, out, _stream()))
        return list(out)

    def amg_setup(self):
        """Builds the two-level preconditioner's aggregates and prolongator (fem_amg_setup, once)."""
        _check(lib().fem_amg_setup(self.handle))

    def _ready(self, opts):
        if opts.precond == PRECOND_AMG:
            self.amg_setup()

    def amg_sizes(self):
        """(aggregates, coarse blocks) of the two-level preconditioner (fem_amg_sizes)."""
        self.amg_setup()
        na, nb = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().fem_amg_sizes(self.handle, ctypes.byref(na), ctypes.byref(nb)))
        return na.value, nb.value

    def amg_export(self) -> dict:
        """Aggregates, prolongator and coarse block pattern (fem_amg_export)."""
        na, nb = self.amg_sizes()
        nc = 6 if self.spec.ndpn == 3 else 1
        dev = self.device
        out = {"agg": torch.empty(self.spec.n_nodes, dtype=torch.int32, device=dev),
               "P": torch.empty(self.n_dofs * nc, dtype=torch.float64, device=dev),
               "coarse_ptr": torch.empty(na + 1, dtype=torch.int64, device=dev),
               "coarse_col": torch.empty(max(nb, 1), dtype=torch.int32, device=dev)}
        _check(lib().fem_amg_export(self.handle, _ptr(out["agg"]), _ptr(out["P"]), _ptr(out["coarse_ptr"]),
                                    _ptr(out["coarse_col"])))
        out["coarse_col"] = out["coarse_col"][:nb]
        out["n_aggregates"], out["n_coarse_blocks"], out["nc"] = na, nb, nc
        return out

    def amg_apply(self, u, r, theta=None, opts: Optional[SolveOpts] = None, **kw):
        """z = M r with the two-level preconditioner of K(u) (fem_amg_apply); returns
        (z, [lmax fine, lmax coarse], coarse operator values FP64)."""
        kw.setdefault("precond", PRECOND_AMG)
        kw.setdefault("krylov", CG)
        opts = self.opts(**kw) if opts is None else opts
        u = self._f64(u, self.n_dofs)
        r = self._f64(r, self.n_dofs)
        theta = self.theta if theta is None else self._f64(theta, self.n_elems)
        na, nb = self.amg_sizes()
        nc = 6 if self.spec.ndpn == 3 else 1
        z = torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        cv = torch.empty(max(nb * nc * nc, 1), dtype=torch.float64, device=self.device)
        lm = (ctypes.c_double * 2)()
        self._ready(opts)
        ws = self.workspace(opts)
        _check(lib().fem_amg_apply(self.handle, _ptr(u), _ptr(theta), _ptr(r), _ptr(z), ctypes.byref(opts), lm,
                                   _ptr(cv), _ptr(ws), ws.numel(), _stream()))
        return z, list(lm), cv[:nb * nc * nc]

    def param_vjp(self, u, lam, theta=None) -> torch.Tensor:
        """-lambda^T dC/dtheta per element for a given lambda (fem_param_vjp)."""
        u = self._f64(u, self.n_dofs)
        lam = self._f64(lam, self.n_dofs)
        theta = self.theta if theta is None else self._f64(theta, self.n_elems)
        g = torch.empty(self.n_elems, dtype=torch.float64, device=self.device)
        _check(lib().fem_param_vjp(self.handle, _ptr(u), _ptr(theta), _ptr(lam), _ptr(g), _stream()))
        return g

    def element_volumes(self, normalized: bool = False) -> torch.Tensor:
        """Element volumes, or with normalized=True the fractions v_e / sum_f v_f."""
        v = torch.empty(self.n_elems, dtype=torch.float64, device=self.device)
        _check(lib().fem_element_volumes(self.handle, _ptr(v), int(normalized), _stream()))
        return v

    def filter_setup(self, rmin: float):
        _check(lib().fem_filter_setup(self.handle, float(rmin)))

    def filter_apply(self, x, mode: int = FILTER_DENSITY, theta=None) -> torch.Tensor:
        x = self._f64(x, self.n_elems)
        theta = None if theta is None else self._f64(theta, self.n_elems)
        out = torch.empty_like(x)
        _check(lib().fem_filter_apply(self.handle, mode, _ptr(theta), _ptr(x), _ptr(out), _stream()))
        return out

    def opts(self, **kw) -> SolveOpts:
        kw.setdefault("krylov", self.spec.krylov)
        kw.setdefault("n_load_steps", self.spec.n_load_steps)
        return default_opts(**kw)

    def newton_solve(self, theta=None, u0=None, dirichlet_values=None, opts: Optional[SolveOpts] = None, **kw):
        opts = self.opts(**kw) if opts is None else opts
        theta = self.theta if theta is None else self._f64(theta, self.n_elems)
        u = (torch.zeros(self.n_dofs, dtype=torch.float64, device=self.device) if u0 is None
             else self._f64(u0, self.n_dofs).clone())
        g = self.dirichlet_values if dirichlet_values is None else self._f64(dirichlet_values, self.n_dofs)
        st = SolveStats()
        self._ready(opts)
        ws = self.workspace(opts)
        _check(lib().fem_newton_solve(self.handle, _ptr(u), _ptr(theta), _ptr(g), ctypes.byref(opts),
                                      ctypes.byref(st), _ptr(ws), ws.numel(), _stream()), st)
        return u, st

    def adjoint_vjp(self, u, dJdu, theta=None, opts: Optional[SolveOpts] = None, want_lambda: bool = True, **kw):
        opts = self.opts(**kw) if opts is None else opts
        theta = self.theta if theta is None else self._f64(theta, self.n_elems)
        u = self._f64(u, self.n_dofs)
        dJdu = self._f64(dJdu, self.n_dofs)
        g = torch.empty(self.n_elems, dtype=torch.float64, device=self.device)
        lam = torch.empty(self.n_dofs, dtype=torch.float64, device=self.device) if want_lambda else None
        st = SolveStats()
        self._ready(opts)
        ws = self.workspace(opts)
        _check(lib().fem_adjoint_vjp(self.handle, _ptr(u), _ptr(theta), _ptr(dJdu), _ptr(g), _ptr(lam),
                                     ctypes.byref(opts), ctypes.byref(st), _ptr(ws), ws.numel(), _stream()), st)
        return g, lam, st


class FemSolve(torch.autograd.Function):
    """u = U(theta): forward = Newton solve, backward = adjoint VJP (Sec. 3, Eq. (adjoint_chain_simp)).

    ``backward(grad_u)`` returns -lambda^T dC/dtheta with (dC/du)^T lambda = grad_u; the
    explicit dJ/dtheta term of a loss is added by torch autograd on the loss itself."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, problem: Problem, opts: Optional[SolveOpts] = None):
        u, st = problem.newton_solve(theta=theta.detach(), opts=opts)
        ctx.problem = problem
        ctx.opts = opts
        ctx.stats = st
        ctx.save_for_backward(theta.detach(), u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        theta, u = ctx.saved_tensors
        g, _, _ = ctx.problem.adjoint_vjp(u, grad_u.detach().to(torch.float64).contiguous(), theta=theta,
                                          opts=ctx.opts, want_lambda=False)
        return g.to(theta.dtype), None, None

"""Full-size checks of the HIP path on the five named workloads.

At these sizes the oracle cannot solve the systems, so the checks are
(a) bit-exact integer structures where the oracle can build them,
(b) outputs the oracle computes one by one (residual vectors, sampled rows of the
    tangent and of the SpMV, per-element VJPs, the SIMP closed form), and
(c) properties that hold at any size (the oracle's residual at the GPU solution,
    the adjoint equation on sampled rows).
Tolerances as in test_gpu_parity; the solve checks derive theirs from the stopping
tolerances passed to the solver.
"""
import os

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2212_00964_amd import inputs as gen
from parity import assert_parity

pytestmark = pytest.mark.gpu
fem = pytest.importorskip("paper_2212_00964_amd.fem")
DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def stretched_state(p, s, seed=0, noise=1e-4):
    """Affine stretch along x plus small seeded noise, with the Dirichlet values of the
    final load scaled to the same stretch."""
    u = np.zeros((p.n_nodes, 3))
    u[:, 0] = s * p.coords[:, 0]
    u = u.ravel() + noise * np.random.default_rng(seed).standard_normal(p.n_dofs)
    m = p.dirichlet_mask.astype(bool)
    u[m] = (s / 0.2) * p.dirichlet_values[m] if p.dirichlet_values[m].any() else 0.0
    return u


class RowReader:
    """Reads single CSR rows of a device matrix without copying the whole pattern."""

    def __init__(self, prob):
        out = prob.export_pattern(slot_map=False, transpose=False)
        self.row_ptr = host(out["row_ptr"])
        self.col_idx = out["col_idx"]

    def row(self, values, r):
        a, b = int(self.row_ptr[r]), int(self.row_ptr[r + 1])
        return host(self.col_idx[a:b]), host(values[a:b]).astype(np.float64)


def sampled_rows_check(p, reader, u, values, rows, tol):
    """Rows of the eliminated tangent summed element by element by the oracle."""
    ref = orc.rows_of_K(p, u, rows)
    for r in rows:
        cols_ref, v_ref = ref[int(r)]
        cols, v = reader.row(values, r)
        full = dict(zip(cols.tolist(), v.tolist()))
        assert set(cols.tolist()) >= set(cols_ref.tolist())
        got = np.array([full[int(c)] for c in cols_ref])
        scale = np.abs(v_ref).max()
        assert np.abs(got - v_ref).max() <= tol * scale, (r, np.abs(got - v_ref).max() / scale)
    return ref


# ----------------------------------------------------------------------------- workload 2: cantilever

def test_cantilever_64x32x32_pattern_assembly_and_solve():
    p = gen.workload(2)
    prob = fem.Problem(p, DEV)
    ref = orc.Pattern(p, with_transpose=True)
    out = prob.export_pattern()
    for k, r in (("row_ptr", ref.row_ptr), ("col_idx", ref.col_idx), ("slot_map", ref.slot.ravel()),
                 ("diag_slot", ref.diag_slot), ("transpose_perm", ref.tperm)):
        assert np.array_equal(host(out[k]), r), k
    del out
    F = orc.load_vector(p)
    assert_parity(host(prob.load_vector()), F, 1e-14)
    u = 1e-4 * np.random.default_rng(0).standard_normal(p.n_dofs)
    r_ref, K_ref = orc.assemble(p, ref, u, F=F)
    r, K = prob.assemble(u)
    assert_parity(host(r), r_ref, 1e-13)
    assert_parity(host(K), K_ref, 1e-13)
    del K
    for prec in (fem.PREC_FP64, fem.PREC_MIXED):
        us, st = prob.newton_solve(precision=prec, krylov=fem.CG, newton_rtol=1e-10, krylov_rtol=1e-6 if prec == 0 else 1e-3)
        res = orc.residual(p, ref, host(us), F=F)
        assert np.linalg.norm(res) <= 1e-9 * np.linalg.norm(F), (prec, st.as_dict())
    prob.close()


@pytest.fixture(scope="module")
def cantilever_ref():
    """The oracle's own solution of the 64x32x32 cantilever: Newton (one lifted step and
    refinements) with Jacobi-PCG to relative residual 1e-13, on the host's cores."""
    p = gen.workload(2)
    with orc.threads(min(16, os.cpu_count() or 1)):
        pat = orc.Pattern(p)
        u = orc.newton_solve(p, linear="cg", rtol=1e-12, krylov_rtol=1e-13, pat=pat)
    return p, u


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6)])
def test_cantilever_64x32x32_solution_matches_oracle_pcg(cantilever_ref, precision, tol):
    p, u_ref = cantilever_ref
    prob = fem.Problem(p, DEV)
    u, st = prob.newton_solve(precision=precision, krylov=fem.CG, newton_rtol=1e-12 if precision == 0 else 1e-11,
                              krylov_rtol=1e-10 if precision == 0 else 1e-3)
    assert_parity(host(u), u_ref, tol, st.as_dict())
    prob.close()


# ----------------------------------------------------------------------------- workload 3: neo-Hookean 100^3

@pytest.fixture(scope="module")
def nh3():
    p = gen.workload(3)
    prob = fem.Problem(p, DEV)
    yield p, prob
    prob.close()


def test_nh_100cube_pattern(nh3):
    p, prob = nh3
    out = prob.export_pattern(slot_map=True, transpose=True)
    row_ptr = np.zeros(p.n_dofs + 1, dtype=np.int64)
    nnz = orc.lib().orc_pattern_rows(p.n_nodes, p.n_elems, 3, np.ascontiguousarray(p.conn, np.int32), row_ptr)
    assert nnz == prob.nnz == 245_438_109
    assert np.array_equal(host(out["row_ptr"]), row_ptr)
    col_idx = np.zeros(nnz, dtype=np.int32)
    orc.lib().orc_pattern_cols(p.n_nodes, p.n_elems, 3, np.ascontiguousarray(p.conn, np.int32), row_ptr, col_idx)
    assert np.array_equal(host(out["col_idx"]), col_idx)
    # slot map on sampled elements, transpose map on sampled entries (sliced on the device)
    sel = gen.sample_elements(p.n_elems, 200, seed=3)
    slot = host(out["slot_map"].view(p.n_elems, 576)[torch.as_tensor(sel, device=DEV)]).reshape(-1, 24, 24)
    for s_, e in zip(slot, sel):
        d = orc.element_dofs(p, e)
        for a in range(24):
            seg = col_idx[row_ptr[d[a]]:row_ptr[d[a] + 1]]
            assert np.array_equal(s_[a], row_ptr[d[a]] + np.searchsorted(seg, d))
    ks = np.random.default_rng(4).integers(0, nnz, 2000)
    tperm = host(out["transpose_perm"][torch.as_tensor(ks, device=DEV)])
    rows = np.searchsorted(row_ptr, ks, side="right") - 1
    for t, k, rr in zip(tperm, ks, rows):
        c = col_idx[k]
        seg = col_idx[row_ptr[c]:row_ptr[c + 1]]
        assert t == row_ptr[c] + np.searchsorted(seg, rr)


def test_nh_100cube_residual_rows_and_spmv(nh3):
    p, prob = nh3
    u = stretched_state(p, 0.16, seed=1)
    pat = orc.Pattern(p, with_slot=False)
    F = orc.load_vector(p)
    r_ref = orc.residual(p, pat, u, F=F)
    r, K = prob.assemble(u, values_dtype=torch.float64)
    assert_parity(host(r), r_ref, 1e-13)
    rows = np.sort(np.random.default_rng(5).choice(p.n_dofs, 24, replace=False))
    reader = RowReader(prob)
    ref = sampled_rows_check(p, reader, u, K, rows, 1e-12)
    x = np.random.default_rng(6).standard_normal(p.n_dofs)
    y = host(prob.spmv(K, torch.as_tensor(x, device=DEV)))
    for rr in rows:
        cols, v = ref[int(rr)]
        assert abs(y[rr] - v @ x[cols]) <= 1e-12 * (np.abs(v) @ np.abs(x[cols]))
    del K
    _, K32 = prob.assemble(u, residual=False, values_dtype=torch.float32)
    sampled_rows_check(p, reader, u, K32, rows, 2e-6)
    x32 = torch.as_tensor(x, dtype=torch.float32, device=DEV)
    y32 = host(prob.spmv(K32, x32))
    del K32
    _, S32 = prob.assemble(u, residual=False, values_dtype=torch.float32, layout=fem.LAYOUT_SYM_BLOCK)
    ys = host(prob.spmv(S32, x32, layout=fem.LAYOUT_SYM_BLOCK))
    for rr in rows:
        cols, v = ref[int(rr)]
        assert abs(y32[rr] - v @ x[cols]) <= 2e-6 * (np.abs(v) @ np.abs(x[cols]))
        assert abs(ys[rr] - v @ x[cols]) <= 2e-6 * (np.abs(v) @ np.abs(x[cols]))


@pytest.fixture(scope="module")
def nh3_tight(nh3):
    """A tight FP64 solution of the 5-step problem (Newton rtol 1e-11, CG rtol 1e-8),
    itself checked below by the oracle's residual."""
    p, prob = nh3
    u, st = prob.newton_solve(precision=fem.PREC_FP64, krylov=fem.CG, newton_rtol=1e-11, krylov_rtol=1e-8)
    uh = host(u)
    r = orc.residual(p, orc.Pattern(p, with_slot=False), uh, F=orc.load_vector(p))
    assert np.linalg.norm(r) <= 1e-11 * st.initial_residual * 1.001 + 1e-12
    return uh


@pytest.mark.parametrize("precision,krylov", [(1, 0), (1, 1), (2, 1), (0, 1)])
def test_nh_100cube_newton_and_adjoint_properties(nh3, nh3_tight, precision, krylov):
    """Full 5-step solve (mixed Jacobi-BiCGSTAB is the workload's named form); the
    oracle's FP64 residual at the GPU solution must meet the Newton tolerance, the
    solution must agree with a tight FP64 one to 1e-6, sampled rows of the adjoint
    equation must hold, and the per-element VJP must equal the oracle's element formula
    at the GPU's state."""
    p, prob = nh3
    opts = prob.opts(precision=precision, krylov=krylov, newton_rtol=1e-9,
                     krylov_rtol=1e-3 if precision != 0 else 1e-5, adjoint_rtol=1e-8)
    u, st = prob.newton_solve(opts=opts)
    uh = host(u)
    print(f"nh 100^3 precision={precision} krylov={krylov}: newton {st.newton_its} krylov {st.krylov_its_total}",
          flush=True)
    assert_parity(uh, nh3_tight, 1e-6, st.as_dict())
    pat = orc.Pattern(p, with_slot=False)
    F = orc.load_vector(p)
    r = orc.residual(p, pat, uh, F=F)
    assert np.linalg.norm(r) <= 1e-9 * st.initial_residual * 1.001 + 1e-12, (np.linalg.norm(r), st.as_dict())
    dJdu = np.where(p.dirichlet_mask.astype(bool), 0.0, uh)
    g, lam, sa = prob.adjoint_vjp(u, torch.as_tensor(dJdu, device=DEV), opts=opts)
    lh, gh = host(lam), host(g)
    rows = np.sort(np.random.default_rng(7).choice(np.nonzero(~p.dirichlet_mask.astype(bool))[0], 24, replace=False))
    ref = orc.rows_of_K(p, uh, rows)
    Klam = np.array([ref[int(rr)][1] @ lh[ref[int(rr)][0]] for rr in rows])
    assert np.abs(Klam - dJdu[rows]).max() <= 1e-8 * np.linalg.norm(dJdu) + 1e-6 * np.abs(dJdu[rows]).max()
    sel = gen.sample_elements(p.n_elems, 64, seed=8)
    g_ref = orc.vjp_theta(p, uh, lh)  # element-by-element formula at the GPU state
    assert_parity(gh[sel], g_ref[sel], 1e-12)
    assert_parity(gh, g_ref, 1e-12)


# ----------------------------------------------------------------------------- workload 4: SIMP gradient

def test_simp_120x60x30_gradient_closed_form_and_fd():
    p = gen.workload(4)
    prob = fem.Problem(p, DEV)
    F = host(prob.load_vector())
    ft = torch.as_tensor(F, device=DEV)
    opts = prob.opts(precision=fem.PREC_FP64, krylov=fem.CG, newton_rtol=1e-11, krylov_rtol=1e-10,
                     adjoint_rtol=1e-11)
    u, _ = prob.newton_solve(opts=opts)
    g, lam, _ = prob.adjoint_vjp(u, ft, opts=opts)
    uh, gh = host(u), host(g)
    assert_parity(host(lam), uh, 1e-9)
    # closed form -E'(theta) U_e^T Khat_e U_e, element matrices from the oracle, in chunks
    unit = gen.workload(4)
    unit.pmap, unit.theta = gen.THETA_IDENTITY, np.ones(p.n_elems)
    closed = np.empty(p.n_elems)
    for c0 in range(0, p.n_elems, 20000):
        idx = np.arange(c0, min(c0 + 20000, p.n_elems))
        _, Ke = orc.elements_dense(unit, idx, uh, residual=False)
        Ue = uh[(3 * p.conn[idx][:, :, None] + np.arange(3)).reshape(len(idx), 24)]
        closed[idx] = -3 * p.theta[idx] ** 2 * (1 - 1e-3) * np.einsum("ei,eij,ej->e", Ue, Ke, Ue)
    assert_parity(gh, closed, 1e-9)
    # central differences of J(theta) = F.U(theta) on 20 elements (forward map of the
    # same library, already parity-checked against the oracle at smaller sizes)
    mixed = prob.opts(precision=fem.PREC_MIXED, krylov=fem.CG, newton_rtol=1e-11, krylov_rtol=1e-3,
                      adjoint_rtol=1e-9)
    gm, _, _ = prob.adjoint_vjp(u, ft, opts=mixed)
    assert_parity(host(gm), gh, 1e-6)
    mixed64 = prob.opts(precision=fem.PREC_MIXED_V64, krylov=fem.BICGSTAB, newton_rtol=1e-11, krylov_rtol=1e-3,
                        adjoint_rtol=1e-9)
    gm64, _, _ = prob.adjoint_vjp(u, ft, opts=mixed64)
    assert_parity(host(gm64), gh, 1e-6)
    # One element moves J by ~1e-5 J here, so J must be accurate to ~1e-13: FP64 solves
    # warm-started from the base state, h = 1e-2 theta_e and a fourth-order stencil
    # (truncation O(h^4)); criterion norm-wise over the 20 elements as specified.
    fd_opts = prob.opts(precision=fem.PREC_FP64, krylov=fem.CG, newton_rtol=1e-11, krylov_rtol=1e-11)
    sel = gen.sample_elements(p.n_elems, 20, seed=1)
    fd = np.empty(sel.size)
    for j, e in enumerate(sel):
        h = 1e-2 * p.theta[e]
        vals = {}
        for k in (-2, -1, 1, 2):
            th = p.theta.copy()
            th[e] += k * h
            ue, _ = prob.newton_solve(theta=th, u0=u, opts=fd_opts)
            vals[k] = float(ft @ ue)
        fd[j] = (-vals[2] + 8 * vals[1] - 8 * vals[-1] + vals[-2]) / (12 * h)
    assert_parity(gh[sel], fd, 1e-5, np.abs(gh[sel] - fd) / np.abs(fd))
    prob.close()


# ----------------------------------------------------------------------------- workload 5: inverse NH

def test_inverse_nh_200x100x100_forward_and_gradient_properties():
    p, theta_true = gen.nh_inverse()
    prob = fem.Problem(p, DEV)
    opts = prob.opts(precision=fem.PREC_MIXED, krylov=fem.CG, newton_rtol=1e-9, krylov_rtol=1e-3,
                     adjoint_rtol=1e-8)
    u_obs, _ = prob.newton_solve(theta=theta_true, opts=opts)
    u, st = prob.newton_solve(opts=opts)
    free = ~p.dirichlet_mask.astype(bool)
    uh, oh = host(u), host(u_obs)
    dJdu = np.where(free, uh - oh, 0.0)
    g, lam, _ = prob.adjoint_vjp(u, torch.as_tensor(dJdu, device=DEV), opts=opts)
    pat = orc.Pattern(p, with_slot=False)
    r = orc.residual(p, pat, uh, F=orc.load_vector(p))
    assert np.linalg.norm(r) <= 1e-9 * st.initial_residual * 1.001 + 1e-12
    lh, gh = host(lam), host(g)
    sel = gen.sample_elements(p.n_elems, 64, seed=9)
    g_ref = orc.vjp_theta(p, uh, lh)
    assert_parity(gh[sel], g_ref[sel], 1e-12)
    rows = np.sort(np.random.default_rng(10).choice(np.nonzero(free)[0], 16, replace=False))
    ref = orc.rows_of_K(p, uh, rows)
    Klam = np.array([ref[int(rr)][1] @ lh[ref[int(rr)][0]] for rr in rows])
    assert np.abs(Klam - dJdu[rows]).max() <= 1e-8 * np.linalg.norm(dJdu) + 1e-6 * np.abs(dJdu[rows]).max()
    prob.close()


def test_inverse_nh_200x100x100_gradient_against_patch_finite_differences():
    """Gradient of the misfit at the inverse workload's full size against central finite
    differences.  One element moves J by about 1e-7 of itself here, below what a Newton
    solve can resolve, so the differences perturb theta on 5 seeded 4x4x4 element patches
    (the sum of the adjoint gradient over a patch is the derivative along that patch's
    indicator): fourth-order stencil, relative step 1e-2, J from solves warm-started at
    the base state and driven to the FP64 residual floor through the mixed path's FP64
    refinement (the forward map already checked against the oracle at smaller sizes)."""
    p, theta_true = gen.nh_inverse()
    prob = fem.Problem(p, DEV)
    tight = dict(precision=fem.PREC_MIXED, krylov=fem.CG, krylov_rtol=1e-3)
    # each solve: to 1e-11, then a few more corrections down to the FP64 residual floor
    polish = prob.opts(n_load_steps=1, newton_fixed_its=4, **tight)
    u_obs, _ = prob.newton_solve(theta=theta_true, newton_rtol=1e-11, **tight)
    u_obs, _ = prob.newton_solve(theta=theta_true, u0=u_obs, opts=polish)
    u, st = prob.newton_solve(newton_rtol=1e-11, **tight)
    u, _ = prob.newton_solve(u0=u, opts=polish)
    free = torch.as_tensor(~p.dirichlet_mask.astype(bool), device=DEV)

    def J(uu):
        e = torch.where(free, uu - u_obs, torch.zeros_like(uu))
        return 0.5 * float(e @ e)

    dJdu = torch.where(free, u - u_obs, torch.zeros_like(u))
    g, _, _ = prob.adjoint_vjp(u, dJdu, precision=fem.PREC_FP64, krylov=fem.CG, krylov_rtol=1e-10,
                               adjoint_rtol=1e-11)
    gh = host(g)
    nx, ny, nz = p.shape
    rng = np.random.default_rng(12)
    fd, adj = [], []
    fd_opts = prob.opts(n_load_steps=1, newton_fixed_its=6, **tight)
    for _ in range(5):
        ex, ey, ez = rng.integers(8, nx - 12), rng.integers(8, ny - 12), rng.integers(8, nz - 12)
        idx = np.array([(ex + i) + nx * ((ey + j) + ny * (ez + k)) for k in range(4) for j in range(4) for i in range(4)])
        h = 1e-2 * p.theta[idx[0]]
        vals = {}
        for kk in (-2, -1, 1, 2):
            th = p.theta.copy()
            th[idx] += kk * h
            ue, _ = prob.newton_solve(theta=th, u0=u, opts=fd_opts)
            vals[kk] = J(ue)
        fd.append((-vals[2] + 8 * vals[1] - 8 * vals[-1] + vals[-2]) / (12 * h))
        adj.append(gh[idx].sum())
    fd, adj = np.array(fd), np.array(adj)
    print(f"patch FD {fd} adjoint {adj} rel {np.abs(adj - fd) / np.abs(fd)}", flush=True)
    assert_parity(adj, fd, 1e-5, np.abs(adj - fd) / np.abs(fd))
    prob.close()


def test_inverse_nh_200x100x100_two_level_on_load_step_5():
    """The two-level preconditioner on the full-size inverse block at load step 5 (from
    the state of load step 4): the fine smoother's interval must end above the top of the
    Jacobi-scaled spectrum (checked against 100 power steps of D^{-1} K on the GPU), and
    every Newton correction of the step needs at most 300 two-level CG iterations (an
    interval that missed the top made the preconditioner indefinite here: 1,238-1,482
    iterations per correction)."""
    p, _ = gen.nh_inverse()
    prob = fem.Problem(p, DEV)
    g = prob.dirichlet_values
    u4, _ = prob.newton_solve(dirichlet_values=0.8 * g, precision=fem.PREC_MIXED_V64, n_load_steps=4,
                              newton_rtol=1e-9, krylov_rtol=1e-3)
    _, K = prob.assemble(u4, residual=False)
    diag_slot = prob.export_pattern(slot_map=False, transpose=False)["diag_slot"]
    sq = torch.rsqrt(K[diag_slot])  # D^{-1/2}: D^{-1} K has the spectrum of D^{-1/2} K D^{-1/2}
    x = torch.sin(1.0 + torch.arange(p.n_dofs, dtype=torch.float64, device=DEV))
    lam = 0.0
    for _ in range(100):  # ||S x|| / ||x|| of the symmetric S never exceeds its top eigenvalue
        x = x / torch.linalg.norm(x)
        y = sq * prob.spmv(K, sq * x)
        lam = float(torch.linalg.norm(y))
        x = y
    del K
    _, lm, _ = prob.amg_apply(u4, torch.ones(p.n_dofs, dtype=torch.float64, device=DEV), precision=fem.PREC_FP64)
    assert lm[0] >= lam, (lm, lam)
    u5, st = prob.newton_solve(u0=u4, precision=fem.PREC_MIXED, krylov=fem.CG, precond=fem.PRECOND_AMG,
                               n_load_steps=1, newton_rtol=1e-9, krylov_rtol=1e-3, krylov_max_it=2000,
                               newton_max_it=12)
    its = list(st.krylov_its[:st.n_hist])
    assert max(its) <= 300, its
    prob.close()

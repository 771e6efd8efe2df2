"""Two-level aggregation preconditioner on the GPU against the oracle (through the C ABI).

Tolerances: aggregation bit-exact; prolongator 1e-13 absolute (FP64 Gram-Schmidt on
both sides); coarse operator, spectrum bounds and one application z = M r 1e-11 in
FP64 (rounding order), 1e-4 in mixed precision (FP32 through two Chebyshev chains of
up to 16 steps); solves to the bars of the other preconditioners (FP64 1e-10, mixed
1e-6); adjoint gradients 1e-8 (FP64) and 1e-5 (mixed) against the oracle adjoint.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import amg
from oracle import oracle as orc
from paper_2212_00964_amd import inputs as gen
from parity import assert_parity

pytestmark = pytest.mark.gpu

fem = pytest.importorskip("paper_2212_00964_amd.fem")
DEV = "cuda:0"


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


CASES = {
    "nh-6x5x7-distorted": gen.nh_tensile(6, 5, 7, n_load_steps=2, seed=4, distort_seed=5),
    "cantilever-9x4x5-relabelled": gen.relabel(gen.cantilever(9, 4, 5, distort_seed=3), seed=7)[0],
    "poisson-9-distorted": gen.poisson_sine(9, distort_seed=2),
}


def _state(p, amp=0.002, seed=0):
    u = amp * np.random.default_rng(seed).standard_normal(p.n_dofs)
    u[p.dirichlet_mask.astype(bool)] = 0.0
    return u


def _coarse_dense(ex, vals):
    na, nc = ex["n_aggregates"], ex["nc"]
    ptr, col = host(ex["coarse_ptr"]), host(ex["coarse_col"])
    v = np.asarray(vals).reshape(-1, nc, nc)
    A = np.zeros((na * nc, na * nc))
    for I in range(na):
        for b in range(ptr[I], ptr[I + 1]):
            J = col[b]
            A[I * nc:(I + 1) * nc, J * nc:(J + 1) * nc] = v[b]
    return A


@pytest.mark.parametrize("name", list(CASES))
def test_aggregation_and_prolongator_match_oracle(name):
    p = CASES[name]
    pat = orc.Pattern(p)
    ptr, nb = amg.node_graph(pat, p.ndpn)
    agg_ref, na_ref = amg.aggregate(ptr, nb)
    P_ref, _ = amg.prolongator(p, agg_ref, na_ref)
    prob = fem.Problem(p, DEV)
    ex = prob.amg_export()
    assert ex["n_aggregates"] == na_ref
    assert np.array_equal(host(ex["agg"]), agg_ref)
    nc = ex["nc"]
    P = host(ex["P"]).reshape(p.n_dofs, nc)
    Pd = np.zeros((p.n_dofs, nc * na_ref))
    for d in range(p.n_dofs):
        a = agg_ref[d // p.ndpn]
        Pd[d, nc * a:nc * (a + 1)] = P[d]
    np.testing.assert_allclose(Pd, P_ref.toarray(), rtol=0, atol=1e-13)
    prob.close()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_coarse_operator_bounds_and_application_match_oracle(name, precision):
    p = CASES[name]
    u = _state(p)
    pat = orc.Pattern(p)
    _, K = orc.assemble(p, pat, u)
    M = amg.TwoLevel(p, pat, pat.matrix(K))
    r = np.random.default_rng(2).standard_normal(p.n_dofs)
    r[p.dirichlet_mask.astype(bool)] = 0.0
    prob = fem.Problem(p, DEV)
    z, lm, cv = prob.amg_apply(u, r, precision=precision)
    ex = prob.amg_export()
    tol = 1e-11 if precision == 0 else 1e-4
    assert_parity(_coarse_dense(ex, host(cv)), M.Ac.toarray(), (1e-12 if precision == 0 else 1e-5))
    assert abs(lm[0] - M.lmax) <= tol * M.lmax and abs(lm[1] - M.lmax_c) <= tol * M.lmax_c
    assert_parity(host(z), M.apply(r), tol)
    prob.close()


SOLVES = {
    "nh-9x7x6-5steps": gen.nh_tensile(9, 7, 6, n_load_steps=5, seed=0, distort_seed=1),
    "cantilever-9x4x5-relabelled": CASES["cantilever-9x4x5-relabelled"],
    "poisson-9-distorted": CASES["poisson-9-distorted"],
    "nh-fan-8x4": gen.nh_fan(8, 4, n_load_steps=2, seed=6),
}


@pytest.mark.parametrize("name", list(SOLVES))
@pytest.mark.parametrize("precision", [0, 1])
def test_newton_with_two_level_preconditioner_matches_oracle(name, precision):
    p = SOLVES[name]
    u_ref = orc.newton_solve(p, linear="direct", rtol=1e-13)
    prob = fem.Problem(p, DEV)
    if precision == 0:
        u, st = prob.newton_solve(precision=0, krylov=fem.CG, precond=fem.PRECOND_AMG, newton_rtol=1e-12,
                                  krylov_rtol=1e-10)
        assert_parity(host(u), u_ref, 1e-10, st.as_dict())
    else:
        u, st = prob.newton_solve(precision=1, krylov=fem.CG, precond=fem.PRECOND_AMG, newton_rtol=1e-10,
                                  krylov_rtol=1e-5)
        assert_parity(host(u), u_ref, 1e-6, st.as_dict())
    prob.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_adjoint_with_two_level_preconditioner_matches_oracle(precision):
    p = SOLVES["nh-9x7x6-5steps"]
    u_ref = orc.newton_solve(p, linear="direct", rtol=1e-13)
    dJdu = np.random.default_rng(3).standard_normal(p.n_dofs)
    g_ref, lam_ref = orc.adjoint_vjp(p, u_ref, dJdu)
    prob = fem.Problem(p, DEV)
    g, lam, st = prob.adjoint_vjp(u_ref, dJdu, precision=precision, krylov=fem.CG, precond=fem.PRECOND_AMG,
                                  adjoint_rtol=1e-11 if precision == 0 else 1e-9,
                                  krylov_rtol=1e-8 if precision == 0 else 1e-3)
    tol = 1e-8 if precision == 0 else 1e-5
    assert_parity(host(lam), lam_ref, tol, st.as_dict())
    assert_parity(host(g), g_ref, tol)
    prob.close()


def test_two_level_needs_far_fewer_iterations_than_jacobi():
    p = gen.nh_tensile(20, 20, 20, n_load_steps=1, seed=0)
    prob = fem.Problem(p, DEV)
    o = dict(precision=1, krylov=fem.CG, newton_rtol=1e-9, krylov_rtol=1e-3)
    _, sj = prob.newton_solve(precond=fem.PRECOND_JACOBI, **o)
    _, sa = prob.newton_solve(precond=fem.PRECOND_AMG, **o)
    assert sa.krylov_its_total * 4 <= sj.krylov_its_total, (sa.krylov_its_total, sj.krylov_its_total)
    prob.close()


def test_two_level_keeps_its_advantage_on_a_late_load_step_of_an_elongated_block():
    """The inverse workload's shape (2x1x1, stretched to 1.2 in 5 load steps) at reduced
    size: the corrections of load step 5, from the state of load step 4, need at most a
    third of Jacobi-CG's iterations with the two-level preconditioner (its fine smoother
    must bound the top of the spectrum: an interval that misses it made the
    preconditioner indefinite on the full-size block)."""
    p, _ = gen.nh_inverse(40, 20, 20)
    prob = fem.Problem(p, DEV)
    g = prob.dirichlet_values
    u4, _ = prob.newton_solve(dirichlet_values=0.8 * g, precision=fem.PREC_MIXED_V64, n_load_steps=4,
                              newton_rtol=1e-9, krylov_rtol=1e-3)
    o = dict(precision=1, krylov=fem.CG, n_load_steps=1, newton_rtol=1e-9, krylov_rtol=1e-3)
    _, sj = prob.newton_solve(u0=u4, precond=fem.PRECOND_JACOBI, **o)
    _, sa = prob.newton_solve(u0=u4, precond=fem.PRECOND_AMG, **o)
    jac = list(sj.krylov_its[:sj.n_hist])
    two = list(sa.krylov_its[:sa.n_hist])
    assert sa.krylov_its_total * 3 <= sj.krylov_its_total, (two, jac)
    assert max(two) * 3 <= max(jac), (two, jac)
    prob.close()


def test_two_level_option_errors():
    p = CASES["poisson-9-distorted"]
    prob = fem.Problem(p, DEV)
    for kw in (dict(krylov=fem.BICGSTAB), dict(krylov=fem.CG, amg_smooth_degree=0),
               dict(krylov=fem.CG, amg_coarse_degree=65)):
        with pytest.raises(fem.FemError) as ei:
            prob.newton_solve(precond=fem.PRECOND_AMG, **kw)
        assert ei.value.name == "FEM_EINVAL"
    prob.close()


def test_two_level_needs_its_setup_call():
    """FEM_PRECOND_AMG through the C ABI on a handle without fem_amg_setup is refused
    (the setup is the one call that allocates the preconditioner's memory)."""
    import ctypes
    p = CASES["poisson-9-distorted"]
    prob = fem.Problem(p, DEV)
    L = fem.lib()
    na, nb = ctypes.c_int64(), ctypes.c_int64()
    assert L.fem_amg_sizes(prob.handle, ctypes.byref(na), ctypes.byref(nb)) == -1
    opts = prob.opts(krylov=fem.CG, precond=fem.PRECOND_AMG)
    u = torch.zeros(p.n_dofs, dtype=torch.float64, device=DEV)
    ws = prob.workspace(opts)
    st = fem.SolveStats()
    rc = L.fem_newton_solve(prob.handle, fem._ptr(u), fem._ptr(prob.theta), fem._ptr(prob.dirichlet_values),
                            ctypes.byref(opts), ctypes.byref(st), fem._ptr(ws), ws.numel(), fem._stream())
    assert rc == -1 and b"fem_amg_setup" in L.fem_last_error()
    assert L.fem_amg_setup(prob.handle) == 0
    assert L.fem_amg_setup(prob.handle) == 0  # once per handle
    rc = L.fem_newton_solve(prob.handle, fem._ptr(u), fem._ptr(prob.theta), fem._ptr(prob.dirichlet_values),
                            ctypes.byref(opts), ctypes.byref(st), fem._ptr(ws), ws.numel(), fem._stream())
    assert rc == 0, L.fem_last_error()
    prob.close()

"""Parity of the HIP path (through the C ABI) against the CPU FP64 oracle.

Sizes are chosen so the oracle finishes in seconds while the GPU grids still span
several blocks with ragged tails (element counts not multiples of 32, node counts
not multiples of 8).  Tolerances:
  * integer structures (CSR pattern, slot map, diagonal, transpose map): bit-exact;
  * FP64 assembly: norm-wise relative 1e-13 (rounding-order differences only);
  * FP32 tangent: norm-wise relative 2e-6 (FP32 arithmetic on O(1) geometry);
  * FP64 Newton solution: relative L2 1e-10; mixed precision after refinement: 1e-6;
  * adjoint gradients: 1e-8 (FP64) / 1e-5 (mixed) relative to the oracle adjoint,
    and 1e-5 relative to central finite differences.
"""
import numpy as np
import pytest
import torch

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


def cases_small():
    return {
        "poisson-5x4x3-distorted": gen.poisson_sine(5, distort_seed=2),
        "cantilever-7x3x5-distorted": gen.cantilever(7, 3, 5, distort_seed=3),
        "nh-5x3x7-lognormal": gen.nh_tensile(5, 3, 7, n_load_steps=2, seed=4, distort_seed=5),
        "simp-6x3x2": gen.simp_cantilever(6, 3, 2, seed=0),
        "single-element-nh": gen.nh_tensile(1, 1, 1, n_load_steps=2),
        # axis nodes with 16 elements and 51 neighbours: the general gather and the
        # SpMV's high-degree pass
        "nh-fan-8x4": gen.nh_fan(8, 4, n_load_steps=2, seed=6),
    }


CASES = cases_small()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


# ----------------------------------------------------------------------------- pattern

def _check_pattern(p):
    ref = orc.Pattern(p, with_transpose=True)
    prob = fem.Problem(p, DEV)
    assert prob.n_dofs == ref.n and prob.nnz == ref.nnz
    out = prob.export_pattern()
    assert np.array_equal(host(out["row_ptr"]), ref.row_ptr)
    assert np.array_equal(host(out["col_idx"]), ref.col_idx)
    assert np.array_equal(host(out["slot_map"]), ref.slot.ravel())
    assert np.array_equal(host(out["diag_slot"]), ref.diag_slot)
    assert np.array_equal(host(out["transpose_perm"]), ref.tperm)
    prob.close()


@pytest.mark.parametrize("name", list(CASES))
def test_pattern_bit_exact(name):
    _check_pattern(CASES[name])


def test_pattern_bit_exact_relabelled_mesh():
    q, _, _ = gen.relabel(gen.nh_tensile(4, 3, 5, n_load_steps=1), seed=11)
    _check_pattern(q)


def test_pattern_bit_exact_poisson_8cube():
    _check_pattern(gen.workload(1))


# ----------------------------------------------------------------------------- loads and assembly

@pytest.mark.parametrize("name", ["poisson-5x4x3-distorted", "cantilever-7x3x5-distorted"])
def test_load_vector(name):
    p = CASES[name]
    prob = fem.Problem(p, DEV)
    assert_parity(host(prob.load_vector()), orc.load_vector(p), 1e-14)
    prob.close()


def _state(p, seed=0, amp=0.03):
    rng = np.random.default_rng(seed)
    return amp * rng.standard_normal(p.n_dofs)


@pytest.mark.parametrize("name", list(CASES))
def test_assembly_fp64_and_fp32(name):
    p = CASES[name]
    u = _state(p)
    pat = orc.Pattern(p)
    F = orc.load_vector(p)
    r_ref, K_ref = orc.assemble(p, pat, u, F=F)
    prob = fem.Problem(p, DEV)
    r, K = prob.assemble(u)
    assert_parity(host(r), r_ref, 1e-13)
    assert_parity(host(K), K_ref, 1e-13)
    _, K32 = prob.assemble(u, residual=False, values_dtype=torch.float32)
    assert_parity(host(K32), K_ref, 2e-6)
    prob.close()


@pytest.mark.parametrize("name", ["nh-5x3x7-lognormal", "nh-fan-8x4"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("transpose", [False, True])
def test_spmv(name, dtype, transpose):
    p = CASES[name]
    u = _state(p, 1)
    pat = orc.Pattern(p)
    _, K_ref = orc.assemble(p, pat, u)
    prob = fem.Problem(p, DEV)
    _, K = prob.assemble(u, residual=False, values_dtype=dtype)
    x = np.random.default_rng(2).standard_normal(p.n_dofs)
    y0 = np.random.default_rng(3).standard_normal(p.n_dofs)
    A = pat.matrix(K_ref)
    if transpose:
        A = A.T
    expect = 0.7 * (A @ x) - 1.3 * y0
    y = torch.as_tensor(y0, dtype=dtype, device=DEV)
    prob.spmv(K, torch.as_tensor(x, dtype=dtype, device=DEV), transpose=transpose, alpha=0.7, beta=-1.3, y=y)
    tol = 1e-13 if dtype == torch.float64 else 5e-6
    assert_parity(host(y), expect, tol)
    # beta = 0 must not read y (fill it with NaN)
    y = torch.full((p.n_dofs,), float("nan"), dtype=dtype, device=DEV)
    prob.spmv(K, torch.as_tensor(x, dtype=dtype, device=DEV), transpose=transpose, y=y)
    assert_parity(host(y), A @ x, tol)
    prob.close()


def sym_to_csr(pat, sym, nd):
    """Expands the symmetric block layout (blocks (n, m), m >= n, CSR order of the node
    graph, row-major) to full CSR values using only the oracle's pattern."""
    N = pat.n
    nn = N // nd
    out = np.zeros(pat.nnz)
    k = 0
    up = {}
    for n in range(nn):
        r0 = pat.row_ptr[nd * n]
        deg = (pat.row_ptr[nd * n + 1] - r0) // nd if nd > 1 else pat.row_ptr[n + 1] - r0
        nbrs = pat.col_idx[r0:r0 + nd * deg:nd] // nd
        for m in nbrs:
            if m >= n:
                up[(n, int(m))] = sym[k * nd * nd:(k + 1) * nd * nd].reshape(nd, nd)
                k += 1
    assert k * nd * nd == sym.size
    for n in range(nn):
        for i in range(nd):
            r = nd * n + i
            for pos in range(pat.row_ptr[r], pat.row_ptr[r + 1]):
                c = pat.col_idx[pos]
                m, kk = divmod(int(c), nd)
                out[pos] = up[(n, m)][i, kk] if m >= n else up[(m, n)][kk, i]
    return out


def test_wide_numbering_takes_32bit_indices():
    """Neighbour numbers more than 32767 apart (randomly relabelled 39,270-node mesh):
    the SpMV reads 32-bit column blocks instead of 16-bit offsets.  SpMV against the
    oracle's matrix; CG and BiCGSTAB solves checked by the oracle's residual."""
    q, _, _ = gen.relabel(gen.cantilever(34, 33, 32), seed=5)
    spread = (q.conn.max(axis=1) - q.conn.min(axis=1)).max()
    assert spread > 32767
    pat = orc.Pattern(q)
    F = orc.load_vector(q)
    _, K_ref = orc.assemble(q, pat, np.zeros(q.n_dofs), F=F)
    A = pat.matrix(K_ref)
    prob = fem.Problem(q, DEV)
    x = np.random.default_rng(4).standard_normal(q.n_dofs)
    for dtype, tol in ((torch.float64, 1e-13), (torch.float32, 5e-6)):
        _, K = prob.assemble(np.zeros(q.n_dofs), residual=False, values_dtype=dtype)
        y = prob.spmv(K, torch.as_tensor(x, dtype=dtype, device=DEV))
        assert_parity(host(y), A @ x, tol)
    for kry in (fem.CG, fem.BICGSTAB):
        u, st = prob.newton_solve(precision=fem.PREC_FP64, krylov=kry, newton_rtol=1e-11, krylov_rtol=1e-11)
        r, _ = orc.assemble(q, pat, host(u), F=F, matrix=False)
        assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(F), st.as_dict()
    prob.close()


@pytest.mark.parametrize("name", ["poisson-5x4x3-distorted", "nh-5x3x7-lognormal", "cantilever-7x3x5-distorted",
                                  "nh-fan-8x4"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_symmetric_block_layout_assembly_and_spmv(name, dtype):
    p = CASES[name]
    u = _state(p, 2)
    pat = orc.Pattern(p)
    _, K_ref = orc.assemble(p, pat, u)
    prob = fem.Problem(p, DEV)
    _, Ks = prob.assemble(u, residual=False, values_dtype=dtype, layout=fem.LAYOUT_SYM_BLOCK)
    assert Ks.numel() < prob.nnz
    full = sym_to_csr(pat, host(Ks).astype(np.float64), p.ndpn)
    tol = 1e-13 if dtype == torch.float64 else 2e-6
    assert_parity(full, K_ref, tol)
    x = np.random.default_rng(8).standard_normal(p.n_dofs)
    y0 = np.random.default_rng(9).standard_normal(p.n_dofs)
    y = torch.as_tensor(y0, dtype=dtype, device=DEV)
    prob.spmv(Ks, torch.as_tensor(x, dtype=dtype, device=DEV), alpha=-0.5, beta=2.0, y=y,
              layout=fem.LAYOUT_SYM_BLOCK)
    expect = -0.5 * (pat.matrix(K_ref) @ x) + 2.0 * y0
    assert_parity(host(y), expect, (1e-13 if dtype == torch.float64 else 5e-6))
    prob.close()


@pytest.mark.parametrize("name", ["cantilever-7x3x5-distorted", "nh-5x3x7-lognormal", "poisson-5x4x3-distorted",
                                  "nh-fan-8x4"])
def test_apply_tangent_matches_assembled_operator(name):
    p = CASES[name]
    u = _state(p, 4)
    pat = orc.Pattern(p)
    _, K_ref = orc.assemble(p, pat, u)
    v = np.random.default_rng(5).standard_normal(p.n_dofs)
    prob = fem.Problem(p, DEV)
    y = prob.apply_tangent(u, v)
    assert_parity(host(y), pat.matrix(K_ref) @ v, 1e-13)
    prob.close()


# ----------------------------------------------------------------------------- solves

SOLVE_CASES = {
    "poisson-8cube": (gen.workload(1), "direct"),
    "cantilever-7x3x5": (CASES["cantilever-7x3x5-distorted"], "direct"),
    "nh-5x3x7": (CASES["nh-5x3x7-lognormal"], "direct"),
    "nh-9x7x6-5steps": (gen.nh_tensile(9, 7, 6, n_load_steps=5, seed=0, distort_seed=1), "direct"),
    "single-element": (CASES["single-element-nh"], "direct"),
    "nh-fan-8x4": (CASES["nh-fan-8x4"], "direct"),
}


@pytest.mark.parametrize("name", list(SOLVE_CASES))
def test_newton_fp64_matches_oracle(name):
    p, lin = SOLVE_CASES[name]
    u_ref = orc.newton_solve(p, linear=lin, rtol=1e-13)
    prob = fem.Problem(p, DEV)
    u, st = prob.newton_solve(precision=fem.PREC_FP64, newton_rtol=1e-13, krylov_rtol=1e-8)
    assert_parity(host(u), u_ref, 1e-10, st.as_dict())
    prob.close()


@pytest.mark.parametrize("name", list(SOLVE_CASES))
def test_newton_mixed_matches_oracle(name):
    p, lin = SOLVE_CASES[name]
    u_ref = orc.newton_solve(p, linear=lin, rtol=1e-13)
    prob = fem.Problem(p, DEV)
    u, st = prob.newton_solve(precision=fem.PREC_MIXED, newton_rtol=1e-10, krylov_rtol=1e-5)
    assert_parity(host(u), u_ref, 1e-6, st.as_dict())
    prob.close()


@pytest.mark.parametrize("name", ["nh-9x7x6-5steps", "cantilever-7x3x5", "poisson-8cube", "nh-fan-8x4"])
@pytest.mark.parametrize("krylov", [fem.CG, fem.BICGSTAB])
def test_newton_mixed_refined_corrections_match_oracle(name, krylov):
    """Mixed precision with FP64-refined corrections (FP32 Krylov sweeps restarted from
    the matrix-free FP64 residual): the oracle's solution to the mixed bar, and each
    correction's FP64 residual within the inner tolerance."""
    p, lin = SOLVE_CASES[name]
    u_ref = orc.newton_solve(p, linear=lin, rtol=1e-13)
    prob = fem.Problem(p, DEV)
    u, st = prob.newton_solve(precision=fem.PREC_MIXED, krylov=krylov, newton_rtol=1e-10, krylov_rtol=1e-3,
                              refine_rtol=0.1)
    assert_parity(host(u), u_ref, 1e-6, st.as_dict())
    assert max(st.krylov_relres[:st.n_hist]) <= 1e-3, st.as_dict()
    prob.close()


@pytest.mark.parametrize("name", list(SOLVE_CASES))
@pytest.mark.parametrize("krylov", [fem.CG, fem.BICGSTAB])
@pytest.mark.parametrize("precond", [fem.PRECOND_JACOBI, fem.PRECOND_BLOCK_JACOBI])
def test_newton_mixed_v64_matches_oracle(name, krylov, precond):
    """FP32 tangent under FP64 Krylov vectors: the oracle's solution to the mixed bar."""
    p, lin = SOLVE_CASES[name]
    u_ref = orc.newton_solve(p, linear=lin, rtol=1e-13)
    prob = fem.Problem(p, DEV)
    u, st = prob.newton_solve(precision=fem.PREC_MIXED_V64, krylov=krylov, precond=precond, newton_rtol=1e-10,
                              krylov_rtol=1e-5)
    assert_parity(host(u), u_ref, 1e-6, st.as_dict())
    prob.close()


def test_mixed_v64_refuses_the_two_level_preconditioner():
    p = CASES["nh-5x3x7-lognormal"]
    prob = fem.Problem(p, DEV)
    prob.amg_setup()
    with pytest.raises(fem.FemError) as e:
        prob.newton_solve(precision=fem.PREC_MIXED_V64, krylov=fem.CG, precond=fem.PRECOND_AMG)
    assert e.value.name == "FEM_EINVAL"
    prob.close()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_nh_homogeneous_closed_form_on_gpu(precision):
    s, G, r = 1.2, 10.0, 10.0
    p = gen.nh_roller_uniaxial(5, 4, 3, stretch=s, G=G, bulk_ratio=r, n_load_steps=4, distort_seed=8)
    # lateral stretch by bisection on P_22(diag(s, t, t)) = 0
    lo, hi = 0.5, 1.0
    for _ in range(200):
        t = 0.5 * (lo + hi)
        J = s * t * t
        c = G * J ** (-2 / 3)
        P22 = c * (t - (s * s + 2 * t * t) / (3 * t)) + r * G * J * (J - 1) / t
        lo, hi = (t, hi) if P22 < 0 else (lo, t)
    exact = p.coords * np.array([s - 1, t - 1, t - 1])
    prob = fem.Problem(p, DEV)
    u, _ = prob.newton_solve(precision=precision, newton_rtol=1e-13 if precision == 0 else 1e-11,
                             krylov_rtol=1e-8 if precision == 0 else 1e-5)
    tol = 1e-11 if precision == 0 else 1e-6
    assert np.abs(host(u).reshape(-1, 3) - exact).max() <= tol * np.abs(exact).max()
    prob.close()


@pytest.mark.parametrize("name", ["cantilever-7x3x5", "nh-9x7x6-5steps", "poisson-8cube", "nh-fan-8x4"])
@pytest.mark.parametrize("krylov", [fem.CG, fem.BICGSTAB])
@pytest.mark.parametrize("precision", [fem.PREC_FP64, fem.PREC_MIXED])
def test_newton_block_jacobi_matches_oracle(name, krylov, precision):
    """Node-block Jacobi preconditioner (3x3 inverse per node; plain Jacobi for Poisson):
    the solution is the oracle's to the same bars as with the point preconditioner."""
    p, lin = SOLVE_CASES[name]
    u_ref = orc.newton_solve(p, linear=lin, rtol=1e-13)
    prob = fem.Problem(p, DEV)
    fp64 = precision == fem.PREC_FP64
    u, st = prob.newton_solve(precision=precision, krylov=krylov, precond=fem.PRECOND_BLOCK_JACOBI,
                              newton_rtol=1e-13 if fp64 else 1e-10, krylov_rtol=1e-8 if fp64 else 1e-5)
    assert_parity(host(u), u_ref, (1e-10 if fp64 else 1e-6), st.as_dict())
    prob.close()


def test_block_jacobi_reduces_iterations_and_matches_point_jacobi():
    p = gen.nh_tensile(12, 10, 8, n_load_steps=2, seed=3, distort_seed=2)
    prob = fem.Problem(p, DEV)
    u1, s1 = prob.newton_solve(precision=fem.PREC_FP64, krylov=fem.CG, newton_rtol=1e-12, krylov_rtol=1e-6)
    u2, s2 = prob.newton_solve(precision=fem.PREC_FP64, krylov=fem.CG, newton_rtol=1e-12, krylov_rtol=1e-6,
                               precond=fem.PRECOND_BLOCK_JACOBI)
    assert_parity(host(u2), host(u1), 1e-9)
    assert s2.krylov_its_total < s1.krylov_its_total, (s1.krylov_its_total, s2.krylov_its_total)
    prob.close()


# ----------------------------------------------------------------------------- adjoint

@pytest.mark.parametrize("name", ["nh-5x3x7-lognormal", "nh-fan-8x4"])
@pytest.mark.parametrize("precision,tol", [(0, 1e-8), (1, 1e-5), (2, 1e-5)])
def test_adjoint_matches_oracle(precision, tol, name):
    p = CASES[name]
    u_ref = orc.newton_solve(p, rtol=1e-13)
    dJdu = np.random.default_rng(7).standard_normal(p.n_dofs)
    g_ref, lam_ref = orc.adjoint_vjp(p, u_ref, dJdu)
    prob = fem.Problem(p, DEV)
    g, lam, st = prob.adjoint_vjp(u_ref, dJdu, precision=precision, adjoint_rtol=1e-11 if precision == 0 else 1e-9,
                                  krylov_rtol=1e-8 if precision == 0 else 1e-5)
    assert_parity(host(lam), lam_ref, tol, st.as_dict())
    assert_parity(host(g), g_ref, tol)
    g2, lam2, st2 = prob.adjoint_vjp(u_ref, dJdu, precision=precision, precond=fem.PRECOND_BLOCK_JACOBI,
                                     adjoint_rtol=1e-11 if precision == 0 else 1e-9,
                                     krylov_rtol=1e-8 if precision == 0 else 1e-5)
    assert_parity(host(lam2), lam_ref, tol, st2.as_dict())
    assert_parity(host(g2), g_ref, tol)
    prob.close()


def test_simp_gradient_closed_form_and_fd():
    p = gen.simp_cantilever(9, 4, 3, seed=0)
    prob = fem.Problem(p, DEV)
    F = host(prob.load_vector())
    opts = prob.opts(precision=fem.PREC_FP64, newton_rtol=1e-12, krylov_rtol=1e-10, krylov=fem.CG)
    u, _ = prob.newton_solve(opts=opts)
    g, lam, _ = prob.adjoint_vjp(u, torch.as_tensor(F, device=DEV), opts=opts)
    u_h, g_h, lam_h = host(u), host(g), host(lam)
    assert_parity(lam_h, u_h, 1e-9)  # compliance is self-adjoint
    # closed form from the oracle's unit-modulus element matrices at the GPU's state
    unit = gen.simp_cantilever(9, 4, 3)
    unit.pmap, unit.theta = gen.THETA_IDENTITY, np.ones(p.n_elems)
    _, Ke = orc.elements_dense(unit, np.arange(p.n_elems), u_h, residual=False)
    closed = np.array([-3 * p.theta[e] ** 2 * (1 - 1e-3) * (u_h[orc.element_dofs(p, e)] @ Ke[e] @ u_h[orc.element_dofs(p, e)])
                       for e in range(p.n_elems)])
    assert_parity(g_h, closed, 1e-9)
    # central finite differences of J(theta) = F.U(theta), J from the oracle's solves
    def J(theta):
        return F @ orc.newton_solve(p, theta=theta, rtol=1e-12)
    for e in gen.sample_elements(p.n_elems, 20, seed=1):
        h = 1e-3 * p.theta[e]
        tp, tm = p.theta.copy(), p.theta.copy()
        tp[e] += h
        tm[e] -= h
        fd = (J(tp) - J(tm)) / (2 * h)
        assert abs(g_h[e] - fd) <= 1e-5 * abs(fd)
    prob.close()


def test_autograd_function_backward_is_adjoint():
    p = CASES["nh-5x3x7-lognormal"]
    prob = fem.Problem(p, DEV)
    opts = prob.opts(precision=fem.PREC_FP64, newton_rtol=1e-13, krylov_rtol=1e-9, adjoint_rtol=1e-11)
    theta = torch.as_tensor(p.theta, device=DEV).requires_grad_(True)
    u = fem.FemSolve.apply(theta, prob, opts)
    w = torch.as_tensor(np.random.default_rng(3).standard_normal(p.n_dofs), device=DEV)
    loss = (w * u).sum() + 0.5 * (theta ** 2).sum()
    loss.backward()
    u_ref = orc.newton_solve(p, rtol=1e-13)
    g_ref, _ = orc.adjoint_vjp(p, u_ref, w.cpu().numpy())
    assert_parity(host(theta.grad), g_ref + p.theta, 1e-8)
    prob.close()


# ----------------------------------------------------------------------------- determinism and errors

def test_bitwise_deterministic():
    p = CASES["nh-5x3x7-lognormal"]
    prob = fem.Problem(p, DEV)
    u = _state(p, 9)
    r1, K1 = prob.assemble(u)
    r2, K2 = prob.assemble(u)
    assert torch.equal(r1, r2) and torch.equal(K1, K2)
    a, _ = prob.newton_solve(precision=fem.PREC_MIXED, newton_rtol=1e-9)
    b, _ = prob.newton_solve(precision=fem.PREC_MIXED, newton_rtol=1e-9)
    assert torch.equal(a, b)
    prob.close()


def test_error_inverted_element_is_reported():
    p = gen.cantilever(3, 2, 2)
    p.coords = p.coords.copy()
    c, conn = p.coords, p.conn
    n = conn[0, 6]
    c[n] = c[conn[0, 0]] - 0.5  # pull a corner through the opposite one
    prob = fem.Problem(p, DEV)
    with pytest.raises(fem.FemError) as ei:
        prob.assemble(np.zeros(p.n_dofs))
    assert ei.value.name == "FEM_EMESH"
    prob.close()


def test_error_inverted_material_is_reported():
    p = gen.nh_tensile(2, 2, 2, n_load_steps=1)
    u = np.zeros((p.n_nodes, 3))
    u[:, 0] = -2.0 * p.coords[:, 0]  # F_xx = -1
    prob = fem.Problem(p, DEV)
    with pytest.raises(fem.FemError) as ei:
        prob.assemble(u.ravel())
    assert ei.value.name == "FEM_EINVERTED"
    prob.close()


def test_error_nan_parameter_is_reported():
    p = gen.cantilever(3, 2, 2)
    theta = p.theta.copy()
    theta[3] = np.nan
    prob = fem.Problem(p, DEV)
    with pytest.raises(fem.FemError) as ei:
        prob.assemble(np.zeros(p.n_dofs), theta=theta)
    assert ei.value.name == "FEM_ENAN"
    prob.close()


def test_error_newton_iteration_limit():
    p = gen.nh_tensile(3, 3, 3, n_load_steps=1)
    prob = fem.Problem(p, DEV)
    with pytest.raises(fem.FemError) as ei:
        prob.newton_solve(newton_max_it=1, newton_rtol=1e-14)
    assert ei.value.name == "FEM_EMAXITER"
    prob.close()


def test_error_zero_modulus_is_reported():
    p = gen.cantilever(3, 2, 2)
    prob = fem.Problem(p, DEV)
    with pytest.raises(fem.FemError) as ei:
        prob.newton_solve(theta=np.zeros(p.n_elems))
    assert ei.value.name == "FEM_ENAN"  # zero diagonal of the Jacobi preconditioner
    prob.close()


def test_error_bad_arguments():
    p = gen.cantilever(2, 2, 2)
    bad = gen.cantilever(2, 2, 2)
    bad.ndpn = 1
    with pytest.raises(fem.FemError) as ei:
        fem.Problem(bad, DEV)
    assert ei.value.name == "FEM_EINVAL"
    bad = gen.cantilever(2, 2, 2)
    bad.conn = bad.conn.copy()
    bad.conn[0, 0] = bad.n_nodes + 5
    with pytest.raises(fem.FemError) as ei:
        fem.Problem(bad, DEV)
    assert ei.value.name == "FEM_EINVAL"
    prob = fem.Problem(p, DEV)
    opts = prob.opts()
    ws = torch.empty(16, dtype=torch.uint8, device=DEV)
    u = torch.zeros(p.n_dofs, dtype=torch.float64, device=DEV)
    st = fem.SolveStats()
    import ctypes
    rc = fem.lib().fem_newton_solve(prob.handle, fem._ptr(u), fem._ptr(prob.theta), fem._ptr(prob.dirichlet_values),
                                    ctypes.byref(opts), ctypes.byref(st), fem._ptr(ws), 16, fem._stream())
    assert rc == -10  # FEM_ENOMEM: workspace too small
    opts.krylov_rtol = 2.0
    with pytest.raises(fem.FemError) as ei:
        prob.newton_solve(opts=opts)
    assert ei.value.name == "FEM_EINVAL"
    prob.close()


def test_empty_mesh_is_a_no_op():
    p = gen.Problem(name="empty", coords=np.zeros((0, 3)), conn=np.zeros((0, 8), np.int32), ndpn=3,
                    model=gen.LINEAR_ELASTIC, theta=np.zeros(0), dirichlet_mask=np.zeros(0, np.uint8),
                    dirichlet_values=np.zeros(0))
    prob = fem.Problem(p, DEV)
    assert prob.n_dofs == 0 and prob.nnz == 0
    u, st = prob.newton_solve()
    assert u.numel() == 0 and st.newton_its == 0
    prob.close()


def test_assemble_is_enqueue_only_and_check_reports_once():
    """fem_assemble returns once its kernels are enqueued; what they find is reported
    by fem_check after the stream has finished, once."""
    p = gen.cantilever(3, 2, 2)
    p.coords = p.coords.copy()
    p.coords[p.conn[0, 6]] = p.coords[p.conn[0, 0]] - 0.5
    prob = fem.Problem(p, DEV)
    prob.assemble(np.zeros(p.n_dofs), check=False)  # no error yet: nothing has been read back
    with pytest.raises(fem.FemError) as ei:
        prob.check()
    assert ei.value.name == "FEM_EMESH"
    prob.check()  # reported once
    prob.close()
    q = CASES["nh-5x3x7-lognormal"]
    prob = fem.Problem(q, DEV)
    r, K = prob.assemble(_state(q), check=False)
    prob.check()
    r2, K2 = prob.assemble(_state(q))
    assert torch.equal(r, r2) and torch.equal(K, K2)
    prob.close()


# ----------------------------------------------------------------------------- load-step recovery

def test_newton_bisects_a_load_step_that_fails():
    """One load step to stretch 1.2 needs n Newton iterations; allowed n - 1 it fails, and
    with the load-step recovery it is cut into sub-steps (each needing fewer) and
    reaches the oracle's solution."""
    p = gen.nh_tensile(4, 4, 3, n_load_steps=5, seed=1, distort_seed=2)
    u_ref = orc.newton_solve(p, rtol=1e-13)
    prob = fem.Problem(p, DEV)
    kw = dict(precision=fem.PREC_FP64, krylov=fem.CG, n_load_steps=1, newton_rtol=1e-13, krylov_rtol=1e-10)
    u_full, st_full = prob.newton_solve(**kw)
    n = st_full.newton_its
    assert n >= 3, st_full.as_dict()
    assert_parity(host(u_full), u_ref, 1e-10, st_full.as_dict())
    with pytest.raises(fem.FemError) as ei:
        prob.newton_solve(newton_max_it=n - 1, **kw)
    assert ei.value.name == "FEM_EMAXITER"
    u, st = prob.newton_solve(newton_max_it=n - 1, max_bisections=8, **kw)
    assert st.bisections >= 1, st.as_dict()
    assert_parity(host(u), u_ref, 1e-10, st.as_dict())
    prob.close()


@pytest.mark.parametrize("precision", [fem.PREC_FP64, fem.PREC_MIXED])
def test_cg_reports_non_positive_curvature(precision):
    """A negative modulus makes the tangent negative definite: CG must stop with
    FEM_EBREAKDOWN instead of returning an iterate; the recovery halves the step up to
    its limit and then reports the same error."""
    p = gen.cantilever(4, 3, 2)
    prob = fem.Problem(p, DEV)
    theta = -np.ones(p.n_elems)
    with pytest.raises(fem.FemError) as ei:
        prob.newton_solve(theta=theta, precision=precision, krylov=fem.CG)
    assert ei.value.name == "FEM_EBREAKDOWN"
    with pytest.raises(fem.FemError) as ei:
        prob.newton_solve(theta=theta, precision=precision, krylov=fem.CG, max_bisections=2)
    assert ei.value.name == "FEM_EBREAKDOWN"
    assert ei.value.stats.bisections == 2
    u, _ = prob.newton_solve(precision=precision, krylov=fem.CG)  # the handle still solves afterwards
    assert torch.isfinite(u).all()
    prob.close()

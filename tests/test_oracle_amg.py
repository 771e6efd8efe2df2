"""Pins of the two-level aggregation preconditioner oracle (CPU).

What fixes it, independently of its own code:
  * the aggregation is a partition of the nodes in which every aggregate founded in
    the first pass is exactly the closed neighbourhood of its seed, and every aggregate
    is connected in the node graph;
  * the rigid-body modes lie in the kernel of the linear-elastic stiffness without
    boundary conditions (a wrong sign or axis in a rotation fails), and the columns of
    P are orthonormal and span every aggregate's restriction of those modes;
  * the Chebyshev recurrence on a diagonal operator leaves exactly the scaled
    Chebyshev polynomial T_m((theta - lambda) / delta) / T_m(theta / delta) as the
    residual factor of every component;
  * the two-level operator M is symmetric and positive definite, and CG preconditioned
    by it reaches the direct solution in at most half the Jacobi-CG iterations;
  * the Chebyshev interval end lies between the largest eigenvalue of D^{-1} A (dense
    eigen-solve) and the Gershgorin / 1.2 x spectral-norm bounds, and equals an exact
    Gershgorin bound where the power estimate would overshoot it;
  * the coarse operator keeps the rigid-body kernel of free elasticity, is the
    Galerkin form of A between prolongated coarse vectors, and has unit rows and
    columns at dropped coarse columns.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import amg
from oracle import oracle as orc
from paper_2212_00964_amd import inputs as gen


def _problem(n=6, model="nh", distort=3):
    if model == "nh":
        return gen.nh_tensile(n, n - 1, n + 1, n_load_steps=1, seed=2, distort_seed=distort)
    return gen.poisson_sine(n, distort_seed=distort)


@pytest.mark.parametrize("model", ["nh", "poisson"])
def test_aggregation_is_a_partition_of_seed_neighbourhoods(model):
    p = _problem(model=model)
    pat = orc.Pattern(p)
    ptr, nb = amg.node_graph(pat, p.ndpn)
    agg, na = amg.aggregate(ptr, nb)
    assert agg.min() == 0 and agg.max() == na - 1 and np.all(np.bincount(agg, minlength=na) > 0)
    nbr = [set(nb[ptr[i]:ptr[i + 1]].tolist()) for i in range(ptr.size - 1)]
    for a in range(na):
        members = set(np.flatnonzero(agg == a).tolist())
        # connected in the node graph
        seen, todo = set(), [min(members)]
        while todo:
            i = todo.pop()
            if i in seen:
                continue
            seen.add(i)
            todo += [j for j in nbr[i] if j in members and j not in seen]
        assert seen == members
    # first-pass aggregates: some member's closed neighbourhood is the whole aggregate
    seeds = [a for a in range(na) if any(nbr[i] == set(np.flatnonzero(agg == a).tolist())
                                        for i in np.flatnonzero(agg == a))]
    assert len(seeds) >= 0.5 * na


def _rigid_global(p):
    c = p.coords
    B = np.zeros((p.n_dofs, 6))
    for k in range(p.n_nodes):
        B[3 * k:3 * k + 3] = amg.rigid_modes(c[k], 3)
    return B


def test_rigid_modes_span_the_kernel_of_free_elasticity():
    p = gen.cantilever(4, 3, 3, distort_seed=5)
    p.dirichlet_mask = np.zeros_like(p.dirichlet_mask)
    pat = orc.Pattern(p)
    _, K = orc.assemble(p, pat, np.zeros(p.n_dofs))
    A = pat.matrix(K)
    B = _rigid_global(p)
    assert np.abs(A @ B).max() <= 1e-9 * np.abs(A).max() * np.abs(B).max()
    # and the modes are independent
    assert np.linalg.matrix_rank(B) == 6


def test_prolongator_orthonormal_and_spanning_the_modes():
    p = _problem()
    pat = orc.Pattern(p)
    ptr, nb = amg.node_graph(pat, p.ndpn)
    agg, na = amg.aggregate(ptr, nb)
    P, dropped = amg.prolongator(p, agg, na)
    G = (P.T @ P).toarray()
    kept = np.setdiff1d(np.arange(6 * na), dropped)
    np.testing.assert_allclose(G[np.ix_(kept, kept)], np.eye(kept.size), atol=1e-12)
    assert np.abs(G[dropped]).max(initial=0.0) == 0.0
    B = _rigid_global(p)
    B[p.dirichlet_mask.astype(bool)] = 0.0
    for a in range(na):  # every aggregate's piece of the modes lies in range(P)
        dofs = (3 * np.flatnonzero(agg == a)[:, None] + np.arange(3)).ravel()
        Ba = np.zeros_like(B)
        Ba[dofs] = B[dofs]
        np.testing.assert_allclose(P @ (P.T @ Ba), Ba, atol=1e-10 * max(np.abs(Ba).max(), 1.0))


@pytest.mark.parametrize("degree", [1, 2, 3, 5, 16])
def test_chebyshev_leaves_the_scaled_chebyshev_polynomial(degree):
    lam = np.linspace(0.01, 2.0, 57)
    A = sp.diags(lam).tocsr()
    dinv = np.ones(lam.size)
    r = np.random.default_rng(1).standard_normal(lam.size)
    lmax = 2.2
    z = amg.chebyshev(A, dinv, r, lmax, degree)
    a, b = lmax / amg.CHEB_RATIO, lmax
    theta, delta = (a + b) / 2, (b - a) / 2
    t = np.polynomial.chebyshev.Chebyshev.basis(degree)
    expect = t((theta - lam) / delta) / t(theta / delta)
    np.testing.assert_allclose((r - A @ z) / r, expect, rtol=1e-10, atol=1e-12)


def _tangent(n=8):
    p = _problem(n)
    pat = orc.Pattern(p)
    u = 0.002 * np.random.default_rng(3).standard_normal(p.n_dofs)
    u[p.dirichlet_mask.astype(bool)] = 0.0
    _, K = orc.assemble(p, pat, u)
    return p, pat, pat.matrix(K).tocsr()


def test_two_level_operator_is_symmetric_positive_definite():
    p, pat, A = _tangent()
    M = amg.TwoLevel(p, pat, A)
    rng = np.random.default_rng(4)
    for _ in range(3):
        x, y = rng.standard_normal(p.n_dofs), rng.standard_normal(p.n_dofs)
        mx, my = M.apply(x), M.apply(y)
        assert abs(mx @ y - x @ my) <= 1e-10 * np.linalg.norm(mx) * np.linalg.norm(y)
        assert x @ mx > 0.0


@pytest.mark.parametrize("model", ["nh", "poisson"])
def test_two_level_cg_reaches_the_direct_solution_in_few_iterations(model):
    if model == "nh":
        p, pat, A = _tangent(10)
    else:
        p = gen.poisson_sine(16, distort_seed=2)
        pat = orc.Pattern(p)
        _, K = orc.assemble(p, pat, np.zeros(p.n_dofs))
        A = pat.matrix(K).tocsr()
    b = np.random.default_rng(5).standard_normal(p.n_dofs)
    b[p.dirichlet_mask.astype(bool)] = 0.0
    x_ref = spla.spsolve(A.tocsc(), b)
    M = amg.TwoLevel(p, pat, A)
    x, its = amg.pcg(A, b, M.apply, 1e-10)
    assert np.linalg.norm(x - x_ref) <= 1e-8 * np.linalg.norm(x_ref)
    dinv = 1.0 / A.diagonal()
    _, its_j = amg.pcg(A, b, lambda r: dinv * r, 1e-10)
    assert its * 2 <= its_j, (its, its_j)


def _small_tangent(n):
    p = gen.nh_tensile(n, n, n, n_load_steps=1, seed=2, distort_seed=3)
    pat = orc.Pattern(p)
    u = 0.002 * np.random.default_rng(3).standard_normal(p.n_dofs)
    u[p.dirichlet_mask.astype(bool)] = 0.0
    _, K = orc.assemble(p, pat, u)
    return pat.matrix(K).tocsr()


@pytest.mark.parametrize("n", [3, 4])
def test_lmax_estimate_brackets_the_top_eigenvalue(n):
    """The Chebyshev interval's upper end must lie above the largest eigenvalue of
    D^{-1} A (the eigenvalues of the symmetric D^{-1/2} A D^{-1/2}, by a dense
    eigen-solve), and below both the Gershgorin bound and 1.2 times the spectral norm
    of D^{-1} A (both computed here from the dense matrix)."""
    A = _small_tangent(n)
    dinv = 1.0 / A.diagonal()
    Ad = A.toarray()
    s = np.sqrt(dinv)
    lam_max = np.linalg.eigvalsh(Ad * s[:, None] * s[None, :]).max()
    gersh = (np.abs(Ad).sum(axis=1) * dinv).max()
    two_norm = np.linalg.norm(Ad * dinv[:, None], 2)
    lmax = amg.lmax_estimate(A, dinv)
    assert lam_max <= lmax <= min(gersh, amg.LMAX_SAFETY * two_norm) * (1 + 1e-12), (lam_max, lmax, gersh)


@pytest.mark.parametrize("n", [3, 4])
def test_fine_interval_end_is_a_bound_of_the_spectrum(n):
    """The fine smoother's interval ends at the Gershgorin bound: at or above the largest
    eigenvalue of D^{-1} A (dense eigen-solve of D^{-1/2} A D^{-1/2}) and equal to the
    largest scaled absolute row sum computed here from the dense matrix."""
    A = _small_tangent(n)
    dinv = 1.0 / A.diagonal()
    Ad = A.toarray()
    s = np.sqrt(dinv)
    lam_max = np.linalg.eigvalsh(Ad * s[:, None] * s[None, :]).max()
    gersh = (np.abs(Ad).sum(axis=1) * dinv).max()
    b = amg.gershgorin_bound(A, dinv)
    assert b == pytest.approx(gersh, rel=1e-14)
    assert lam_max <= b * (1 + 1e-12)


def test_lmax_estimate_is_capped_by_an_exact_gershgorin_bound():
    """Pairs [[1, 1], [1, 1]] scaled by different factors: D^{-1} A has eigenvalues 0 and
    2 and its Gershgorin bound is exactly 2; the power estimate reaches 2 from below, so
    1.2 times it exceeds the spectrum and the cap must bring the interval end to 2."""
    c = np.array([1.0, 3.0, 0.5, 7.0])
    blocks = [ci * np.ones((2, 2)) for ci in c]
    A = sp.block_diag(blocks).tocsr()
    dinv = 1.0 / A.diagonal()
    assert amg.lmax_estimate(A, dinv) == pytest.approx(2.0, rel=1e-14)


def _free_cantilever():
    p = gen.cantilever(4, 3, 3, distort_seed=5)
    p.dirichlet_mask = np.zeros_like(p.dirichlet_mask)
    pat = orc.Pattern(p)
    _, K = orc.assemble(p, pat, np.zeros(p.n_dofs))
    return p, pat, pat.matrix(K).tocsr()


def test_coarse_operator_keeps_the_rigid_body_kernel():
    """Without boundary conditions the rigid-body modes B span the kernel of A, and each
    aggregate's piece of B lies in range(P); so the coarse vectors c = P^T B represent
    the modes exactly (P c = B) and A_c c = P^T A B must vanish, while A_c itself is of
    the size of A.  A one-sided product (P^T A or A P) or a transposed P fails this."""
    p, pat, A = _free_cantilever()
    ptr, nb = amg.node_graph(pat, p.ndpn)
    agg, na = amg.aggregate(ptr, nb)
    P, dropped = amg.prolongator(p, agg, na)
    assert dropped.size == 0
    Ac = amg.coarse_operator(A, P, dropped)
    B = _rigid_global(p)
    C = P.T @ B
    np.testing.assert_allclose(P @ C, B, atol=1e-10 * np.abs(B).max())
    scale = abs(Ac).max() * np.abs(C).max()
    assert np.abs(Ac @ C).max() <= 1e-10 * scale
    # and A_c is symmetric positive semi-definite with exactly the 6 modes as its kernel
    Acd = Ac.toarray()
    np.testing.assert_allclose(Acd, Acd.T, atol=1e-12 * np.abs(Acd).max())
    ev = np.linalg.eigvalsh(Acd)
    assert np.sum(ev < 1e-9 * ev.max()) == 6 and ev.min() > -1e-9 * ev.max()


def test_coarse_operator_is_the_galerkin_form_with_unit_dropped_diagonal():
    """Bilinear form of A_c between random coarse vectors equals that of A between their
    prolongations (evaluated by sparse products, term by term), and every dropped
    coarse column (here the x translation of an aggregate whose x components are all
    Dirichlet dofs) has a unit row and column."""
    p = _problem(6)
    pat = orc.Pattern(p)
    ptr, nb = amg.node_graph(pat, p.ndpn)
    agg, na = amg.aggregate(ptr, nb)
    # fix the x component on every node of aggregate 0: its x translation vanishes
    p.dirichlet_mask = p.dirichlet_mask.copy()
    p.dirichlet_mask[3 * np.flatnonzero(agg == 0)] = 1
    u = 0.002 * np.random.default_rng(3).standard_normal(p.n_dofs)
    u[p.dirichlet_mask.astype(bool)] = 0.0
    _, K = orc.assemble(p, pat, u)
    A = pat.matrix(K).tocsr()
    P, dropped = amg.prolongator(p, agg, na)
    Ac = amg.coarse_operator(A, P, dropped)
    rng = np.random.default_rng(7)
    keep = np.ones(Ac.shape[0], dtype=bool)
    keep[dropped] = False
    for _ in range(4):
        c, d = rng.standard_normal(Ac.shape[0]), rng.standard_normal(Ac.shape[0])
        c[~keep] = d[~keep] = 0.0
        lhs = c @ (Ac @ d)
        rhs = (P @ c) @ (A @ (P @ d))
        assert abs(lhs - rhs) <= 1e-12 * abs(Ac).max() * np.linalg.norm(c) * np.linalg.norm(d)
    assert dropped.size > 0
    Acd = Ac.toarray()
    for j in dropped:
        e = np.zeros(Ac.shape[0])
        e[j] = 1.0
        np.testing.assert_array_equal(Acd[j], e)
        np.testing.assert_array_equal(Acd[:, j], e)

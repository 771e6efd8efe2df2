"""Pins of the oracle's SIMP optimisation pieces (CPU): filter, MMA, the loop."""
import numpy as np
import pytest

from paper_2212_00964_amd import inputs as gen
from oracle import oracle as orc
from oracle import topopt as to


def test_filter_matrix_equals_brute_force_distances():
    p = gen.simp_cantilever(6, 4, 3)
    rmin = 1.6 * (2.0 / 6)
    H = to.filter_matrix(p, rmin).toarray()
    c = p.coords[p.conn].mean(axis=1)
    D = np.linalg.norm(c[:, None, :] - c[None, :, :], axis=2)
    np.testing.assert_allclose(H, np.maximum(0.0, rmin - D), rtol=0, atol=1e-15)
    assert np.allclose(H, H.T) and (H >= 0).all()


def test_density_filter_keeps_constants_and_sensitivity_filter_identity():
    p = gen.simp_cantilever(6, 4, 3)
    H = to.filter_matrix(p, 0.5)
    np.testing.assert_allclose(to.density_filter(H, np.full(p.n_elems, 0.37)), 0.37, rtol=1e-15)
    # constant theta >= gamma and constant sensitivity: the filter returns the sensitivity
    dc = np.full(p.n_elems, -2.5)
    np.testing.assert_allclose(to.sensitivity_filter(H, np.full(p.n_elems, 0.4), dc), dc, rtol=1e-14)
    # below gamma the denominator uses gamma
    th = np.full(p.n_elems, 1e-5)
    np.testing.assert_allclose(to.sensitivity_filter(H, th, dc), dc * 1e-5 / 1e-3, rtol=1e-13)


def test_element_volumes_sum_to_box_volume():
    p = gen.simp_cantilever(6, 4, 3)
    lx, ly, lz = p.coords.max(axis=0) - p.coords.min(axis=0)
    assert abs(to.element_volumes(p).sum() - lx * ly * lz) <= 1e-13 * lx * ly * lz


def test_mma_solves_separable_convex_problem_to_its_closed_form():
    # min sum_j c_j / x_j  s.t.  mean(x) <= V  on [0, 1]: x_j = n V sqrt(c_j) / sum sqrt(c)
    rng = np.random.default_rng(3)
    n, V = 40, 0.4
    c = rng.uniform(0.5, 2.0, n)
    exact = n * V * np.sqrt(c) / np.sqrt(c).sum()
    assert exact.max() < 1.0
    x = np.full(n, V)
    xold1, xold2 = x.copy(), x.copy()
    low, upp = np.zeros(n), np.ones(n)
    for it in range(80):
        xn, low, upp, lam = to.mma_step(it, x, xold1, xold2, -c / x ** 2, x.mean() - V, np.full(n, 1.0 / n), low,
                                        upp)
        xold2, xold1, x = xold1, x, xn
    np.testing.assert_allclose(x, exact, rtol=1e-6)
    # KKT: lambda * df1 = -df0 at the optimum (lambda is the multiplier of the last subproblem)
    np.testing.assert_allclose(lam / n, c / x ** 2, rtol=1e-4)


def test_mma_first_iterations_use_initial_asymptotes_and_stay_in_move_limits():
    rng = np.random.default_rng(5)
    n = 25
    x = rng.uniform(0.2, 0.8, n)
    xn, low, upp, _ = to.mma_step(0, x, x, x, -rng.uniform(1, 2, n), 0.1, np.full(n, 1.0 / n), np.zeros(n),
                                  np.ones(n))
    np.testing.assert_allclose(low, x - 0.5)
    np.testing.assert_allclose(upp, x + 0.5)
    assert (xn >= np.maximum(0.0, low + 0.1 * (x - low)) - 1e-15).all()
    assert (xn <= np.minimum(1.0, upp - 0.1 * (upp - x)) + 1e-15).all()


def test_mma_asymptotes_contract_on_oscillation_and_widen_otherwise():
    x, x1, x2 = np.array([0.5, 0.5]), np.array([0.6, 0.4]), np.array([0.5, 0.3])
    low, upp = np.array([0.2, 0.2]), np.array([0.9, 0.9])
    lo, up = to.mma_asymptotes(3, x, x1, x2, low, upp)
    # coordinate 0 oscillates (+0.1 then -0.1): factor 0.7; coordinate 1 is monotone: 1.2
    np.testing.assert_allclose(lo, [0.5 - 0.7 * (0.6 - 0.2), 0.5 - 1.2 * (0.4 - 0.2)])
    np.testing.assert_allclose(up, [0.5 + 0.7 * (0.9 - 0.6), 0.5 + 1.2 * (0.9 - 0.4)])


def test_compliance_gradient_matches_finite_differences():
    p = gen.simp_cantilever(6, 3, 2)
    F = orc.load_vector(p)
    u = orc.newton_solve(p, rtol=1e-12)
    g = orc.vjp_theta(p, u, u)
    for e in (0, 7, 20):
        h = 1e-4
        cs = []
        for s in (1, -1):
            th = p.theta.copy()
            th[e] += s * h
            cs.append(F @ orc.newton_solve(p, theta=th, rtol=1e-12))
        fd = (cs[0] - cs[1]) / (2 * h)
        assert abs(g[e] - fd) <= 1e-6 * abs(fd), (e, g[e], fd)


def test_compliance_loop_decreases_compliance_and_keeps_the_material_fraction():
    p = gen.simp_cantilever(10, 5, 3)
    hx, hc = to.compliance_loop(p, 8, rmin=1.5 * (2.0 / 10))
    assert all(b < a for a, b in zip(hc[1:], hc[2:])), hc
    v = to.element_volumes(p)
    for x in hx[1:]:
        assert v @ x / v.sum() <= 0.5 + 1e-9
        assert x.min() >= 0.0 and x.max() <= 1.0

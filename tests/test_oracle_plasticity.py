"""Pins of the perfect-J2-plasticity oracle (Sec. 2.3, plasticity paragraph).

What fixes the oracle here, independently of its own code:
  * the return map's defining properties: returned stress on the von Mises surface
    (s_vm = sigma_y) with the deviator parallel to the trial deviator and the pressure
    unchanged; below the surface the trial stress itself, which for a zero history is
    Hooke's law;
  * the consistent tangent against central differences of the stress, in the elastic
    and the plastic regime, and the assembled tangent against differences of the
    assembled residual (with a non-trivial history);
  * homogeneous uniaxial stress on symmetry rollers (distorted mesh): the volume
    averaged sigma_zz after every load step of a loading-unloading path equals the
    one-dimensional elastic-perfectly-plastic recursion
    sigma_k = clip(sigma_{k-1} + E (eps_k - eps_{k-1}), -sigma_y, sigma_y),
    with zero lateral stress, at every Gauss point;
  * with a yield stress no path reaches, the path solution equals the linear-elastic
    oracle solution (incremental = total for a linear law).
"""
import numpy as np
import pytest

from oracle import oracle as orc
from oracle import plasticity as pl
from oracle import topopt
from paper_2212_00964_amd import inputs as gen

E, NU, SY = 70e3, 0.3, 250.0


def _lame(E=E, nu=NU):
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


def _hist(rng, eps_amp, sig_amp):
    h = np.zeros(12)
    h[:6] = eps_amp * rng.standard_normal(6)
    h[6:] = sig_amp * rng.standard_normal(6)
    return h


def _sym(v):
    return np.array([[v[0], v[5], v[4]], [v[5], v[1], v[3]], [v[4], v[3], v[2]]])


def _trial(Gu, h):
    lam, mu = _lame()
    de = 0.5 * (Gu + Gu.T) - _sym(h[:6])
    return _sym(h[6:]) + lam * np.trace(de) * np.eye(3) + 2 * mu * de


def _dev(S):
    return S - np.trace(S) / 3 * np.eye(3)


def _vm(S):
    d = _dev(S)
    return np.sqrt(1.5 * np.sum(d * d))


P = gen.j2_roller_uniaxial(2, 2, 2, yield_stress=SY)


@pytest.mark.parametrize("seed", range(6))
def test_return_map_lands_on_the_yield_surface(seed):
    rng = np.random.default_rng(seed)
    h = _hist(rng, 1e-3, 200.0)
    Gu = 5e-3 * rng.standard_normal((3, 3))
    St = _trial(Gu, h)
    assert _vm(St) > SY  # these draws are plastic
    S, y = pl.j2_stress(P, E, Gu, h)
    assert y
    assert abs(_vm(S) - SY) <= 1e-12 * SY
    np.testing.assert_allclose(np.trace(S), np.trace(St), rtol=1e-13, atol=1e-9)
    d, dt = _dev(S), _dev(St)
    np.testing.assert_allclose(d, dt * (SY / _vm(St)), rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(S, S.T, atol=0)


def test_elastic_state_is_the_trial_stress_and_hooke_for_zero_history():
    rng = np.random.default_rng(7)
    lam, mu = _lame()
    Gu = 1e-4 * rng.standard_normal((3, 3))
    S, y = pl.j2_stress(P, E, Gu, np.zeros(12))
    eps = 0.5 * (Gu + Gu.T)
    assert not y
    np.testing.assert_allclose(S, lam * np.trace(eps) * np.eye(3) + 2 * mu * eps, rtol=1e-14, atol=1e-12)
    h = _hist(rng, 1e-5, 20.0)
    S, y = pl.j2_stress(P, E, Gu, h)
    assert not y
    np.testing.assert_allclose(S, _trial(Gu, h), rtol=1e-14, atol=1e-11)


@pytest.mark.parametrize("regime", ["elastic", "plastic"])
def test_consistent_tangent_against_central_differences(regime):
    rng = np.random.default_rng(3 if regime == "elastic" else 4)
    if regime == "elastic":
        h, Gu = _hist(rng, 1e-5, 20.0), 1e-4 * rng.standard_normal((3, 3))
    else:
        h, Gu = _hist(rng, 1e-3, 200.0), 5e-3 * rng.standard_normal((3, 3))
    assert pl.j2_stress(P, E, Gu, h)[1] == (regime == "plastic")
    A = pl.j2_tangent(P, E, Gu, h)
    step = 1e-7
    for k in range(3):
        for L in range(3):
            dG = np.zeros((3, 3))
            dG[k, L] = step
            fd = (pl.j2_stress(P, E, Gu + dG, h)[0] - pl.j2_stress(P, E, Gu - dG, h)[0]) / (2 * step)
            np.testing.assert_allclose(A[:, :, k, L], fd, rtol=1e-6, atol=1e-6 * E * 1e-3)


def test_assembled_tangent_against_residual_differences():
    p = gen.j2_roller_uniaxial(2, 3, 2, distort_seed=4)
    rng = np.random.default_rng(8)
    hist = np.concatenate([_hist(rng, 1e-3, 150.0) for _ in range(p.n_elems * 8)])
    u = 2e-3 * rng.standard_normal(p.n_dofs)
    pat = orc.Pattern(p)
    _, K = pl.assemble(p, pat, u, hist, residual=False, eliminate=False)
    Kd = pat.matrix(K).toarray()
    v = rng.standard_normal(p.n_dofs)
    step = 1e-8
    rp, _ = pl.assemble(p, pat, u + step * v, hist, matrix=False, eliminate=False)
    rm, _ = pl.assemble(p, pat, u - step * v, hist, matrix=False, eliminate=False)
    fd = (rp - rm) / (2 * step)
    assert np.linalg.norm(Kd @ v - fd) <= 1e-6 * np.linalg.norm(fd)
    np.testing.assert_allclose(Kd, Kd.T, rtol=0, atol=1e-9 * np.abs(Kd).max())  # major symmetry


def _uniaxial_path(n_steps):
    strains = [0.01 * k / n_steps for k in range(1, n_steps + 1)]
    strains += [0.01 - 0.01 * k / n_steps for k in range(1, n_steps + 1)]
    out, s, e0 = [], 0.0, 0.0
    for e in strains:
        s = min(max(s + E * (e - e0), -SY), SY)
        e0 = e
        out.append(s)
    return np.array(out)


def test_uniaxial_loading_unloading_matches_closed_form():
    p = gen.j2_roller_uniaxial(3, 2, 2, strain=0.01, n_load_steps=5, distort_seed=3)
    u, hist, rec = pl.solve_path(p, [p.dirichlet_values, np.zeros(p.n_dofs)], 5)
    expect = _uniaxial_path(5)
    # the path must cross both yield limits for the pin to mean anything
    assert expect.max() == SY and expect.min() == -SY and np.any(np.abs(expect) < SY)
    for (_, avg), s in zip(rec, expect):
        assert abs(avg[2] - s) <= 1e-9 * SY
        assert np.abs(avg[[0, 1, 3, 4, 5]]).max() <= 1e-9 * SY
    H = hist.reshape(p.n_elems, 8, 12)
    assert np.abs(H[:, :, 8] - expect[-1]).max() <= 1e-9 * SY
    assert np.abs(H[:, :, 2].mean() - 0.0) <= 1e-12  # eps_zz back to zero at the end


def test_unreachable_yield_reduces_to_linear_elasticity():
    p = gen.j2_cylinder(3, 4, yield_stress=1e12, disp=0.05, n_load_steps=3)
    u, _, _ = pl.solve_path(p, [p.dirichlet_values], 3)
    q = gen.j2_cylinder(3, 4, disp=0.05)
    q.model, q.n_load_steps = gen.LINEAR_ELASTIC, 1
    u_lin = orc.newton_solve(q, rtol=1e-13)
    assert np.linalg.norm(u - u_lin) <= 1e-10 * np.linalg.norm(u_lin)


def test_cylinder_mesh_is_valid_and_on_the_disk():
    coords, conn = gen.cylinder_mesh(6, 4, R=5.0, H=10.0)
    r = np.hypot(coords[:, 0], coords[:, 1])
    assert r.max() <= 5.0 + 1e-12
    on_rim = np.isclose(r, 5.0)
    assert on_rim.sum() == 4 * 6 * 5  # the square's boundary nodes, every layer
    v = topopt.element_volumes(gen.j2_cylinder(6, 4))  # raises if det J <= 0 at a Gauss point
    assert np.all(v > 0)
    # straight element edges on the rim: the volume falls short of pi R^2 H by the chord segments only
    assert 0.95 * np.pi * 250.0 <= v.sum() < np.pi * 250.0

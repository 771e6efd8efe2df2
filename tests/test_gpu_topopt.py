"""SIMP compliance optimisation on the GPU against the oracle (through the C ABI)."""
import numpy as np
import pytest
import torch

from paper_2212_00964_amd import fem
from paper_2212_00964_amd import inputs as gen
from paper_2212_00964_amd.topopt import SimpCompliance
from oracle import oracle as orc
from oracle import topopt as to
from parity import assert_parity

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


@pytest.mark.parametrize("name", ["simp-8x4x3-distorted", "nh-fan-8x4", "nh-relabelled"])
def test_param_vjp_matches_oracle(name):
    p = {"simp-8x4x3-distorted": lambda: gen.simp_cantilever(8, 4, 3, distort_seed=6),
         "nh-fan-8x4": lambda: gen.nh_fan(8, 4, n_load_steps=2, seed=6),
         "nh-relabelled": lambda: gen.relabel(gen.nh_tensile(5, 4, 3, n_load_steps=2, seed=1, distort_seed=2),
                                              seed=3)[0]}[name]()
    u = orc.newton_solve(p, rtol=1e-12)
    lam = np.random.default_rng(1).standard_normal(p.n_dofs)
    prob = fem.Problem(p, DEV)
    g = host(prob.param_vjp(u, lam))
    assert_parity(g, orc.vjp_theta(p, u, lam), 1e-12)
    prob.close()


@pytest.mark.parametrize("normalized", [False, True])
def test_element_volumes_match_oracle(normalized):
    p = gen.nh_tensile(5, 4, 3, seed=2, distort_seed=3)
    prob = fem.Problem(p, DEV)
    v_ref = to.element_volumes(p)
    if normalized:
        v_ref = v_ref / v_ref.sum()
    np.testing.assert_allclose(host(prob.element_volumes(normalized)), v_ref, rtol=1e-13)
    prob.close()


@pytest.mark.parametrize("rmin", [0.2, 0.45])
def test_filters_match_oracle(rmin):
    p = gen.relabel(gen.nh_tensile(7, 5, 4, seed=2, distort_seed=3), seed=4)[0]
    rng = np.random.default_rng(2)
    theta = rng.uniform(0.0, 1.0, p.n_elems)
    theta[:5] = 1e-6  # below the filter's floor
    x = rng.standard_normal(p.n_elems)
    H = to.filter_matrix(p, rmin)
    prob = fem.Problem(p, DEV)
    prob.filter_setup(rmin)
    d = host(prob.filter_apply(x, fem.FILTER_DENSITY))
    s = host(prob.filter_apply(x, fem.FILTER_SENSITIVITY, theta=theta))
    assert_parity(d, to.density_filter(H, x), 1e-13)
    assert_parity(s, to.sensitivity_filter(H, theta, x), 1e-13)
    prob.close()


def test_dot_matches_numpy():
    rng = np.random.default_rng(4)
    for n in (1, 255, 257, 100003):
        a, b = rng.standard_normal(n), rng.standard_normal(n)
        got = fem.dot(torch.as_tensor(a, device=DEV), torch.as_tensor(b, device=DEV))
        assert abs(got - a @ b) <= 1e-13 * np.abs(a * b).sum()


@pytest.mark.parametrize("it,target", [(0, 0.4), (1, 0.45), (2, 0.48), (5, 0.49), (3, 0.3)])
def test_mma_update_matches_oracle(it, target):
    """Steps at several iteration counts; target 0.3 at iteration 3 cannot be reached
    inside the move limits (the step takes the limit multiplier on both sides)."""
    rng = np.random.default_rng(10 + it)
    n = 3001
    x = rng.uniform(0.05, 0.95, n)
    xold1 = np.clip(x + rng.uniform(-0.05, 0.05, n), 0, 1)
    xold2 = np.clip(xold1 + rng.uniform(-0.05, 0.05, n), 0, 1)
    low = x - rng.uniform(0.1, 0.6, n)
    upp = x + rng.uniform(0.1, 0.6, n)
    df0 = -rng.uniform(0.1, 3.0, n)
    df0[::7] *= -0.01  # some positive entries
    df1 = rng.uniform(0.5, 1.5, n) / n
    f1 = float(df1 @ x) - target
    xr, lr, ur, lam_r = to.mma_step(it, x, xold1, xold2, df0, f1, df1, low.copy(), upp.copy())
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=DEV)
    lo_d, up_d = T(low), T(upp)
    xn, lam = fem.mma_update(it, T(x), T(xold1), T(xold2), T(df0), f1, T(df1), lo_d, up_d)
    np.testing.assert_allclose(host(lo_d), lr, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(host(up_d), ur, rtol=1e-14, atol=1e-15)
    assert np.isfinite(lam_r) and abs(lam - lam_r) <= 1e-9 * max(abs(lam_r), 1e-300)
    assert np.abs(host(xn) - xr).max() <= 1e-10


def test_compliance_loop_matches_oracle():
    p = gen.simp_cantilever(12, 6, 3)
    rmin = 1.5 * (2.0 / 12)
    n_iter = 6
    hx, hc = to.compliance_loop(p, n_iter, rmin=rmin)
    prob = fem.Problem(p, DEV)
    opt = SimpCompliance(prob, rmin=rmin, vfrac=0.5)
    opt.run(n_iter)
    np.testing.assert_allclose(opt.compliance, hc, rtol=1e-9)
    assert_parity(host(opt.x), hx[-1], 1e-8)
    prob.close()


def test_filter_errors():
    p = gen.simp_cantilever(4, 2, 2)
    prob = fem.Problem(p, DEV)
    x = torch.zeros(p.n_elems, dtype=torch.float64, device=DEV)
    with pytest.raises(fem.FemError) as ei:
        prob.filter_apply(x)
    assert ei.value.name == "FEM_EINVAL"
    with pytest.raises(fem.FemError):
        prob.filter_setup(0.0)
    prob.close()

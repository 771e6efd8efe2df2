"""Full-field inference on the GPU against the oracle (through the C ABI)."""
import numpy as np
import pytest
import torch

from paper_2212_00964_amd import fem
from paper_2212_00964_amd import inputs as gen
from paper_2212_00964_amd.inference import SourceInference, lbfgs
from oracle import inference as inf
from oracle import oracle as orc
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


@pytest.mark.parametrize("case", ["poisson", "elastic"])
def test_mass_apply_matches_oracle(case):
    if case == "poisson":
        p, _ = gen.poisson_inference(6, 5, 4, distort_seed=2)
    else:
        p = gen.relabel(gen.cantilever(5, 3, 4, distort_seed=1), seed=2)[0]
    x = np.random.default_rng(5).standard_normal(p.n_dofs)
    prob = fem.Problem(p, DEV)
    assert_parity(host(prob.mass_apply(x)), inf.mass_apply(p, x), 1e-13)
    prob.close()


def test_axpby_and_misfit():
    rng = np.random.default_rng(6)
    n = 1001
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    X, Yt = torch.as_tensor(x, device=DEV), torch.as_tensor(y, device=DEV)
    fem.axpby(0.5, X, -2.0, Yt)
    np.testing.assert_allclose(host(Yt), 0.5 * x - 2.0 * y, rtol=1e-15, atol=1e-15)
    idx = np.sort(rng.choice(n, 77, replace=False))
    obs = rng.standard_normal(77)
    dJ = torch.empty(n, dtype=torch.float64, device=DEV)
    J = fem.obs_misfit(X, torch.as_tensor(idx, device=DEV), torch.as_tensor(obs, device=DEV), dJ)
    r = x[idx] - obs
    assert abs(J - r @ r) <= 1e-13 * (r @ r)
    ref = np.zeros(n)
    ref[idx] = 2 * r
    np.testing.assert_allclose(host(dJ), ref, rtol=1e-15, atol=0)


def _problem(nx=10, ny=10, nz=3, n_obs=40):
    p, obs = gen.poisson_inference(nx, ny, nz, n_obs=n_obs)
    fwd = inf.Inference(p, obs, np.zeros(obs.size))
    u_true = fwd.solve(p.source_nodal)
    return p, obs, u_true


def test_forward_value_and_gradient_match_oracle():
    p, obs, u_true = _problem()
    fun_o = inf.Inference(p, obs, u_true[obs])
    theta = np.random.default_rng(2).uniform(0.0, 4.0, p.n_nodes)
    J_o, g_o = fun_o.value_and_grad(theta)
    prob = fem.Problem(p, DEV)
    fun = SourceInference(prob, obs, u_true[obs])
    T = torch.as_tensor(theta, device=DEV)
    u = fun.solve(T)
    assert_parity(host(u), fun_o.solve(theta), 1e-10)
    J, g = fun.value_and_grad(T)
    assert abs(J - J_o) <= 1e-9 * J_o
    assert_parity(host(g), g_o, 1e-9)
    prob.close()


def test_lbfgs_iterations_match_oracle():
    p, obs, u_true = _problem()
    hx_o, hJ_o = inf.lbfgs(inf.Inference(p, obs, u_true[obs]), np.zeros(p.n_nodes), 6)
    prob = fem.Problem(p, DEV)
    fun = SourceInference(prob, obs, u_true[obs])
    hx, hJ = lbfgs(fun, torch.zeros(p.n_nodes, dtype=torch.float64, device=DEV), 6)
    np.testing.assert_allclose(hJ, hJ_o, rtol=1e-6)
    for a, b in zip(hx, hx_o):
        assert_parity(host(a), b, 1e-6)
    prob.close()


def test_gradient_taylor_rates_on_gpu():
    p, obs, u_true = _problem()
    prob = fem.Problem(p, DEV)
    fun = SourceInference(prob, obs, u_true[obs])
    rng = np.random.default_rng(3)
    theta = torch.as_tensor(rng.uniform(0.0, 5.0, p.n_nodes), device=DEV)
    d = torch.as_tensor(rng.standard_normal(p.n_nodes), device=DEV)
    J0, g = fun.value_and_grad(theta)
    gd = fem.dot(g, d)
    r0, r1 = [], []
    for h in (1e-1, 1e-2, 1e-3):
        th = fem.axpby(h, d, 1.0, theta.clone())
        Jh = fun.value(th)
        r0.append(abs(Jh - J0))
        r1.append(abs(Jh - J0 - h * gd))
    rate0 = np.log10(np.array(r0[:-1]) / np.array(r0[1:]))
    rate1 = np.log10(np.array(r1[:-1]) / np.array(r1[1:]))
    assert np.all(np.abs(rate0 - 1.0) < 0.05), rate0
    assert np.all(np.abs(rate1 - 2.0) < 0.1), rate1
    prob.close()

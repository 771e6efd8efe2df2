"""The host half of the pattern build (fem_pattern_host, no GPU) against the oracle:
the CSR pattern bit for bit and the external load vector to rounding, on meshes with
distorted, relabelled and high-degree (fan prism) connectivity, plus its refusals.
These run on the CPU, so the sanitizer build of the library covers the host graph
builder with them."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2212_00964_amd import inputs as gen
from parity import assert_parity

fem = pytest.importorskip("paper_2212_00964_amd.fem")


def _lib_or_skip():
    if not fem.library_path().exists():
        pytest.skip("libfem.so not built")


CASES = {
    "poisson-5-distorted": lambda: gen.poisson_sine(5, distort_seed=2),
    "cantilever-7x3x5-distorted": lambda: gen.cantilever(7, 3, 5, distort_seed=3),
    "nh-5x3x7": lambda: gen.nh_tensile(5, 3, 7, n_load_steps=2, seed=4, distort_seed=5),
    "nh-fan-8x4": lambda: gen.nh_fan(8, 4, n_load_steps=2, seed=6),
    "nh-relabelled": lambda: gen.relabel(gen.nh_tensile(4, 3, 5, n_load_steps=1), seed=11)[0],
    "single-element": lambda: gen.nh_tensile(1, 1, 1, n_load_steps=1),
    "poisson-8cube": lambda: gen.workload(1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_host_pattern_and_load_match_oracle(name):
    _lib_or_skip()
    p = CASES[name]()
    row_ptr, col_idx, f = fem.pattern_host(p)
    ref = orc.Pattern(p, with_slot=False)
    assert np.array_equal(row_ptr, ref.row_ptr)
    assert np.array_equal(col_idx, ref.col_idx)
    F = orc.load_vector(p)
    if np.abs(F).max() > 0:
        assert_parity(f, F, 1e-14)
    else:
        assert np.abs(f).max() == 0.0


def test_host_pattern_refusals():
    _lib_or_skip()
    p = gen.cantilever(2, 2, 2)
    p.conn = p.conn.copy()
    p.conn[1, 3] = p.conn[1, 0]
    with pytest.raises(fem.FemError) as ei:
        fem.pattern_host(p)
    assert ei.value.name == "FEM_EINVAL" and b"twice" in fem.lib().fem_last_error()
    q = gen.cantilever(2, 2, 2)
    q.conn = q.conn.copy()
    q.conn[0, 0] = q.n_nodes
    with pytest.raises(fem.FemError) as ei:
        fem.pattern_host(q)
    assert ei.value.name == "FEM_EINVAL"

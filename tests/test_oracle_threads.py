"""The oracle's opt-in threaded loops (used to time it on all host cores and to finish
large reference solves) agree with its sequential form, which the parity tests use."""
import numpy as np

from oracle import oracle as orc
from paper_2212_00964_amd import inputs as gen


def _colouring_is_proper(p):
    ptr, elems = orc.element_colours(p)
    assert np.array_equal(np.sort(elems), np.arange(p.n_elems))  # every element exactly once
    for c in range(len(ptr) - 1):
        members = elems[ptr[c]:ptr[c + 1]]
        assert np.all(np.diff(members) > 0)  # ascending within a colour
        nodes = p.conn[members].ravel()
        assert np.unique(nodes).size == nodes.size  # no node shared inside a colour
    return len(ptr) - 1


def test_element_colouring_structured_and_fan():
    assert _colouring_is_proper(gen.nh_tensile(7, 5, 4, n_load_steps=1)) == 8
    q, _, _ = gen.relabel(gen.cantilever(6, 4, 3), seed=2)
    _colouring_is_proper(q)
    assert _colouring_is_proper(gen.nh_fan(8, 4, n_load_steps=1, seed=6)) >= 16  # 16 elements at an axis node


def test_threaded_assembly_matches_sequential():
    p = gen.nh_tensile(9, 7, 6, n_load_steps=1, seed=1, distort_seed=2)
    pat = orc.Pattern(p)
    u = 0.003 * np.random.default_rng(0).standard_normal(p.n_dofs)
    F = orc.load_vector(p)
    r1, K1 = orc.assemble(p, pat, u, F=F)
    with orc.threads(4):
        r2, K2 = orc.assemble(p, pat, u, F=F)
    assert orc.lib().orc_get_threads() == 1  # restored after the block
    # colour order instead of element order: the same sums up to rounding
    assert np.abs(r2 - r1).max() <= 1e-14 * np.abs(r1).max()
    assert np.abs(K2 - K1).max() <= 1e-14 * np.abs(K1).max()


def test_threaded_krylov_and_vjp_match_sequential():
    p = gen.cantilever(8, 4, 4, distort_seed=3)
    pat = orc.Pattern(p)
    F = orc.load_vector(p)
    _, K = orc.assemble(p, pat, np.zeros(p.n_dofs), F=F)
    x1, _, _ = orc.krylov(pat, K, F, "cg", rtol=1e-12)
    xb1, _, _ = orc.krylov(pat, K, F, "bicgstab", rtol=1e-12)
    with orc.threads(4):
        x2, _, _ = orc.krylov(pat, K, F, "cg", rtol=1e-12)
        xb2, _, _ = orc.krylov(pat, K, F, "bicgstab", rtol=1e-12)
        g2 = orc.vjp_theta(p, x1, x1)
        y2 = orc.spmv(pat, K, x1)
    g1 = orc.vjp_theta(p, x1, x1)
    assert np.array_equal(g1, g2)  # independent per element: bit-identical
    assert np.array_equal(y2, orc.spmv(pat, K, x1))  # rows independent: bit-identical
    direct = orc.linear_solve(pat, K, F, "direct")
    for x in (x1, x2, xb1, xb2):
        assert np.linalg.norm(x - direct) <= 1e-9 * np.linalg.norm(direct)

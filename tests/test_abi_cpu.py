"""CPU checks of the C-ABI library: it loads, exports every function the header
declares, and the binding refuses to run without it.  No compute calls (no GPU here)."""
import ctypes
import pathlib
import re

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "fem.h"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^[A-Za-z_][\w\s\*]*?\b(fem_\w+)\s*\(", text, flags=re.M)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fem_build_pattern", "fem_assemble", "fem_spmv", "fem_newton_solve", "fem_adjoint_vjp"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2212_00964_amd import fem
    path = fem.library_path()
    if not path.exists():
        pytest.skip("libfem.so not built (run __graft_entry__.build())")
    L = ctypes.CDLL(str(path))
    names = declared_functions()
    assert sorted(names) == sorted(fem.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_host_only_entry_points():
    from paper_2212_00964_amd import fem
    if not fem.library_path().exists():
        pytest.skip("libfem.so not built")
    o = fem.default_opts()
    assert o.precision == fem.PREC_FP64 and o.krylov == fem.BICGSTAB and o.newton_max_it == 30
    assert fem.lib().fem_last_error() == b""
    assert fem.lib().fem_default_opts(None) == -1
    assert b"NULL" in fem.lib().fem_last_error()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2212_00964_amd import fem
    monkeypatch.setattr(fem, "_LIB_PATH", tmp_path / "missing.so")
    monkeypatch.setattr(fem, "_lib", None)
    with pytest.raises(fem.FemLibraryMissing):
        fem.lib()


def test_product_path_never_touches_the_oracle():
    pkg = ROOT / "paper_2212_00964_amd"
    for f in list(pkg.rglob("*.py")) + list(pkg.rglob("*.hip")) + list(pkg.rglob("*.cpp")) + list(pkg.rglob("*.h")):
        text = f.read_text()
        assert "import oracle" not in text and "from oracle" not in text and "liboracle" not in text, f


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; asking for more exits with status 2 and says why
    (before touching torch or the GPU)."""
    import subprocess
    import sys

    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_build_pattern_refuses_a_collapsed_element():
    """An element that lists a node twice is refused with FEM_EINVAL before any device
    work (the mesh checks run on the host first)."""
    import ctypes

    import numpy as np

    from paper_2212_00964_amd import fem
    if not fem.library_path().exists():
        pytest.skip("libfem.so not built")
    coords = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [1, 1, 1]], dtype=np.float64)
    conn = np.array([[0, 1, 2, 3, 4, 5, 6, 6]], dtype=np.int32)
    vp = ctypes.c_void_p
    d = fem.MeshDesc(7, 1, 3, 2, 0, 0, 0.3, 10.0, 3.0, 1e-3, 1.0, coords.ctypes.data_as(vp), conn.ctypes.data_as(vp),
                     None, None, None, 0, None, None, 0.0)
    h, n, nnz = vp(), ctypes.c_int64(), ctypes.c_int64()
    rc = fem.lib().fem_build_pattern(ctypes.byref(d), ctypes.byref(h), ctypes.byref(n), ctypes.byref(nnz))
    assert rc == -1 and not h.value
    assert b"lists a node twice" in fem.lib().fem_last_error()


def test_roofline_byte_counts_of_the_benchmark():
    """The algorithmic bytes the benchmark divides by: the 100^3 node-block SpMV
    (245,438,109 values, 27,270,901 blocks of 3x3, 1,030,301 nodes, 3,090,903 dofs) with
    FP32 values and FP32 or FP64 vectors and in FP64, counted by hand from those sizes,
    and the minimum assembly bytes."""
    import sys
    from types import SimpleNamespace

    sys.path.insert(0, str(ROOT))
    import bench

    nn, ne, n, nnz = 101 ** 3, 100 ** 3, 3 * 101 ** 3, (3 * 101 - 2) ** 3 * 9  # prod(3 n_i - 2) blocks
    assert nnz == 245_438_109
    prob = SimpleNamespace(nnz=nnz, n_dofs=n, spec=SimpleNamespace(ndpn=3, n_nodes=nn, n_elems=ne))
    blocks = nnz // 9
    assert bench.spmv_bytes(prob, 4) == nnz * 4 + blocks * 4 + (nn + 1) * 8 + 3 * n * 4 == 1_136_169_292
    assert bench.spmv_bytes(prob, 4, 8) == 1_173_260_128
    assert bench.spmv_bytes(prob, 8) == 2_155_012_564
    assert bench.assembly_bytes(prob, 4) == nnz * 4 + n * 8 + ne * 8 + nn * 24 + ne * 32 == 1_071_206_884

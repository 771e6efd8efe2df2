"""Host-side AddressSanitizer + UndefinedBehaviorSanitizer builds, and the CPU test tier
run under them.

Builds libfem.so with the sanitizers on its host code only (the device code of the
HIP kernels is compiled as usual) and the C oracle with the same clang, then runs
``pytest -m "not gpu"`` with the ASan runtime preloaded and both sanitized libraries
selected through FEM_LIBRARY / ORACLE_LIB.  On a machine without a GPU this covers the
host graph and load-vector builders (fem_pattern_host), the ABI argument checks and the
whole oracle.  Usage: python tests/sanitize_cpu.py
"""
import glob
import os
import pathlib
import subprocess
import sys

ROOT = pathlib.Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))
OUT = ROOT / "_build" / "sanitized"
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("clang's shared ASan runtime was not found")
    return hits[-1]


def build_fem() -> pathlib.Path:
    from paper_2212_00964_amd import build as B
    obj = OUT / "obj"
    obj.mkdir(parents=True, exist_ok=True)
    objs = []
    for src in B.SOURCES:
        o = obj / (src + ".o")
        subprocess.run([B.HIPCC] + B.COMMON + ["-O1", "-g"] + SAN + ["-c", str(B.SRC / src), "-o", str(o)],
                       check=True)
        objs.append(str(o))
    lib = OUT / "libfem.so"
    subprocess.run([B.HIPCC, "-shared", "-fPIC", f"--offload-arch={B.ARCH}", "-shared-libasan"] + SAN
                   + ["-o", str(lib)] + objs, check=True)
    return lib


def build_oracle() -> pathlib.Path:
    lib = OUT / "liboracle.so"
    subprocess.run([CLANG, "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-shared-libasan",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    "-o", str(lib), str(ROOT / "oracle" / "oracle.c"), "-lm"], check=True)
    return lib


def main() -> int:
    OUT.mkdir(parents=True, exist_ok=True)
    fem_lib, orc_lib = build_fem(), build_oracle()
    env = dict(os.environ)
    env.update({"LD_PRELOAD": asan_runtime(), "FEM_LIBRARY": str(fem_lib), "ORACLE_LIB": str(orc_lib),
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    cmd = [sys.executable, "-m", "pytest", str(ROOT / "tests"), "-q", "-m", "not gpu", "-p", "no:cacheprovider"]
    print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, env=env, cwd=str(ROOT)).returncode


if __name__ == "__main__":
    sys.exit(main())

"""Builds liboracle.so from oracle.c with the host C compiler (test infrastructure only)."""
import pathlib
import subprocess

HERE = pathlib.Path(__file__).resolve().parent


def build(verbose: bool = False) -> pathlib.Path:
    out = HERE / "liboracle.so"
    tmp = HERE / "liboracle.so.tmp"
    # -O2 without -ffast-math: IEEE double arithmetic, no reassociation.  OpenMP for the
    # opt-in threaded loops (orc_set_threads; one thread, the default, is sequential).
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", str(tmp),
           str(HERE / "oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    tmp.replace(out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))

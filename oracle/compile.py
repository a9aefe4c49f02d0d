"""Build step for the C oracle (test infrastructure): gcc, -O2, OpenMP,
-ffp-contract=off so that no fused multiply-add changes the operation order of
the printed loop nests; no fast-math."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "thiim_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
          "-Wall", "-Wextra", "-shared", "-fPIC"]


def compile_source(src_path: str, out_path: str) -> str:
    """Compile an oracle source file (also used by the planted-mistake tests
    on modified copies) into a shared library."""
    tmp = out_path + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, src_path, "-o", tmp, "-lm"])
    os.replace(tmp, out_path)
    return out_path


def build_oracle(force: bool = True) -> str:
    if not force and os.path.exists(OUT) and os.path.getmtime(OUT) >= os.path.getmtime(SRC):
        return OUT
    return compile_source(SRC, OUT)


if __name__ == "__main__":
    print(build_oracle())

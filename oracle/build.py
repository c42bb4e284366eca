"""Build the FP64 CPU oracle (test infrastructure only) into oracle/librzo.so,
and its OpenMP timing build (rzo_omp.c, the benchmark's all-core CPU
baseline) into oracle/librzo_omp.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "librzo.so")
LIB_OMP = os.path.join(HERE, "librzo_omp.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB):
        return LIB
    cmd = [
        "gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off",
        "-fPIC", "-shared", os.path.join(HERE, "rzo.c"), "-o", LIB + ".tmp", "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    cmd = [
        "gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fopenmp", "-ffp-contract=off",
        "-fPIC", "-shared", "-I", HERE, os.path.join(HERE, "rzo_omp.c"), "-o", LIB_OMP + ".tmp",
        "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(LIB_OMP + ".tmp", LIB_OMP)
    return LIB


if __name__ == "__main__":
    print(build())

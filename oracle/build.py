"""Build the FP64 CPU oracle (test infrastructure only) into oracle/librzo.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "librzo.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB):
        return LIB
    cmd = [
        "gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off",
        "-fPIC", "-shared", os.path.join(HERE, "rzo.c"), "-o", LIB + ".tmp", "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())

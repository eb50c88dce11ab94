"""Compile the oracle's C library with gcc (plain -O2, no FMA contraction)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sbd_oracle.c")
LIB_PATH = os.path.join(HERE, "liborc.so")


def build() -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-o", LIB_PATH + ".tmp", SRC]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build())

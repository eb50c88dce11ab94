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


ASAN_LIB_PATH = os.path.join(HERE, "_build_asan", "liborc_asan.so")


def build_sanitized() -> str:
    """The oracle built with clang's AddressSanitizer and UBSan (serial: without
    OpenMP), for CPU checks; load it with ORC_LIB_PATH pointing at it and the
    ASan runtime preloaded."""
    os.makedirs(os.path.dirname(ASAN_LIB_PATH), exist_ok=True)
    cmd = ["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-shared-libsan", "-ffp-contract=off", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-Wno-unknown-pragmas", "-o", ASAN_LIB_PATH, SRC]
    subprocess.run(cmd, check=True)
    return ASAN_LIB_PATH


if __name__ == "__main__":
    import sys
    print(build_sanitized() if len(sys.argv) > 1 and sys.argv[1] == "--sanitize" else build())

"""Compile the HIP library libsbd.so for gfx950 in-tree with hipcc.

The library records a hash of the sources it was built from
(``sbd_source_hash``); the Python binding refuses to load a library whose
hash differs from the sources next to it, so a stale build fails loudly."""
import hashlib
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB_PATH = os.path.join(HERE, "libsbd.so")
SOURCES = ["abi.cpp", "davidson.cpp", "tune.cpp", "serve.cpp", "pool.cpp", "noalloc.cpp", "full.cpp", "sqd.cpp", "k_tables.hip", "k_ham.hip", "k_sigma.hip", "k_vec.hip", "k_project.hip", "k_csr.hip", "k_full.hip", "k_devloop.hip"]
ARCH = os.environ.get("SBD_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-result"]


def source_hash() -> str:
    """Hash of every source and header the library is built from."""
    h = hashlib.sha256()
    names = sorted(SOURCES) + ["internal.h"]
    for n in names:
        h.update(n.encode())
        with open(os.path.join(CSRC, n), "rb") as f:
            h.update(f.read())
    with open(os.path.join(HERE, "..", "include", "sbd.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def _compile(src, digest):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, f'-DSBD_SOURCE_HASH="{digest}"', "-x", "hip", "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    return obj, warn


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    digest = source_hash()
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(lambda s: _compile(s, digest), SOURCES))
    if verbose:
        for _, w in results:
            if w.strip():
                print(w, file=sys.stderr)
    objs = [o for o, _ in results]
    tmp = LIB_PATH + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


ASAN_BUILD = os.path.join(HERE, "_build_asan")
ASAN_LIB_PATH = os.path.join(ASAN_BUILD, "libsbd_asan.so")
# AddressSanitizer and UBSan on the host code only (the device code is built as usual)
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer",
              "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-g"]


def build_sanitized() -> str:
    """libsbd with its host code instrumented by AddressSanitizer and UBSan, for
    CPU-only checks of the host logic (argument validation, handles, the
    serving queue bookkeeping).  Load it with SBD_LIB_PATH pointing at it and
    the compiler's ASan runtime preloaded (it records the same source hash)."""
    os.makedirs(ASAN_BUILD, exist_ok=True)
    digest = source_hash()

    def one(src):
        obj = os.path.join(ASAN_BUILD, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *FLAGS, *ASAN_FLAGS, f'-DSBD_SOURCE_HASH="{digest}"', "-x", "hip", "-c",
               os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(one, SOURCES))
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-Xarch_host", "-fsanitize=address,undefined",
           "-shared-libsan", *objs, "-o", ASAN_LIB_PATH]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    return ASAN_LIB_PATH


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--sanitize":
        print(build_sanitized())
    else:
        print(build(verbose=True))

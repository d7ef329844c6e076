"""Build libckv.so (HIP, gfx950) in-tree."""

from __future__ import annotations

import glob
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_DIR = os.path.join(HERE, "_lib")
LIB_PATH = os.path.join(LIB_DIR, "libckv.so")
ARCH = os.environ.get("CKV_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


STAMP_PATH = os.path.join(LIB_DIR, "libckv.sources")


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.cpp")) +
                  glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def source_hash() -> str:
    """SHA-256 (16 hex digits) of every file the library is built from: the
    kernel and host sources, the internal header and the public header."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(HERE, "csrc", "*"))) + \
        [os.path.join(ROOT, "include", "ckv.h")]
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def built_hash():
    """Source hash recorded when the library in _lib/ was linked, or None."""
    try:
        with open(STAMP_PATH) as f:
            return f.read().strip()
    except OSError:
        return None


def build(verbose: bool = False, extra_flags=()) -> str:
    os.makedirs(LIB_DIR, exist_ok=True)
    stamp = source_hash()            # taken before compiling: an edit during the build shows
    objs = []
    common = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
              "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
              # packed FP32 math stays off: scalar FP32 only
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wall", "-Wno-unused-function", *extra_flags]
    for src in sources():
        obj = os.path.join(LIB_DIR, os.path.basename(src) + ".o")
        cmd = common + ["-x", "hip", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{out}")
        if verbose and out.strip():
            print(out)
        objs.append(obj)
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB_PATH)
    with open(STAMP_PATH + ".tmp", "w") as f:
        f.write(stamp + "\n")
    os.replace(STAMP_PATH + ".tmp", STAMP_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

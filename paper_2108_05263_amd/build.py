"""Build libgi.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc."""
import hashlib
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libgi.so")
SOURCES = [os.path.join(CSRC, "gi_kernels.hip"), os.path.join(CSRC, "gi_mlp.hip"), os.path.join(CSRC, "gi_accel.cpp")]
DEPS = SOURCES + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))] + \
    [os.path.join(INCLUDE, "gi.h")]

# -packed-fp32-ops: no packed FP32 instructions are generated
HIPCC_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared", "-I", INCLUDE, "-I", CSRC,
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.exists(cand) or cand == "hipcc"):
            return cand
    return "hipcc"


def source_hash(extra=()) -> str:
    """SHA-256 (16 hex digits) of every source and header the library is
    built from and of the compiler flags: the library embeds it, and loading
    refuses a library whose hash differs from that of the sources in the tree."""
    h = hashlib.sha256()
    for d in sorted(DEPS):
        with open(d, "rb") as fh:
            h.update(os.path.basename(d).encode() + b"\0" + fh.read())
    # flags without the tree's absolute include paths (the box copies the tree elsewhere)
    flags = [os.path.relpath(f, ROOT) if os.path.isabs(f) else f for f in HIPCC_FLAGS + list(extra)]
    h.update(" ".join(flags).encode())
    return h.hexdigest()[:16]


MARKER = b"GI_BUILD_HASH="


def built_hash():
    """The source hash embedded in the built library, or None."""
    if not os.path.exists(LIB):
        return None
    with open(LIB, "rb") as fh:
        m = re.search(re.escape(MARKER) + rb"([0-9a-f]{16})", fh.read())
    return m.group(1).decode() if m else None


def build(verbose: bool = False, extra=()) -> str:
    tag = source_hash(extra)
    cmd = [hipcc()] + HIPCC_FLAGS + list(extra) + [f'-DGI_BUILD_HASH="{tag}"', "-o", LIB + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def is_stale() -> bool:
    """True when the library is missing or was built from other sources or flags."""
    return built_hash() != source_hash()


if __name__ == "__main__":
    extra = sys.argv[1:]
    print(build(verbose=True, extra=extra))

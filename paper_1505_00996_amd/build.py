"""Build libgf.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1505_00996_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libgf.so")
SOURCES = ["gf_kernels.hip", "gf_kernels_padded.hip", "gf_kernels_color.hip", "gf_kernels_outbox.hip", "gf_batched.hip", "gf_noalloc.hip", "gf_api.cpp", "gf_ctx.cpp", "gf_tune.cpp",
           "gf_batch_host.cpp", "gf_engine.cpp"]
ARCH = "gfx950"
# Measurement-only bandwidth probes (bench.py), a library of their own.
PROBE_SRC = "gf_bwprobe.hip"
PROBE_LIB = os.path.join(PKG, "libgf_bwprobe.so")

# Packed FP32 instructions are disabled for the device code on purpose.
HIPFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def _inputs():
    """Every file the library is built from: sources, headers, this script."""
    files = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp", ".h"))]
    inc = os.path.join(ROOT, "include")
    files += [os.path.join(inc, f) for f in os.listdir(inc) if f.endswith(".h")]
    return files + [os.path.abspath(__file__)]


def source_hash() -> str:
    """SHA-256 over the contents of every file the library is built from."""
    import hashlib
    h = hashlib.sha256()
    for f in sorted(_inputs()):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stale(out: str = LIB) -> bool:
    """True when the library is missing or was built from other sources than
    the current ones (the hash written beside it at build time differs)."""
    try:
        with open(out + ".sources") as fh:
            built_from = fh.read().strip()
    except OSError:
        return True
    return not os.path.exists(out) or built_from != source_hash()


def build(out: str = LIB, verbose: bool = False, incremental: bool = False) -> str:
    """Compile the sources and link libgf.so.  By default every translation
    unit is recompiled; with incremental=True only those whose object is
    older than the source, any header or this script."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    digest = source_hash()  # of the sources as this build reads them
    objs, procs = [], []
    bdir = os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    headers = [f for f in _inputs() if not f.endswith((".hip", ".cpp"))]
    newest_header = max(os.path.getmtime(f) for f in headers)
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(bdir, src + ".o")
        if incremental and os.path.exists(obj) and \
                os.path.getmtime(obj) >= max(os.path.getmtime(path), newest_header):
            objs.append(obj)
            continue
        cmd = [hipcc, *HIPFLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", path, "-o", obj]
        if src.endswith(".cpp"):  # host-only code: plain C++ against the HIP runtime API
            cxx = os.environ.get("CXX_HOST", "/opt/rocm/llvm/bin/clang++")
            cmd = [cxx, "-x", "c++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__",
                   "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                   "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))  # translation units compile in parallel
        objs.append(obj)
    failed = [src for src, pr in procs if pr.wait() != 0]
    if failed:
        raise RuntimeError(f"compilation failed: {failed}")
    tmp = out + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    with open(out + ".sources", "w") as fh:
        fh.write(digest + "\n")
    if out == LIB:
        build_probe()
    return out


def build_probe(out: str = PROBE_LIB) -> str:
    """Compile the bandwidth probes (gf_bwprobe.hip) into their own library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    subprocess.check_call([hipcc, *HIPFLAGS, "-shared", "-o", tmp, os.path.join(CSRC, PROBE_SRC)])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))

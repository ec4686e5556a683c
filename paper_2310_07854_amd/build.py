"""Builds libvapr.so (HIP kernels + C ABI) for gfx950 in-tree with hipcc.

Usage: python -m paper_2310_07854_amd.build [--ubsan]  (or build() from Python).  Always recompiles.
--ubsan builds libvapr_ubsan.so, the same library with undefined-behaviour checks in its host code;
VAPR_LIB=<path> makes the binding load that file instead of libvapr.so.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libvapr.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["kernels.hip", "seednet.hip", "vapr.cpp"]
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 math stays off: hipcc must not form v_pk_{add,mul,fma}_f32 on its own
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-rdc",
    "-Wall",
    "-Wno-unused-function",
]


# Host-code undefined-behaviour checks (bounds, overflow, misaligned or null access, bad casts)
# for the C ABI and the launch wrappers; device code is compiled as usual.  The runtime is linked
# as a shared library, so the build loads into an unsanitised Python like the plain one.
UBSAN_LIB = os.path.join(PKG, "libvapr_ubsan.so")
UBSAN_CFLAGS = ["-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
UBSAN_LDFLAGS = ["-Xarch_host", "-fsanitize=undefined", "-shared-libsan"]


def _ubsan_rpath():
    """-rpath to the directory of the driver's shared UBSan runtime."""
    res = subprocess.run([HIPCC, "-print-file-name=libclang_rt.ubsan_standalone-x86_64.so"], capture_output=True,
                         text=True)
    f = res.stdout.strip().splitlines()[-1] if res.returncode == 0 and res.stdout.strip() else ""
    return [f"-Wl,-rpath,{os.path.dirname(f)}"] if os.path.isabs(f) and os.path.exists(f) else []


def build(verbose: bool = False, ubsan: bool = False) -> str:
    """Compile every source to an object in parallel, then link the shared library (with ubsan:
    the undefined-behaviour-checked host build, libvapr_ubsan.so, beside the plain one)."""
    lib_out = UBSAN_LIB if ubsan else LIB
    tmp = lib_out + ".tmp"
    objdir = os.path.join(PKG, "_build_ubsan" if ubsan else "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in FLAGS if f != "-shared"] + (UBSAN_CFLAGS if ubsan else [])
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmd = [HIPCC, *compile_flags, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = False
    for obj, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out)
            failed = True
        elif verbose and out.strip():
            sys.stderr.write(out)
    if failed:
        raise RuntimeError("hipcc failed")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-fno-gpu-rdc", *[o for o, _ in procs], "-o", tmp]
    if ubsan:
        cmd[1:1] = UBSAN_LDFLAGS + _ubsan_rpath()
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc link failed with exit code {res.returncode}")
    os.replace(tmp, lib_out)
    return lib_out


if __name__ == "__main__":
    print(build(verbose=True, ubsan="--ubsan" in sys.argv[1:]))

"""Build librt.so (gfx950) in-tree with hipcc.

Usage: python -m paper_1110_4894_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librt.so")
SOURCES = ["rt_api.hip", "rt_kernels.hip", "rt_pm.hip"]
HEADERS = ["rt_internal.h", "rt_geodesic.h", os.path.join("..", "..", "include", "rt.h")]

# Packed FP32 instructions are switched off for every HIP source (the FP32
# field sum is written for the scalar VALU and the transcendental unit).
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")]
OBJDIR = os.path.join(ROOT, "_build")


def hipcc() -> str:
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if p and os.path.exists(p):
            return p
    return "hipcc"


def llvm_tool(name: str) -> str:
    for d in ("/opt/rocm/llvm/bin", "/opt/rocm/lib/llvm/bin"):
        p = os.path.join(d, name)
        if os.path.exists(p):
            return p
    return name


def check_no_calls(obj: str) -> None:
    """Every device function of the library is inlined into its kernel.  A large
    called function reaches its far blocks through long branches, and the
    compiler builds their targets in the register pair that holds the
    function's return address, so such a function may never return.  Fail the
    build if a gfx950 kernel of this object calls anything."""
    import tempfile
    sections = subprocess.run([llvm_tool("llvm-readobj"), "--sections", obj], check=True, capture_output=True,
                              text=True).stdout
    if ".hip_fatbin" not in sections:
        return   # host code only
    with tempfile.TemporaryDirectory() as tmp:
        fat = os.path.join(tmp, "fatbin")
        co = os.path.join(tmp, "co")
        subprocess.run([llvm_tool("llvm-objcopy"), "--dump-section=.hip_fatbin=" + fat, obj], check=True)
        subprocess.run([llvm_tool("clang-offload-bundler"), "--unbundle", "--type=o",
                        "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", "--input=" + fat, "--output=" + co],
                       check=True)
        dis = subprocess.run([llvm_tool("llvm-objdump"), "-d", "--mcpu=gfx950", co], check=True,
                             capture_output=True, text=True).stdout
    bad = [l.strip() for l in dis.splitlines() if "s_swappc_b64" in l or "s_getpc_b64 s[30:31]" in l]
    if bad:
        raise RuntimeError("%s: gfx950 code calls a device function (%d instructions, e.g. %s); mark it "
                           "__forceinline__" % (os.path.basename(obj), len(bad), bad[0]))


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link librt.so."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJDIR, exist_ok=True)
    objs = [os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]

    def compile_one(i):
        cmd = [hipcc()] + FLAGS + ["-c", os.path.join(CSRC, SOURCES[i]), "-o", objs[i]]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    with ThreadPoolExecutor(len(SOURCES)) as ex:
        list(ex.map(compile_one, range(len(SOURCES))))
    for o in objs:
        check_no_calls(o)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS]
    return any(os.path.getmtime(d) > t for d in deps if os.path.exists(d))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build libnfs.so (gfx950) in-tree with hipcc.

    python -m paper_1209_3362_amd.build        # or paper_1209_3362_amd.build.build()

Every call compiles every source again; objects go to _build/ at the repo
root, the library to paper_1209_3362_amd/libnfs.so.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libnfs.so")

HIP_SOURCES = ["fft.hip", "pairs.hip", "bins.hip", "misc.hip", "backward.hip",
               "static_scratch.hip"]
CPP_SOURCES = ["pair_plan.cpp", "nfs_host.cpp", "nfs_api.cpp", "nfs_batch.cpp"]
ARCH = "gfx950"


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; ROCm is required to build libnfs.so")
    return exe


def rocm_path():
    return os.environ.get("ROCM_PATH", "/opt/rocm")


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def compile_cmds():
    cmds = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        # Packed FP32 instructions are switched off for all device code.
        cmds.append((obj, [hipcc(), "-x", "hip", "--offload-arch=" + ARCH,
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-ffp-contract=fast"] + common_flags()
                     + ["-c", os.path.join(CSRC, src), "-o", obj]))
    for src in CPP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmds.append((obj, [hipcc(), "-x", "c++", "-D__HIP_PLATFORM_AMD__",
                           "-I" + os.path.join(rocm_path(), "include")] + common_flags()
                     + ["-c", os.path.join(CSRC, src), "-o", obj]))
    return cmds


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("command failed:\n" + " ".join(cmd) + "\n" + p.stdout + p.stderr)
    return p.stderr


def build(verbose=False, jobs=None):
    """Compile every source and link paper_1209_3362_amd/libnfs.so."""
    os.makedirs(BUILD, exist_ok=True)
    cmds = compile_cmds()
    jobs = jobs or min(8, os.cpu_count() or 1, len(cmds))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        logs = list(ex.map(lambda c: _run(c[1], verbose), cmds))
    for log in logs:
        # hipcc's host pass does not know the packed-fp32 feature: harmless.
        lines = [l for l in log.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if lines and verbose:
            print("\n".join(lines))
    tmp = LIB + ".tmp"
    _run([hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp]
         + [obj for obj, _ in cmds], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)

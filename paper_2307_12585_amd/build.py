"""Build libfdemri.so (HIP, gfx950) in-tree.

    python -m paper_2307_12585_amd.build

Every source is compiled for gfx950 only, with packed FP32 instructions
disabled, into objects under _build/ and linked into
paper_2307_12585_amd/libfdemri.so next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libfdemri.so")
SOURCES = ["spline.hip", "pieces.hip", "gather.hip", "vjp.hip", "select.hip", "td.hip", "traj.hip", "spa_eval.hip", "api.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast-honor-pragmas", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    f"-I{os.path.join(ROOT, 'include')}",
]


# Host-code sanitizers for the C-ABI exercise (tests/native/abi_driver.cpp):
# the runtime's host code (api.hip) and the driver are built with
# AddressSanitizer and UndefinedBehaviorSanitizer; each -fsanitize= applies to
# the host pass only (-Xarch_host before it), the device code is unchanged.
SAN_EXE = os.path.join(BUILD, "abi_driver_san")
SAN_DRIVER = os.path.join(ROOT, "tests", "native", "abi_driver.cpp")
SAN_HOST_FLAGS = ["-Xarch_host -fsanitize=address", "-Xarch_host -fsanitize=undefined",
                  "-Xarch_host -fno-omit-frame-pointer", "-Xarch_host -fno-sanitize-recover=undefined"]
CLANGXX = os.environ.get("FDEMRI_HOST_CXX", "/opt/rocm/llvm/bin/clang++")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _split(flags):
    return [x for f in flags for x in f.split()]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose: bool = False) -> str:
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objs = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in srcs]

    def compile_one(pair):
        src, obj = pair
        return _run([HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])

    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        logs = list(ex.map(compile_one, zip(srcs, objs)))
    tmp = LIB + ".tmp"
    logs.append(_run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]))
    os.replace(tmp, LIB)
    logs.append(build_sanitized(objs))
    if verbose:
        for lg in logs:
            if lg.strip():
                print(lg)
    return LIB


def build_sanitized(objs) -> str:
    """The sanitized C-ABI driver: api.hip again with host sanitizers, the
    other objects as built, the driver, linked by the host compiler with the
    sanitizer runtimes."""
    api_san = os.path.join(BUILD, "api_san.o")
    drv = os.path.join(BUILD, "abi_driver_san.o")
    logs = [_run([HIPCC, *FLAGS, "-g", *_split(SAN_HOST_FLAGS), "-c", os.path.join(CSRC, "api.hip"), "-o", api_san]),
            _run([CLANGXX, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                  "-D__HIP_PLATFORM_AMD__", f"-I{os.path.join(ROOT, 'include')}", f"-I{ROCM}/include", "-c",
                  SAN_DRIVER, "-o", drv])]
    others = [o for o in objs if os.path.basename(o) != "api.o"]
    tmp = SAN_EXE + ".tmp"
    logs.append(_run([CLANGXX, "-fsanitize=address,undefined", "-o", tmp, drv, api_san, *others, f"-L{ROCM}/lib",
                      "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib"]))
    os.replace(tmp, SAN_EXE)
    return "\n".join(logs)


if __name__ == "__main__":
    print(build(verbose=True))

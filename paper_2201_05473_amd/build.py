"""Build liblbmpwfa.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_DIR = os.path.join(HERE, "_lib")
LIB_PATH = os.path.join(LIB_DIR, "liblbmpwfa.so")
SOURCES = ("csrc/lbm_kernels.hip", "csrc/lbm_adjoint.hip", "csrc/lbm_bunch.hip", "csrc/lbm_capi.cpp")
HIPCC_FLAGS = (
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off (compiler-generated v_pk_* FP32 ops are avoided)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
)


OBJ_DIR = os.path.join(os.path.dirname(HERE), "_build")


def build(verbose: bool = False) -> str:
    """Compile the library (one object per source, compiled in parallel, then linked); returns its
    path.  Raises CalledProcessError on failure."""
    os.makedirs(LIB_DIR, exist_ok=True)
    os.makedirs(OBJ_DIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    jobs = []
    for src in SOURCES:
        obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
        cmd = [hipcc, *flags, "-c", "-o", obj, os.path.join(HERE, src)]
        jobs.append((cmd, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    objs = []
    for cmd, obj, proc in jobs:
        out, err = proc.communicate()
        if proc.returncode != 0:
            raise subprocess.CalledProcessError(proc.returncode, cmd, out, err)
        if verbose and err:
            print(err)
        objs.append(obj)
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise subprocess.CalledProcessError(res.returncode, cmd, res.stdout, res.stderr)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


C_CLIENT = os.path.join(LIB_DIR, "lbm_c_run")


def build_c_client() -> str:
    """Compile the plain-C client of the ABI (tests/c_api/lbm_c_run.c, host code only, linked to
    the library next to it); returns its path."""
    root = os.path.dirname(HERE)
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = [os.environ.get("CC", "gcc"), "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(rocm, "include"), "-I" + os.path.join(root, "include"),
           "-o", C_CLIENT, os.path.join(root, "tests", "c_api", "lbm_c_run.c"),
           "-L" + LIB_DIR, "-llbmpwfa", "-L" + os.path.join(rocm, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + os.path.join(rocm, "lib")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise subprocess.CalledProcessError(res.returncode, cmd, res.stdout, res.stderr)
    return C_CLIENT


PATTERN_CEILING = os.path.join(LIB_DIR, "pattern_ceiling")


def build_pattern_ceiling() -> str:
    """Compile the standalone memory-pattern ceiling program (csrc/pattern_ceiling.hip: the FP32
    step's access pattern with no arithmetic, and a float4 copy of the same bytes); returns its
    path."""
    os.makedirs(LIB_DIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = [f for f in HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    cmd = [hipcc, *flags, "-o", PATTERN_CEILING, os.path.join(HERE, "csrc", "pattern_ceiling.hip")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise subprocess.CalledProcessError(res.returncode, cmd, res.stdout, res.stderr)
    return PATTERN_CEILING


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_c_client())
    print(build_pattern_ceiling())

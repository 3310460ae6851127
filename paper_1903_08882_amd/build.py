"""Build the gfx950 shared library from csrc/ with hipcc (in-tree).

    python -m paper_1903_08882_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_NAME = "libp1903lbm.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "api.hip", "wsnet.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "-fvisibility=hidden",
    "--offload-arch=gfx950",
    # no packed FP32 instructions are generated (plain scalar/vector FP32 only)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


DEMO_SRC = os.path.join(HERE, "examples", "c_abi_demo.c")
DEMO_PATH = os.path.join(HERE, "c_abi_demo")


def build_demo(verbose=False):
    """The C example (plain C, gcc) against the built library and the HIP runtime."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(rocm, "include"), "-I" + os.path.join(ROOT, "include"), DEMO_SRC,
           "-L" + HERE, "-lp1903lbm", "-L" + os.path.join(rocm, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + os.path.join(rocm, "lib"), "-o", DEMO_PATH]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("gcc failed on the C example:\n" + r.stdout + r.stderr)
    return DEMO_PATH


def build(verbose=False, extra_flags=()):
    """Compile every source into LIB_PATH (always recompiles), then the C example."""
    tmp = LIB_PATH + ".tmp"
    cmd = [HIPCC, *FLAGS, *extra_flags, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB_PATH)
    build_demo(verbose)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build the plain-C caller of the C-ABI (tests/abi_c/abi_check) with gcc
against include/hwenou.h, the HIP runtime and the in-tree libhwenou.so.
Test infrastructure, built by __graft_entry__.build()."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
OUT = os.path.join(HERE, "abi_check")


def build():
    lib_dir = os.path.join(ROOT, "paper_2402_03074_amd")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROCM, "include"), "-I" + os.path.join(ROOT, "include"),
           os.path.join(HERE, "abi_check.c"), "-o", OUT + ".tmp",
           "-L" + lib_dir, "-lhwenou", "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_2402_03074_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
           "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("building abi_check failed:\n" + r.stderr)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(), file=sys.stderr)

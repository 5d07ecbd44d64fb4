"""Compile tests/c/abi_consumer.c (a plain C99 user of libawg) with gcc.

The binary links libawg.so from the package directory through a relative
rpath, so it runs wherever the tree is copied.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SRC = os.path.join(HERE, "abi_consumer.c")
BIN = os.path.join(HERE, "abi_consumer")


def build(out=BIN):
    pkg = os.path.join(ROOT, "paper_2403_15582_amd")
    rel = os.path.relpath(pkg, os.path.dirname(os.path.abspath(out)))
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROCM, "include"), SRC, "-o", out,
           "-L" + pkg, "-lawg", "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/" + rel, "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("abi_consumer build failed: %s\n%s" % (" ".join(cmd), r.stdout))
    return out


if __name__ == "__main__":
    print(build())

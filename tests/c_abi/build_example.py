"""Builds tests/c_abi/solve_example (plain C11 against include/lamp.h and liblamp.so)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build() -> str:
    exe = os.path.join(HERE, "solve_example")
    cmd = ["gcc", "-std=c11", "-Wall", "-Wextra", "-O2", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
           "-o", exe, os.path.join(HERE, "solve_example.c"),
           "-L", os.path.join(ROOT, "paper_2511_11359_amd"), "-llamp",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_2511_11359_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    subprocess.run(cmd, check=True)
    return exe


if __name__ == "__main__":
    print(build())

"""Builds tests/cpp/abi_client, a plain C program that calls the library
through its C ABI (include/aesgpu.h) and the HIP runtime only.  Run by the
package build entry point after libaesgpu.so is built; the GPU test
tests/test_gpu_abi_client.py runs the binary."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
EXE = os.path.join(HERE, "abi_client")


def build():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    pkg = os.path.join(ROOT, "paper_1403_7295_amd")
    tmp = EXE + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(rocm, "include"), "-I" + os.path.join(ROOT, "include"),
           os.path.join(HERE, "abi_client.c"), "-o", tmp,
           "-L" + pkg, "-laesgpu", "-L" + os.path.join(rocm, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_1403_7295_amd", "-Wl,-rpath," + os.path.join(rocm, "lib")]
    subprocess.run(cmd, check=True)
    os.replace(tmp, EXE)
    return EXE


if __name__ == "__main__":
    print(build())

"""Build the C client of the library's ABI (lb_client.c) beside its source:
plain gcc, C99, the HIP runtime for device memory and the stream, and
liblbf.so found through a run path relative to the executable."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SRC = os.path.join(HERE, "lb_client.c")
EXE = os.path.join(HERE, "lb_client")


def build() -> str:
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"), SRC, "-o", EXE,
           "-L", os.path.join(ROOT, "paper_0707_1581_amd"), "-llbf", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_0707_1581_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"gcc failed ({proc.returncode}):\n{proc.stderr}")
    return EXE


if __name__ == "__main__":
    print(build())

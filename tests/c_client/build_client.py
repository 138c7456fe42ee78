"""Builds fk_client, the plain-C consumer of libfkmi.so (gcc, C11, the HIP
runtime API for device memory), next to its source.  The binary finds the
library through an $ORIGIN-relative run path, so the tree can move."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "fk_client.c")
BIN = os.path.join(HERE, "fk_client")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(out: str = BIN) -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           f"-I{ROCM}/include", f"-I{os.path.join(ROOT, 'include')}", SRC, "-o", out,
           f"-L{os.path.join(ROOT, 'paper_2508_07071_amd')}", "-lfkmi", f"-L{ROCM}/lib", "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_2508_07071_amd", f"-Wl,-rpath,{ROCM}/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("fk_client build failed:\n" + r.stderr)
    return out


if __name__ == "__main__":
    print(build())

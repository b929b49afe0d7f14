"""Compile the plain-C clients of the C ABI in this folder against the
in-tree library (gcc, the HIP runtime for device memory, no torch)."""
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))


def build() -> list:
    out = []
    for src in sorted(glob.glob(os.path.join(HERE, "*.c"))):
        exe = src[:-2]
        cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
               "-I" + os.path.join(ROOT, "include"), src, "-L" + os.path.join(ROOT, "paper_2402_01181_amd"),
               "-lmpm355", "-L/opt/rocm/lib", "-lamdhip64", "-lm",
               "-Wl,-rpath,$ORIGIN/../../paper_2402_01181_amd", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
        subprocess.run(cmd, check=True)
        out.append(exe)
    return out


if __name__ == "__main__":
    print("\n".join(build()))

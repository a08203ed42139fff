"""Build the CPU emulation of libfdas (test infrastructure only): the same
C-ABI and kernel sources compiled with g++ against tests/emu/hip/*.h, where
each workgroup runs as threads on the host.  Output: tests/emu/_build/libfdas_emu.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1804_05335_amd", "csrc")
OUT = os.path.join(HERE, "_build", "libfdas_emu.so")
CXX = "/opt/rocm/llvm/bin/clang++"


def build() -> str:
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    srcs = [os.path.join(CSRC, f) for f in ("fdas_api.cpp", "fdas_templates.cpp", "fdas_kernels.hip",
                                                  "fdas_r2c.hip", "fdas_harmonic.hip",
                                                  "fdas_stream.hip")]
    tmp = OUT + f".tmp{os.getpid()}"
    # clang (ROCm's, as a host compiler): the kernels use clang vector types
    # a small persistent grid for the batched harmonic kernels: every
    # emulated workgroup is a set of host threads
    cmd = [CXX, "-O2", "-std=c++20", "-fPIC", "-shared", "-pthread", "-I", HERE,
           "-I", os.path.join(ROOT, "include"), "-DFDAS_HARM_BATCHED_GRID=3",
           "-x", "c++"] + srcs + ["-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


def build_lds_layout() -> str:
    """The transforms' LDS index map alone (tests/emu/lds_layout.cpp)."""
    out = os.path.join(HERE, "_build", "liblds_layout.so")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + f".tmp{os.getpid()}"
    subprocess.run([CXX, "-O1", "-std=c++20", "-fPIC", "-shared", "-I", HERE, "-x", "c++",
                    os.path.join(HERE, "lds_layout.cpp"), "-o", tmp], check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())

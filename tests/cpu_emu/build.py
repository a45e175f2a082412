"""Builds the CPU emulation of libevsim (TEST INFRASTRUCTURE): the unmodified HIP sources of
paper_2209_04634_amd/csrc compiled as host C++ against tests/cpu_emu/hip/hip_runtime.h."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2209_04634_amd", "csrc")
SOURCES = [os.path.join(CSRC, "evsim_kernels.hip"), os.path.join(CSRC, "evsim_runtime.hip"),
           os.path.join(CSRC, "evsim_server.hip"), os.path.join(CSRC, "evsim_lk.hip")]


def lib_path(asan: bool = False, ubsan: bool = False) -> str:
    name = "libevsim_cpu_asan.so" if asan else ("libevsim_cpu_ubsan.so" if ubsan else
                                                 "libevsim_cpu.so")
    return os.path.join(HERE, name)


def build(asan: bool = False, force: bool = False, ubsan: bool = False) -> str:
    """asan: AddressSanitizer build (load with libasan preloaded) that also aborts at the first
    undefined operation (signed overflow, shift out of range, misaligned or null access); ubsan:
    the undefined-behaviour checks alone."""
    out = lib_path(asan, ubsan)
    deps = SOURCES + [os.path.join(CSRC, "evsim_internal.h"), os.path.join(HERE, "emu.cpp"),
                      os.path.join(HERE, "hip", "hip_runtime.h"),
                      os.path.join(ROOT, "include", "sim.h")]
    if (not force and os.path.exists(out)
            and os.path.getmtime(out) >= max(os.path.getmtime(d) for d in deps)):
        return out
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
             "-fno-fast-math", "-Wno-unknown-pragmas", "-Wno-unused-result",
             "-I", HERE, "-I", os.path.join(ROOT, "include"), "-Wl,-Bsymbolic"]
    if asan:   # undefined-behaviour checks ride along with the address checks
        flags += ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                  "-fno-sanitize=vptr", "-fno-omit-frame-pointer"]
    elif ubsan:
        flags += ["-fsanitize=undefined", "-fno-sanitize-recover=undefined", "-fno-sanitize=vptr"]
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["g++", *flags, "-x", "c++", *SOURCES, "-x", "none", os.path.join(HERE, "emu.cpp"),
           "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(force=True))
    print(build(asan=True, force=True))
    print(build(ubsan=True, force=True))

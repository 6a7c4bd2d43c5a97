"""Build the test-only CPU version of liblrdm's kernels with AddressSanitizer.

The kernel sources are copied with their <<<...>>> launches rewritten as calls
of lrdm_emu::launch and compiled by the host clang against the HIP stand-in in
tests/cpu_emu/hip/hip_runtime.h, then linked with the C ABI layer (api.cpp,
validate.cpp) and a driver into one executable.  Used only by tests.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2211_07894_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "emu")
CLANG = "/opt/rocm/llvm/bin/clang++"
FLAGS = ["-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
         "-Wno-unused-result", f"-I{HERE}", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]

LAUNCH = re.compile(r"(\b[\w:]+(?:<[^;{}()]*?>)?)\s*<<<\s*(.*?)\s*>>>\s*\(", re.S)


DYN_SMEM = re.compile(r"extern __shared__ (?:__attribute__\(\(aligned\(\d+\)\)\) )?unsigned char (\w+)\[\];")
WAIT_BARRIER = re.compile(r'asm volatile\("s_waitcnt[^"]*s_barrier"[^;]*;')


def translate(src: str) -> str:
    src = LAUNCH.sub(lambda m: f"lrdm_emu::launch({m.group(1)}, {m.group(2)}, ", src)
    src = DYN_SMEM.sub(lambda m: f"unsigned char* {m.group(1)} = lrdm_emu::dyn_smem();", src)
    # a wait for this wave's global->LDS copies plus a block barrier: the stand-in
    # performs those copies at once, so a barrier remains
    src = WAIT_BARRIER.sub("__syncthreads();", src)
    return src


def build(driver: str, shared: bool = False) -> str:
    """The ASan driver executable, or (shared=True) an optimised shared library
    exporting the C ABI on host memory, without a sanitizer, for numerical checks
    of the kernels against the oracle on the CPU."""
    out = os.path.join(OUT, "shared") if shared else OUT
    flags = ([f for f in FLAGS if f not in ("-fsanitize=address", "-O1")] + ["-O2", "-fPIC"]
             if shared else FLAGS)
    os.makedirs(os.path.join(out, "src"), exist_ok=True)
    units = []
    for f in sorted(os.listdir(CSRC)):
        if not f.endswith((".hip", ".cpp")):
            continue
        text = open(os.path.join(CSRC, f)).read()
        dst = os.path.join(out, "src", f.rsplit(".", 1)[0] + ".cpp")
        open(dst, "w").write(translate(text) if f.endswith(".hip") else text)
        units.append(dst)
    units.append(os.path.join(HERE, "emu_runtime.cpp"))
    if not shared:
        units.append(driver)

    def comp(u):
        obj = os.path.join(out, os.path.basename(u) + ".o")
        r = subprocess.run([CLANG, *flags, "-c", u, "-o", obj], capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError(f"{u}:\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(comp, units))
    if shared:
        exe = os.path.join(out, "liblrdm_emu.so")
        cmd = [CLANG, "-shared", *objs, "-o", exe, "-lpthread"]
    else:
        exe = os.path.join(out, "lrdm_emu_driver")
        cmd = [CLANG, "-fsanitize=address", *objs, "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(r.stderr)
    return exe


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--shared":
        print(build("", shared=True))
    else:
        print(build(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "driver.cpp")))

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


def build(driver: str) -> str:
    os.makedirs(os.path.join(OUT, "src"), exist_ok=True)
    units = []
    for f in sorted(os.listdir(CSRC)):
        if not f.endswith((".hip", ".cpp")):
            continue
        text = open(os.path.join(CSRC, f)).read()
        dst = os.path.join(OUT, "src", f.rsplit(".", 1)[0] + ".cpp")
        open(dst, "w").write(translate(text) if f.endswith(".hip") else text)
        units.append(dst)
    units.append(os.path.join(HERE, "emu_runtime.cpp"))
    units.append(driver)

    def comp(u):
        obj = os.path.join(OUT, os.path.basename(u) + ".o")
        r = subprocess.run([CLANG, *FLAGS, "-c", u, "-o", obj], capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError(f"{u}:\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(comp, units))
    exe = os.path.join(OUT, "lrdm_emu_driver")
    r = subprocess.run([CLANG, "-fsanitize=address", *objs, "-o", exe, "-lpthread"],
                       capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(r.stderr)
    return exe


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "driver.cpp")))

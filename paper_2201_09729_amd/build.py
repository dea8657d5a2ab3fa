"""Build libdlma.so (HIP for gfx950) in-tree.

Each source compiles to an object in ``_build/`` in parallel, then one link
produces ``paper_2201_09729_amd/libdlma.so``.  Packed FP32 instructions are
disabled for all device code (-packed-fp32-ops).

Every kernel's machine code is then checked for one hazard: a vector-memory store
with more than 64 bits of data whose data registers a vector ALU instruction
overwrites less than two wait states later.  Such a store reads its data after
issue, the compiler in use does not separate the two, and the result is a
corrupted store that varies from run to run.  Code that stores wide vectors fences
them (``wide_store_begin`` / ``wide_store_end`` in csrc/common.h); the check
fails the build if any such pair remains.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdlma.so")
ARCH = os.environ.get("DLMA_ARCH", "gfx950")

SOURCES = [
    "hop_p64.hip", "hop_p32.hip", "hop_p16.hip", "hop_pb16.hip",
    "kern_misc.hip", "laplace.hip", "contract.hip", "bicg.hip",
    "runtime.cpp", "api_gauge.cpp", "api_solve.cpp", "api_eigs.cpp", "api_noalloc.cpp",
]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + CSRC, "-I" + os.path.join(ROOT, "include")]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src.replace(".", "_") + ".o")
    # every file is HIP: the host files include the kernel headers for their launch descriptors
    cmd = [HIPCC, "-x", "hip"] + DEVICE + COMMON + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


LLVM = os.environ.get("DLMA_LLVM_BIN", "/opt/rocm/llvm/bin")
WIDE_STORE = re.compile(r"(buffer|global|flat|scratch)_store_dwordx[34]$")


def _vregs(tok: str) -> set:
    m = re.match(r"v\[(\d+):(\d+)\]", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", tok)
    return {int(m.group(1))} if m else set()


def store_data_hazards(asm: str, need: int = 2) -> list:
    """(kernel, store, instruction) for each vector ALU write of a wide store's data
    registers fewer than `need` wait states after the store (s_nop N counts N + 1)."""
    out, fn, pending = [], "?", []
    for line in asm.splitlines():
        m = re.match(r"^[0-9a-f]+ <(\S+)>:", line)
        if m:
            fn, pending = m.group(1), []
            continue
        ins = line.split("//")[0].strip()
        if not ins or ins.endswith(":"):
            continue
        t = ins.replace(",", " ").split()
        op = t[0]
        if op.startswith("v_") and not op.startswith("v_cmp") and len(t) > 1:
            dst = _vregs(t[1])
            for data, store, _ in pending:
                if dst & data:
                    out.append((fn, store, ins))
        ws = int(t[1]) + 1 if op == "s_nop" and len(t) > 1 else 1
        pending = [(d, st, w + ws) for d, st, w in pending if w + ws < need]
        if WIDE_STORE.match(op):
            data = _vregs(t[1] if op.startswith("buffer") else t[2])
            pending.append((data, ins, 0))
    return out


def check_object(obj: str) -> list:
    """Disassemble the gfx950 code object of one of our objects and scan it."""
    with tempfile.TemporaryDirectory() as d:
        fb, co = os.path.join(d, "fatbin"), os.path.join(d, "co")
        r = subprocess.run([os.path.join(LLVM, "llvm-objcopy"), "--dump-section", ".hip_fatbin=" + fb, obj],
                           capture_output=True, text=True)
        if r.returncode != 0:
            return []  # host-only object
        subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o", "--input=" + fb,
                        "--targets=hipv4-amdgcn-amd-amdhsa--" + ARCH, "--output=" + co], check=True,
                       capture_output=True)
        asm = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", "--mcpu=" + ARCH, co], check=True,
                             capture_output=True, text=True).stdout
    return store_data_hazards(asm)


def build(jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(8, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
        found = [h for hs in ex.map(check_object, objs) for h in hs]
    if found:
        raise RuntimeError("wide-store data hazard in the machine code:\n" +
                           "\n".join("  %s: %s -> %s" % h for h in found))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lamdhip64"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else None))

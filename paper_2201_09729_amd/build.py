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


_ADDR = re.compile(r"//\s*([0-9A-Fa-f]+):")
_TARGET = re.compile(r"<(\S+)\+0x([0-9a-fA-F]+)>")
_ENDS = ("s_endpgm", "s_setpc_b64", "s_trap", "s_rfe_b64")


def _functions(asm: str):
    """Per function: its name and [(address, op, tokens, text, branch target address)]."""
    fns, cur, base = [], None, 0
    for line in asm.splitlines():
        m = re.match(r"^([0-9a-f]+) <(\S+)>:", line)
        if m:
            base = int(m.group(1), 16)
            cur = (m.group(2), [])
            fns.append(cur)
            continue
        if cur is None:
            continue
        code, _, comment = line.partition("//")
        ins = code.strip()
        if not ins or ins.endswith(":"):
            continue
        ma = _ADDR.search(line)
        addr = int(ma.group(1), 16) if ma else (cur[1][-1][0] + 4 if cur[1] else base)
        mt = _TARGET.search(comment)
        tgt = base + int(mt.group(2), 16) if (mt and mt.group(1) == cur[0]) else None
        t = ins.replace(",", " ").split()
        cur[1].append((addr, t[0], t, ins, tgt))
    return fns


def store_data_hazards(asm: str, need: int = 2) -> list:
    """(kernel, store, instruction) for each vector ALU write of a wide store's data
    registers fewer than `need` wait states after the store (s_nop N counts N + 1), on
    every path from the store: fall-through and branch targets both.  Every issued
    instruction other than s_nop counts as one wait state, branches included."""
    out = []
    for fn, code in _functions(asm):
        at = {a: i for i, (a, *_rest) in enumerate(code)}
        for i, (_, op, t, ins, _) in enumerate(code):
            if not WIDE_STORE.match(op):
                continue
            data = _vregs(t[1] if op.startswith("buffer") else t[2])
            stack, seen = [(i + 1, 0)], set()
            while stack:
                j, w = stack.pop()
                if j >= len(code) or (j, w) in seen:
                    continue
                seen.add((j, w))
                _, opj, tj, insj, tgt = code[j]
                if opj.startswith("v_") and not opj.startswith("v_cmp") and len(tj) > 1 and _vregs(tj[1]) & data:
                    out.append((fn, ins, insj))
                    continue
                is_branch = opj.startswith("s_branch") or opj.startswith("s_cbranch")
                w2 = w + (int(tj[1]) + 1 if opj == "s_nop" and len(tj) > 1 else 1)
                if w2 >= need or opj in _ENDS:
                    continue
                if is_branch and tgt is not None and tgt in at:
                    stack.append((at[tgt], w2))
                if opj != "s_branch":
                    stack.append((j + 1, w2))
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

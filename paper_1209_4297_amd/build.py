"""Build the RIDC HIP library (``libridc.so``) in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import re
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libridc.so")

ARCH = "gfx950"
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 vector instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the RIDC library)")


# Matrix-core accumulator check.  An MFMA whose accumulator source (srcC) is not its destination
# can still be waiting for the matrix core (two waves share it) when the instructions after it
# issue; a non-MFMA instruction that writes one of those srcC registers shortly after (an LDS
# load of the next fragments, a VALU op) then changes the value the MFMA accumulates.  The
# compiler's wait states did not cover this for LDS loads: such a schedule gave results off by
# 1e-8..1e-4 that changed from run to run, and the schedules without it were exact.  build()
# rejects any kernel whose assembly contains the pattern within MFMA_WAR_WINDOW instructions.
MFMA_WAR_WINDOW = 16
_REG = re.compile(r"([va])\[(\d+):(\d+)\]|([va])(\d+)$")


def _regs(tok: str):
    m = _REG.match(tok.strip())
    if not m:
        return set()
    if m.group(1):
        return {(m.group(1), r) for r in range(int(m.group(2)), int(m.group(3)) + 1)}
    return {(m.group(4), int(m.group(5)))}


def mfma_accumulator_hazards(asm: str, window: int = MFMA_WAR_WINDOW):
    """(function, line, mfma, writer) for every MFMA with srcC != vdst whose srcC registers a
    non-MFMA instruction writes within `window` instructions after it."""
    out = []
    func = None
    body = []

    def flush():
        for i, line in enumerate(body):
            if not line.startswith("v_mfma"):
                continue
            ops = [t.strip() for t in line.split(None, 1)[1].split(",")]
            if len(ops) < 4 or _regs(ops[0]) == _regs(ops[3]):
                continue
            srcc = _regs(ops[3])
            for j in range(i + 1, min(len(body), i + 1 + window)):
                nxt = body[j]
                parts = nxt.split(None, 1)
                if (len(parts) < 2 or nxt.startswith("v_mfma")
                        or nxt.startswith(("ds_write", "global_store", "buffer_store", "s_"))):
                    continue
                if _regs(parts[1].split(",")[0]) & srcc:
                    out.append((func, i, line, nxt))
                    break

    for raw in asm.splitlines():
        line = raw.strip()
        if not line or line.startswith(";"):
            continue
        if re.match(r"^[A-Za-z_][\w.$]*:", line) and not line.startswith(".L"):
            flush()
            func, body = line.split(":")[0], []
            continue
        if line.startswith("."):
            continue
        body.append(line.split(";")[0].strip())
    flush()
    return out


def check_mfma_schedule(hipcc: str, src: str) -> None:
    """Compile `src` to gfx950 assembly and raise if any kernel holds the accumulator pattern."""
    asm_path = os.path.join(BUILD, os.path.basename(src) + ".s")
    cmd = [hipcc, *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "--cuda-device-only", "-S", src,
           "-o", asm_path]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc -S failed on {src}:\n{res.stdout}\n{res.stderr}")
    with open(asm_path) as f:
        hits = mfma_accumulator_hazards(f.read())
    if hits:
        fn, _, mfma, writer = hits[0]
        raise RuntimeError(f"{src}: {len(hits)} MFMA accumulator sources overwritten while the "
                           f"MFMA may not have read them, first in {fn}: '{mfma}' then '{writer}'")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def build(verbose: bool = False) -> str:
    """Compile every source under csrc/ and link ``libridc.so``; returns its path."""
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()

    def compile_one(src):
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        cmd = [hipcc, *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{res.stdout}\n{res.stderr}")
        return obj

    mfma_srcs = [s for s in srcs if s.endswith(".hip") and "mfma" in open(s).read()]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs) + len(mfma_srcs))) as ex:
        checks = [ex.submit(check_mfma_schedule, hipcc, s) for s in mfma_srcs]
        objs = list(ex.map(compile_one, srcs))
        for c in checks:
            c.result()
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

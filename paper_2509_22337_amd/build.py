"""Builds libfastlbp.so for gfx950 with hipcc (in-tree, next to this file).

Every source compiles to its own object in parallel; the per-precision executor translation units
(exec_*.hip) hold the bulk of the kernel instantiations. Each device compilation reports the
resources of every kernel (-Rpass-analysis=kernel-resource-usage): the build fails if any kernel
uses scratch memory or spills registers, so a change that pushes a kernel past its register budget
is caught here rather than on the device. The per-kernel report is written to _build/resources.txt.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfastlbp.so")
BUILD_DIR = os.path.join(HERE, "_build")
SOURCES = ["exec_persistent_f32.hip", "exec_persistent_f64.hip", "exec_levels_f32.hip", "exec_levels_f64.hip",
           "runtime.hip", "alarms.hip", "autotune.hip", "host_graph.cpp", "server.cpp"]

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed fp32 instructions stay off: scalar float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]

_REMARK = re.compile(r"remark:\s+(Function Name|ScratchSize \[bytes/lane\]|VGPRs Spill|SGPRs Spill|VGPRs|"
                     r"Occupancy \[waves/SIMD\]|LDS Size \[bytes/block\]):\s+(\S+)")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> tuple[str, str, int]:
    obj = os.path.join(BUILD_DIR, src + ".o")
    cmd = [hipcc(), *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", os.path.join(CSRC, src),
           "-o", obj]
    if src.endswith(".hip"):
        cmd.insert(1, "-Rpass-analysis=kernel-resource-usage")
    res = subprocess.run(cmd, capture_output=True, text=True)
    return obj, res.stdout + res.stderr, res.returncode


def _kernel_resources(log: str) -> list[dict]:
    """Per-kernel resource records from the remarks of one device compilation."""
    out, cur = [], None
    for m in _REMARK.finditer(log):
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = {"name": val}
            out.append(cur)
        elif cur is not None:
            cur[key] = val
    return out


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1), 16)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_compile, SOURCES))
    errs, report, bad = [], [], []
    for src, (obj, log, rc) in zip(SOURCES, results):
        text = "\n".join(l for l in log.splitlines()
                         if "packed-fp32-ops" not in l and "kernel-resource-usage" not in l
                         and not l.startswith("In file included from") and not re.match(r"\s+\d* \|", l))
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{text}")
        if text.strip():
            errs.append(f"{src}:\n{text}")
        for k in _kernel_resources(log):
            report.append(f"{src}\t{k['name']}\tVGPRs {k.get('VGPRs')}\tscratch {k.get('ScratchSize [bytes/lane]')}\t"
                          f"spill {k.get('VGPRs Spill')}/{k.get('SGPRs Spill')}\toccupancy "
                          f"{k.get('Occupancy [waves/SIMD]')}\tLDS {k.get('LDS Size [bytes/block]')}")
            if k.get("ScratchSize [bytes/lane]", "0") != "0" or k.get("VGPRs Spill", "0") != "0":
                bad.append(report[-1])
    with open(os.path.join(BUILD_DIR, "resources.txt"), "w") as fh:
        fh.write("\n".join(sorted(set(report))) + "\n")
    if bad:
        raise RuntimeError("kernels using scratch memory or spilling registers:\n" + "\n".join(bad))
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", OUT + ".tmp"] + [r[0] for r in results]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    if verbose and errs:
        print("\n".join(errs), file=sys.stderr)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))

"""Build the HIP library (libmce.so) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import glob
import json
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmce.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    "-shared",
    # keep hipcc from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    # per-kernel register / scratch / occupancy report (parsed into RESOURCES)
    "-Rpass-analysis=kernel-resource-usage",
]

# Per-source additions.  The enumeration kernel's search loops branch on
# wave-uniform values only; by default the compiler rewrites every loop into
# structured, predicated control flow, which costs scalar moves and lane-mask
# flag updates on each iteration.  This option leaves regions whose branches
# are all uniform as they are.
SOURCE_FLAGS = {
    "enumerate.hip": ["-mllvm", "-structurizecfg-skip-uniform-regions"],
}

RESOURCES = os.path.join(HERE, "_build", "kernel_resources.json")
_REMARK = re.compile(r"remark:\s+(Function Name|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]|"
                     r"SGPRs Spill|VGPRs Spill|LDS Size \[bytes/block\]):\s+(\S+)")


def parse_resources(text: str) -> dict:
    """Kernel name -> resource figures from the compiler's resource remarks."""
    out, cur = {}, None
    for key, val in _REMARK.findall(text):
        if key == "Function Name":
            cur = out.setdefault(val, {})
        elif cur is not None:
            cur[key.split(" [")[0].lower().replace(" ", "_")] = int(val) if val.isdigit() else val
    return out


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object in parallel, then link libmce.so."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [HIPCC, *[f for f in FLAGS if f != "-shared"], *SOURCE_FLAGS.get(os.path.basename(src), []),
               "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[0][1].wait()
    failed = []
    resources = {}
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        resources.update(parse_resources(text))
        text = "\n".join(ln for ln in text.splitlines()
                         if ("packed-fp32-ops" not in ln and "remark" not in ln and not ln.startswith(" ")) or "error" in ln)
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        for src, text in failed:
            sys.stderr.write(f"---- {src}\n{text}\n")
        raise RuntimeError("hipcc failed for " + ", ".join(os.path.basename(s) for s, _ in failed))
    with open(RESOURCES, "w") as f:
        json.dump(resources, f, indent=1, sort_keys=True)
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build libnbbfrac.so (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled to an object of its own, in parallel
(tiled_inst.hip once per (BATCH, TEAM, EDGE) combination of the tiled step),
then linked into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnbbfrac.so")
OBJDIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("NBB_OFFLOAD_ARCH", "gfx950")

# Packed-FP32 instructions are kept out of the device code on purpose.
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unknown-warning-option"]
NOISE = "is not a recognized feature for this target"


def units():
    """(source, object name, extra flags) of every translation unit."""
    out = [("plan.cpp", "plan.o", []), ("kernels.hip", "kernels.o", []), ("api.hip", "api.o", []),
           ("temporal.hip", "temporal.o", [])]
    for batch in (0, 1):
        for team in (64, 256):
            for edge in (0, 1):
                out.append(("tiled_inst.hip", f"tiled_b{batch}_t{team}_e{edge}.o",
                            [f"-DNBB_INST_BATCH={batch}", f"-DNBB_INST_TEAM={team}", f"-DNBB_INST_EDGE={edge}"]))
    for batch in (0, 1):
        for edge, rule in ((0, 0), (0, 1), (0, 2), (1, 1)):
            out.append(("edges_inst.hip", f"edges_b{batch}_e{edge}_r{rule}.o",
                        [f"-DNBB_INST_BATCH={batch}", f"-DNBB_INST_EDGE={edge}", f"-DNBB_INST_RULE={rule}"]))
    return out


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if NOISE not in l)
    return r.returncode, err


def build(verbose: bool = False, extra=(), jobs: int = 0, out: str = LIB) -> str:
    """Compiles every unit with `extra` flags added and links them into `out`."""
    os.makedirs(OBJDIR, exist_ok=True)
    tag = "%d" % os.getpid()
    cmds = []
    objs = []
    for src, obj, flags in units():
        o = os.path.join(OBJDIR, obj + "." + tag)
        objs.append(o)
        cmds.append(["hipcc", *FLAGS, *extra, *flags, "-c", os.path.join(CSRC, src), "-o", o])
    jobs = jobs or min(len(cmds), os.cpu_count() or 4, 16)
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_run, cmds))
    failed = [(c, e) for c, (rc, e) in zip(cmds, results) if rc != 0]
    if failed:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
        raise RuntimeError("hipcc failed:\n" + "\n\n".join(" ".join(c) + "\n" + e for c, e in failed))
    if verbose:
        for e in (e for _, e in results if e.strip()):
            print(e)
    tmp = out + ".tmp" + tag
    link = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    rc, err = _run(link)
    for o in objs:
        if os.path.exists(o):
            os.remove(o)
    if rc != 0:
        raise RuntimeError("link failed:\n" + err)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build libmess_hip.so for gfx950 with hipcc (in-tree, parallel).

Usage: python -m paper_2406_03121_amd.build [--force] [--jobs N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmess_hip.so")
ROOT = os.path.dirname(HERE)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wno-unused-result",
    "-I" + os.path.join(ROOT, "include"),
]

# unique angular classes (bra pair class >= ket pair class), pair classes
# ss ps pp ds dp dd = 0..5
CLASSES = [(cb, ck) for cb in range(6) for ck in range(cb + 1)]
# classes evaluated by the wave-cooperative kernel (coop.hip) instead
COOP_CLASSES = {(2, 2), (4, 2), (4, 4), (5, 2), (5, 3), (5, 4), (5, 5)}
UNROLLED_CLASSES = [c for c in CLASSES if c not in COOP_CLASSES]
# primitive-lane kernels (plane.hip), one object per class and precision
PLANE_CLASSES = [(5, 4), (5, 3), (5, 2), (5, 1), (4, 4), (4, 2), (2, 2)]
# recursion passes over ket subtrees (fewer live values for the largest;
# measured per build on the 60-atom cluster, one pass -> three (x | y | z)
# -> six (one per second-level ket component): (dd|dp) 8.76 -> 4.52 ->
# 3.27 ms (spill 1.6 KB -> 640 -> 152 B per lane), (dd|ds) at two waves
# 7.07 -> 5.65 -> 5.20 (260 -> 148 B), (dp|dp) 1.56 -> 1.44 -> 1.43,
# (dd|pp) 1.15 -> 1.06 (two passes) -> 1.05)
PLANE_PASSES = {(5, 4): 6, (5, 3): 6, (5, 2): 6, (4, 4): 6, (4, 2): 3}
# waves per SIMD asked of the compiler (default: its own choice, one wave
# with 512 registers here); these run faster at two waves despite their
# spill, with the passes sharing one Boys evaluation (measured on one box,
# 60-atom build / 1024-molecule batch step: (dd|ds) 7.37 -> 4.81 ms;
# (dp|pp) with three passes 1.06 -> 0.64 / 63 -> 37 ms, (dp|dp) 1.44 ->
# 1.15 / 32 -> 23, (dd|pp) 1.02 -> 0.73 / 22 -> 15; (dd|ps) with passes at
# three waves and (pp|pp) with passes were slower)
PLANE_WAVES = {(5, 3): 2, (4, 2): 2, (4, 4): 2, (5, 2): 2}
# the FP32 kernels need half the registers, so more of their waves fit a
# SIMD (measured per 60-atom FP32 build: (dd|ds) 4.22 -> 3.27 ms at three
# waves, (dd|dp) 2.60 -> 1.43 at two, (dp|pp) 0.55 -> 0.41, (dp|dp) 0.80 ->
# 0.71, (dd|pp) 0.54 -> 0.47 at three)
PLANE_WAVES_F32 = {(5, 3): 3, (5, 4): 2, (5, 2): 3, (4, 2): 3, (4, 4): 3}
# kernels whose passes each evaluate the Boys function themselves instead of
# sharing one evaluation through LDS (measured on the same box: sharing takes
# FP64 (dd|ds) 5.07 -> 4.85 ms and FP32 (dd|ds) 3.19 -> 2.81, but FP32
# (dd|dp) 1.44 -> 1.54)
PLANE_NO_SHARE_F32 = {(5, 4)}
# wave-per-primitive-quartet kernels (wave.hip)
WAVE_CLASSES = [(5, 5), (5, 4), (5, 3)]


def _units():
    units = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        name = os.path.splitext(os.path.basename(src))[0]
        if name == "eri_class":
            for cb, ck in UNROLLED_CLASSES:
                units.append((src, os.path.join(OBJ, f"eri_class_{cb}{ck}.o"),
                              [f"-DMESS_CB={cb}", f"-DMESS_CK={ck}"]))
        elif name == "wave":
            for cb, ck in WAVE_CLASSES:
                for real in ("double", "float"):
                    units.append((src, os.path.join(OBJ, f"wave_{cb}{ck}_{real}.o"),
                                  [f"-DMESS_WCB={cb}", f"-DMESS_WCK={ck}", f"-DMESS_WREAL={real}"]))
        elif name == "plane":
            for cb, ck in PLANE_CLASSES:
                for real in ("double", "float"):
                    waves = {**PLANE_WAVES, **PLANE_WAVES_F32} if real == "float" else PLANE_WAVES
                    units.append((src, os.path.join(OBJ, f"plane_{cb}{ck}_{real}.o"),
                                  [f"-DMESS_PCB={cb}", f"-DMESS_PCK={ck}", f"-DMESS_PREAL={real}",
                                   f"-DMESS_PLANE_PASSES={PLANE_PASSES.get((cb, ck), 1)}"] +
                                  ([f"-DMESS_PLANE_WAVES={waves[(cb, ck)]}"] if (cb, ck) in waves else []) +
                                  (["-DMESS_PLANE_SHARE=0"] if real == "float" and (cb, ck) in PLANE_NO_SHARE_F32
                                   else [])))
        else:
            units.append((src, os.path.join(OBJ, name + ".o"), []))
    # heaviest classes first so the parallel build finishes sooner
    def weight(u):
        w = 0
        for d in u[2]:
            if d.startswith("-DMESS_CB=") or d.startswith("-DMESS_CK=") or d.startswith("-DMESS_PC") \
                    or d.startswith("-DMESS_WC"):
                w += int(d.split("=")[1])
        return -w - (10 if "plane" in u[1] else 0)
    units.sort(key=weight)
    return units


def _headers_mtime():
    # this file too: its per-class flags (passes, waves) change the objects
    hs = glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(ROOT, "include", "*.h")) + [__file__]
    return max(os.path.getmtime(h) for h in hs)


def _clean_stale(units):
    keep = {u[1] for u in units}
    for o in glob.glob(os.path.join(OBJ, "*.o")):
        if o not in keep:
            os.remove(o)


def _compile(unit, force):
    src, obj, defs = unit
    if not force and os.path.exists(obj):
        if os.path.getmtime(obj) >= max(os.path.getmtime(src), _headers_mtime()):
            return obj, 0.0, ""
    import time
    t = time.time()
    cmd = [HIPCC] + FLAGS + defs + ["-c", src, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(obj + ".tmp", obj)
    return obj, time.time() - t, r.stderr


def build(force: bool = False, jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    units = _units()
    _clean_stale(units)
    jobs = jobs or min(16, os.cpu_count() or 4)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for obj, dt, _err in ex.map(lambda u: _compile(u, force), units):
            objs.append(obj)
            if verbose and dt:
                print(f"  {os.path.basename(obj)}: {dt:.1f}s", flush=True)
    newest = max(os.path.getmtime(o) for o in objs)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < newest:
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--force", action="store_true")
    ap.add_argument("--jobs", type=int, default=None)
    a = ap.parse_args()
    print(build(force=a.force, jobs=a.jobs, verbose=True))
    sys.exit(0)

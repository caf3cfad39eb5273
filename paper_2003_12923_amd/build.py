"""Build libesmp2.so for gfx950 with hipcc (in-tree, next to this file).

The library is linked from several objects compiled in parallel: the
orchestration and every kernel but the Sylvester products in one translation
unit (csrc/esmp2_all.hip), and one object per instantiation of the Sylvester
kernels (csrc/vv3.hip per (type, tile count), csrc/vv3b.hip per tile count),
which dominate the compile time.  Objects go to _build/ at the repository
root.  build() recompiles every object; build(incremental=True) only those
older than one of their sources.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libesmp2.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]

# (object name, source, extra defines)
UNITS = [("esmp2_all", "esmp2_all.hip", [])]
UNITS += [(f"vv3_{t}_{nt}", "vv3.hip", [f"-DESMP2_VV3_T={t}", f"-DESMP2_VV3_NT={nt}"])
          for t in ("double", "float") for nt in (10, 7, 5)]
UNITS += [(f"vv3b_{nt}", "vv3b.hip", [f"-DESMP2_VV3_NT={nt}"]) for nt in (10, 7, 5)]


def _sources():
    out = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".h"))]
    out += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    return out


def _deps(src):
    """Sources an object depends on: the Sylvester units read only their own
    source and the headers; the main unit reads every source."""
    if src == "esmp2_all.hip":
        return _sources()
    return [p for p in _sources() if p.endswith(".h") or os.path.basename(p) == src]


def _compile(hipcc, unit, incremental, verbose):
    name, src, defs = unit
    obj = os.path.join(OBJ, name + ".o")
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if all(os.path.getmtime(p) <= t for p in _deps(src)):
            return obj, None
    cmd = [hipcc] + HIPCC_FLAGS + defs + ["-c", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
                                          os.path.join(CSRC, src), "-o", obj + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        return obj, r.stdout + r.stderr
    os.replace(obj + ".tmp", obj)
    return obj, None


def build(verbose=False, incremental=False, jobs=None):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or max(1, min(len(UNITS), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as ex:
        res = list(ex.map(lambda u: _compile(hipcc, u, incremental, verbose), UNITS))
    errs = [e for _, e in res if e]
    if errs:
        sys.stderr.write("\n".join(errs))
        raise RuntimeError("hipcc failed building libesmp2.so")
    tmp = LIB + ".tmp"
    # rocBLAS serves the plain strided GEMMs of the set-up (rotations, integral blocks)
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + [o for o, _ in res] + ["-o", tmp, "-lrocblas"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libesmp2.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))

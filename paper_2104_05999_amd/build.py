"""Build the HIP library libdec_hip.so for gfx950 (hipcc, in-tree).

Each source is compiled to its own object with its own flags (the geometry,
crack, topology and boundary sources are compiled without floating-point
contraction so that decisions taken from floating point follow a fixed
operation order), then the objects are linked into one shared library.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libdec_hip.so")

NO_CONTRACT = ["-ffp-contract=off"]
SOURCES = {
    "api.hip": [],
    "topology.hip": NO_CONTRACT,
    "hodge.hip": NO_CONTRACT,
    "assemble.hip": [],
    "bc.hip": NO_CONTRACT,
    "pcg.hip": [],
    "fsai.hip": [],
    "flux.hip": [],
    "serve.hip": [],
    "dual.hip": NO_CONTRACT,
    "tetgen.hip": [],
    "reorder.hip": [],
    "rms.hip": [],
}

COMMON = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src, extra, cc):
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [cc, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    if res.stderr.strip():
        noise = [ln for ln in res.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if noise:
            sys.stderr.write(f"[{src}] " + "\n".join(noise) + "\n")
    return obj


def build(verbose=False):
    """Compile every HIP source for gfx950 and link libdec_hip.so. Returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        futs = [ex.submit(_compile, s, f, cc) for s, f in SOURCES.items()]
        objs = [f.result() for f in futs]
    tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)

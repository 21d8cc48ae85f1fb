"""Build the HIP library ``libcbct.so`` (gfx950) from ``csrc/`` with hipcc.

Every call compiles from source.  Flags: -ffp-contract=off keeps the chord
arithmetic of the forward and back kernels identical operation for operation;
packed FP32 instructions are disabled.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libcbct.so")
SOURCES = ["geom.cpp", "proj.hip", "piccs.hip", "server.cpp", "fdk.hip", "noalloc.hip"]
ARCH = os.environ.get("CBCT_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument", f"-I{INCLUDE}"]


# The projector kernels never see NaN (all plane parameters are finite by
# construction), so min/max need no NaN canonicalisation there.
PER_FILE = {"proj.hip": ["-fno-honor-nans"]}


def _compile(src: str, outdir: str, verbose: bool) -> str:
    obj = os.path.join(outdir, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC, *FLAGS, *PER_FILE.get(src, []), *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


SIM_LIB = os.path.join(HERE, "libcbct_sim.so")


def build_sim(verbose: bool = False) -> str:
    """Host-only library driving the server's scheduling core with a simulated
    device (tests of admission and residency without a GPU)."""
    tmp = SIM_LIB + ".tmp"
    cmd = [os.environ.get("CXX", "g++"), "-O2", "-std=c++17", "-fPIC", "-shared", "-Wall",
           f"-I{INCLUDE}", os.path.join(CSRC, "serve_sim.cpp"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SIM_LIB)
    return SIM_LIB


PROBE = os.path.join(HERE, "valu_probe")


def build_probe(verbose: bool = False) -> str:
    """The VALU issue-rate probe (a measurement helper of bench.py's roofline,
    not part of the library)."""
    tmp = PROBE + ".tmp"
    cmd = [HIPCC, *FLAGS, "-x", "hip", os.path.join(CSRC, "valu_probe.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for valu_probe.hip:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, PROBE)
    return PROBE


def build(verbose: bool = False) -> str:
    outdir = os.path.join(HERE, "_build")
    os.makedirs(outdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, outdir, verbose), SOURCES))
    tmp = LIB + ".tmp"
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    # roctx marker ranges (solver iterations, served requests)
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, f"-L{rocm_lib}",
           f"-Wl,-rpath,{rocm_lib}", "-lrocprofiler-sdk-roctx", "-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    build_sim(verbose)
    build_probe(verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build the HIP library libfamsa_lcs.so for gfx950 (in-tree).

    python -m paper_1603_06958_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfamsa_lcs.so")
SOURCES = ["lcs_kernels.hip", "mst.hip", "gapped.hip", "peak.hip", "noalloc.hip", "profile_dp.hip", "runtime.cpp", "plan.cpp", "autotune.cpp", "slink.cpp", "server.cpp", "guide_tree.cpp"]
ARCH = os.environ.get("FAMSA_LCS_ARCH", "gfx950")


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str, objdir: str, common, verbose: bool) -> str:
    path = os.path.join(CSRC, src)
    if not os.path.exists(path):
        raise RuntimeError("missing source: " + path)
    obj = os.path.join(objdir, src + ".o")
    cmd = [hipcc(), "-c", path, "-o", obj] + common + ["--offload-arch=" + ARCH]
    if src.endswith(".hip"):  # device code: HIP for gfx950
        cmd += ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("compile failed: " + src)
    return obj


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (in parallel) and link the shared library; returns its path."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
              "-I" + os.path.join(HERE, "..", "include")]
    jobs = jobs or min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, objdir, common, verbose), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-o", tmp] + objs + ["--offload-arch=" + ARCH]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

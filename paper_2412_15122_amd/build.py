"""Build the HIP library (gfx950) in-tree: paper_2412_15122_amd/libapsp.so.

hipcc compiles every csrc/*.hip file for gfx950 only (one object per file,
in parallel, under _build/) and links them into one shared library exporting
the C ABI of include/apsp.h.
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libapsp.so")
OBJ_DIR = os.path.join(ROOT, "_build")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    jobs = []
    for src in sources():
        obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
        jobs.append((obj, [hipcc, *FLAGS, *inc, "-c", src, "-o", obj]))

    def run(job):
        obj, cmd = job
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        return obj, r.returncode, r.stdout

    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(run, jobs))
    failed = [(o, out) for o, rc, out in results if rc != 0]
    for o, rc, out in results:
        text = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
        if text.strip() and (verbose or rc != 0):
            print(text, file=sys.stderr)
    if failed:
        raise subprocess.CalledProcessError(1, f"hipcc ({', '.join(os.path.basename(o) for o, _ in failed)})")
    tmp = LIB + ".tmp"
    link = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *[o for o, _, _ in results], "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)

"""Build libfmt.so (HIP kernels + host runtime + C ABI) for gfx950.

Usage: python -m paper_1511_01353_amd.csrc.build   (or call build()).
Every call recompiles.  Objects go to a scratch folder; the shared library is
written next to the Python package, where the binding loads it.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
SOURCES = ["k_sort.hip", "k_gram.hip", "k_moments.hip", "k_pyramid.hip", "k_level.hip", "k_solve_reg.hip", "k_eval.hip", "k_wide.hip",
           "k_rbf.hip", "fmt_host.hip"]
# (source, extra flags, object): the moment kernels of each large order are
# compiled in an object of their own, in parallel with the rest
VARIANTS = [("k_moments.hip", [f"-DFMT_MOMENTS_WIDE_P={p}"], f"k_moments_p{p}.o") for p in (10, 12, 14)]
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed-FP32 VALU forms stay off: scalar float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]
LIB_NAME = "libfmt.so"


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; ROCm is required to build the library")
    return path


def _compile(src: str, obj: str, extra=()) -> str:
    cmd = [hipcc(), *FLAGS, *extra, "-c", os.path.join(HERE, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    out = os.path.join(PKG, LIB_NAME)
    with tempfile.TemporaryDirectory(prefix="fmt_build_") as tmp:
        jobs = [(s, os.path.join(tmp, s.replace(".hip", ".o")), []) for s in SOURCES]
        jobs += [(s, os.path.join(tmp, o), f) for s, f, o in VARIANTS]
        # the slowest objects first, so they overlap the rest
        jobs.sort(key=lambda j: 0 if ("moments" in j[0] or "level" in j[0] or "eval" in j[0]) else 1)
        objs = [j[1] for j in jobs]
        with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
            list(ex.map(lambda j: _compile(*j), jobs))
        tmp_lib = os.path.join(tmp, LIB_NAME)
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp_lib, *objs]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        shutil.move(tmp_lib, out + ".tmp")
        os.replace(out + ".tmp", out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

"""Build libmanyclaw.so (all HIP sources under csrc/) for gfx950 with hipcc.

Run as ``python -m paper_1308_1464_amd.build`` or through
``__graft_entry__.build()``.  The library is written next to this file.
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmanyclaw.so")
ROOT = os.path.dirname(HERE)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no implicit multiply-add contraction: the kernels write fma() where they
    # want one, so results are bitwise independent of unrolling and tiling
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose: bool = False, extra=None) -> str:
    """Compile every source to an object (in parallel, one hipcc per file),
    then link the shared library."""
    import concurrent.futures
    import tempfile
    srcs = sources()
    inc = ["-I", os.path.join(ROOT, "include")]
    cflags = [f for f in FLAGS if f != "-shared"] + list(extra or [])
    with tempfile.TemporaryDirectory(prefix="mcbuild") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in srcs]
        cmds = [[HIPCC] + cflags + inc + ["-c", s, "-o", o] for s, o in zip(srcs, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        jobs = min(len(cmds), int(os.environ.get("MAX_JOBS", "8")) or 1)
        with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
            for r in ex.map(lambda c: subprocess.run(c, cwd=HERE), cmds):
                if r.returncode != 0:
                    raise subprocess.CalledProcessError(r.returncode, r.args)
        tmp = LIB + ".tmp"
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True, cwd=HERE)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])

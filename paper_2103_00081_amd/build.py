"""Build libhts.so (HIP for gfx950) in-tree with hipcc.

Every ``csrc/*.hip`` translation unit is compiled to an object file under
``paper_2103_00081_amd/_build`` and linked into
``paper_2103_00081_amd/libhts.so``.
"""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhts.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("HTS_ARCH", "gfx950")

CFLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I" + os.path.join(os.path.dirname(HERE), "include"),
]


def _torch_hip_runtime():
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec is None or spec.origin is None:
            return None
        p = os.path.join(os.path.dirname(spec.origin), "lib", "libamdhip64.so")
        return p if os.path.exists(p) else None
    except Exception:
        return None


def _compile(src: str) -> str:
    obj = os.path.join(OUT, os.path.basename(src) + ".o")
    cmd = [HIPCC] + CFLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    msgs = [ln for ln in r.stdout.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, "\n".join(msgs)))
    return obj


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(OUT, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(SRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    # One HIP runtime per process: link the runtime that PyTorch loads (it
    # carries no SONAME, so a second copy would otherwise be mapped).
    # A symlink _rt/libamdhip64.so.7 -> torch's runtime lets the library's
    # RUNPATH resolve the runtime's SONAME to the same file (same inode)
    # whichever of the two is loaded first.
    rt = _torch_hip_runtime()
    if rt:
        rtdir = os.path.join(HERE, "_rt")
        os.makedirs(rtdir, exist_ok=True)
        link = os.path.join(rtdir, "libamdhip64.so.7")
        if os.path.lexists(link):
            os.remove(link)
        os.symlink(rt, link)
        cmd = ["g++", "-shared", "-fPIC", "-o", tmp] + objs + [
            "-L" + rtdir, "-l:libamdhip64.so.7", "-Wl,-rpath,$ORIGIN/_rt",
            "-Wl,--no-undefined", "-lstdc++", "-lm"]
    else:
        cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, file=sys.stderr)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

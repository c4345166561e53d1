"""Build libstaggermhd.so (the C ABI of include/mhd.h) for gfx950 with hipcc.

Usage:  python -m paper_2405_02483_amd.csrc.build   (or call build())

Every HIP source in this directory is compiled to an object under
``paper_2405_02483_amd/_build`` in parallel, then linked into
``paper_2405_02483_amd/libstaggermhd.so``.  Always recompiles.
"""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libstaggermhd.so")
ARCH = "gfx950"

CFLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    # multiply-adds are fused per source expression (not across statements
    # at the backend's choice), so every template instantiation rounds the
    # same way and all tile shapes agree bit for bit
    "-ffp-contract=on",
    # packed fp32 instructions stay off (compiler-generated only, never by hand)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + HERE,
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def _compile(src, obj):
    cmd = [_hipcc()] + CFLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, out))
    return out


def build(verbose=False):
    bdir = os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(HERE, "*.hip")))
    objs = [os.path.join(bdir, os.path.basename(s)[:-4] + ".o") for s in srcs]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        logs = list(ex.map(_compile, srcs, objs))
    if verbose:
        for s, l in zip(srcs, logs):
            if l.strip():
                print(os.path.basename(s), l)
    tmp = LIB + ".tmp"
    # rocFFT (div B cleaning) from the ROCm installation
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    cmd = ([_hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs +
           ["-L" + rocm_lib, "-Wl,-rpath," + rocm_lib, "-lrocfft"])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Build libpfspec.so (HIP, gfx950) in-tree.

    python -m paper_2306_04322_amd.build [-j N]

Every source under csrc/ is compiled with hipcc for gfx950 into _build/ at
the repository root and linked into paper_2306_04322_amd/libpfspec.so.
Packed FP32 instructions are disabled for every device compilation.
"""

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libpfspec.so")

SOURCES = ["pfspec.hip", "k_row_f32.hip", "k_row_f64.hip", "k_col_f32.hip", "k_col_f64.hip",
           "k_reduce.hip", "k_fd.hip", "k_adj_f32.hip", "k_adj_f64.hip"]

ARCH = "gfx950"
CFLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-fno-gpu-rdc",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"), "-Wno-unused-result"]


# The files the FP32 FS row and column kernels are compiled from.
FS_F32_KERNEL_SOURCES = ["pf_fe.h", "pf_fft.h", "pf_kernels.h", "pf_launch.h",
                         "k_row.inc", "k_row_f32.hip", "k_col.inc", "k_col_f32.hip"]


def source_digest(names=None):
    """sha256 over the named HIP sources (default: every source and header) and
    the compile flags other than include paths (which name the checkout's
    location); identifies the build of the kernels they define."""
    import hashlib
    h = hashlib.sha256(" ".join(f for f in CFLAGS if not f.startswith("-I")).encode())
    if names is None:
        names = [n for n in os.listdir(CSRC) if n.endswith((".hip", ".h", ".inc"))]
    for name in sorted(names):
        h.update(name.encode())
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def fs_kernel_digest():
    """Digest of the FP32 FS row and column kernels alone: counter figures
    taken on them stay valid while other kernels change."""
    return source_digest(FS_F32_KERNEL_SOURCES)


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src, defines=(), build_dir=BUILD):
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + CFLAGS + ["-D" + d for d in defines] + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(jobs=None, verbose=True, defines=(), out=None):
    """Compile and link.  `defines` (NAME=VALUE strings) override the kernel
    tuning parameters; `out` writes the library elsewhere (tuning sweeps)."""
    lib = out or LIB
    build_dir = BUILD if not defines else os.path.join(BUILD, "variant_" + "_".join(defines).replace("=", ""))
    os.makedirs(build_dir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(len(srcs), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, defines, build_dir), srcs))
    tmp = lib + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    if out is None:
        build_example(verbose)
    return lib


EXAMPLE_SRC = os.path.join(PKG, "examples", "fs_example.cpp")
EXAMPLE_BIN = os.path.join(PKG, "examples", "fs_example")


def build_example(verbose=True):
    """The C-ABI example program (host code only), linked against the
    in-tree library and finding it at run time next to itself."""
    cmd = [hipcc(), "-O2", "-std=c++17", "-I" + os.path.join(ROOT, "include"), EXAMPLE_SRC,
           "-L" + PKG, "-lpfspec", "-Wl,-rpath,$ORIGIN/..", "-o", EXAMPLE_BIN]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("example build failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    if verbose:
        print("built", EXAMPLE_BIN)
    return EXAMPLE_BIN


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("-D", dest="defines", action="append", default=[],
                    help="override a kernel tuning parameter, e.g. -D PF_COL_CB_LONG_F32=8")
    ap.add_argument("-o", dest="out", default=None, help="output library path")
    args = ap.parse_args(argv)
    build(args.j, defines=args.defines, out=args.out)


if __name__ == "__main__":
    sys.exit(main())

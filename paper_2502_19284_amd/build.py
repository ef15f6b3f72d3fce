"""Build libspx.so (HIP for gfx950) in-tree: one hipcc compile per source, then one link.

    python -m paper_2502_19284_amd.build          # or build() from Python
"""
import concurrent.futures
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libspx.so")
SOURCES = ["spx_api.cpp", "spx_prof.cpp", "spx_noalloc.cpp", "spx_serve.cpp", "spx_batch.cpp",
           "k_convert.hip", "k_partition.hip", "k_spmv.hip", "k_spmv_crs.hip", "k_spmm.hip",
           "k_hot.hip", "k_serve.hip", "k_batch.hip", "k_bcoh.hip", "k_probe.hip"]
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def _compile(src, out_dir=OUT_DIR, extra=()):
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + list(extra) + ["-I", os.path.join(PKG, "..", "include"), "-c",
                                           os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    warnings = [l for l in r.stderr.splitlines()
                if "warning" in l and "packed-fp32-ops" not in l]
    return obj, warnings


def build(verbose=False, lib=LIB, extra_flags=()):
    """Compile every source for gfx950 and link `lib` (always rebuilds).  extra_flags are added
    to every compile and to the link (e.g. host-only sanitizer flags for a checking build)."""
    out_dir = OUT_DIR if lib == LIB else os.path.join(os.path.dirname(lib), "_build_" +
                                                      os.path.basename(lib))
    os.makedirs(out_dir, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(lambda src: _compile(src, out_dir, extra_flags), SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for _, w in results:
            for line in w:
                print(line, file=sys.stderr)
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH] + list(extra_flags) + \
        ["-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))

"""Build libsht.so (all HIP sources for gfx950) in-tree.

    python -m paper_2507_12144_amd.build        # or build() from Python
    python -m paper_2507_12144_amd.build debug  # the race-check library
    python -m paper_2507_12144_amd.build release debug asan   # all three
    python -m paper_2507_12144_amd.build asan   # host-sanitizer test build

Every source is compiled with hipcc for --offload-arch=gfx950 with packed
float32 instructions disabled, then linked into the package directory.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libsht.so")
BUILD_DIR = os.path.join(os.path.dirname(PKG), "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    """The HIP sources, the slowest to compile first (the three-plane bf16
    kernels, the float32 contraction per NCB, then the other bf16 plane
    counts), so that the parallel build ends soonest."""
    names = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    heavy = ("_np3_", "_ncb", "_np2_", "_np1_")
    order = lambda f: (next((i for i, h in enumerate(heavy) if h in f), len(heavy)), f)
    return [os.path.join(CSRC, f) for f in sorted(names, key=order)]


# Library variants: the release library and the race-check build (every
# barrier drains all memory counters, every Legendre stage ends with a drain
# and a barrier; see kernel_common.h), whose results must equal the
# release library's bit for bit.
VARIANTS = {
    "release": (OUT, BUILD_DIR, []),
    "debug": (os.path.join(PKG, "libsht_debug.so"), os.path.join(BUILD_DIR, "debug"), ["-DSHT_DEBUG_BARRIERS=1"]),
}


def _compile(src, build_dir, extra):
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + extra + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns that it does not know the packed-fp32 feature
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    return obj, err


def build(verbose=False, variant="release", variants=None):
    """Compile every source for each library variant named (``variants``, or
    the one ``variant``) and link each; the compile jobs of all of them share
    one pool, slowest first.  Returns the path of the last library."""
    names = list(variants or [variant])
    jobs = []
    for src in sources():
        for v in names:
            out, build_dir, extra = VARIANTS[v]
            os.makedirs(build_dir, exist_ok=True)
            jobs.append((v, src, build_dir, extra))
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        results = list(ex.map(lambda j: (j[0],) + _compile(j[1], j[2], j[3]), jobs))
    for _, obj, err in results:
        if verbose and err.strip():
            print(err, file=sys.stderr)
    for v in names:
        out = VARIANTS[v][0]
        tmp = out + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for w, o, _ in results if w == v]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed ({v}):\n{r.stderr}")
        os.replace(tmp, out)
    return out


ROOT = os.path.dirname(PKG)
ASAN_DIR = os.path.join(ROOT, "tests", "asan")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build_host_asan():
    """Host-sanitizer test build in tests/asan: the library's host logic
    (api.hip) compiled with AddressSanitizer on the host pass only (device
    code unchanged), linked with the release objects of the other sources
    (run build() first) into libsht_asan.so, and the C driver abi_driver.c
    built against it.  The sanitizer is never applied to GPU code."""
    out_dir = os.path.join(BUILD_DIR, "asan")
    os.makedirs(out_dir, exist_ok=True)
    api = os.path.join(CSRC, "api.hip")
    others = [os.path.join(BUILD_DIR, os.path.basename(s) + ".o") for s in sources() if s != api]
    missing = [o for o in others if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"release objects missing ({os.path.basename(missing[0])}): run build() first")
    obj = os.path.join(out_dir, "api.hip.o")
    host_asan = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    r = subprocess.run([HIPCC] + FLAGS + host_asan + ["-c", api, "-o", obj], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc (host sanitizer) failed:\n{r.stderr}")
    clangxx = os.path.join(ROCM, "llvm", "bin", "clang++")
    clang = os.path.join(ROCM, "llvm", "bin", "clang")
    lib = os.path.join(ASAN_DIR, "libsht_asan.so")
    link = [clangxx, "-shared", "-fPIC", "-fsanitize=address", "-o", lib, obj] + others + [
        "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link (host sanitizer) failed:\n{r.stderr}")
    drv = os.path.join(ASAN_DIR, "abi_driver")
    cc = [clang, "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
          "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROCM, "include"),
          "-o", drv, os.path.join(ASAN_DIR, "abi_driver.c"), "-L" + ASAN_DIR, "-lsht_asan",
          "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath,$ORIGIN",
          "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cc, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"driver build (host sanitizer) failed:\n{r.stderr}")
    return drv


if __name__ == "__main__":
    args = sys.argv[1:] or ["release"]
    libs = [v for v in args if v != "asan"]
    if libs:
        print(build(verbose=True, variants=libs))
    if "asan" in args:
        print(build_host_asan())

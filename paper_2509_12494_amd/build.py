"""Compile the HIP library libmwntt.so for gfx950 (in-tree, next to this file).

    python -m paper_2509_12494_amd.build [-v]

Each source is compiled to an object under _build/ (in parallel), then linked
with hipcc into paper_2509_12494_amd/libmwntt.so.  The binding's direct-call
shim (csrc/mw_pycall.c, argument marshalling only) is compiled with the host C
compiler into paper_2509_12494_amd/_mwcall<suffix>.so.  Always recompiles.
"""
import concurrent.futures
import os
import subprocess
import sys
import sysconfig

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libmwntt.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["mw_ntt_w8_fwd.hip", "mw_ntt_w8_inv.hip", "mw_ntt_w4_fwd.hip", "mw_ntt_w4_inv.hip",
           "mw_ntt_w2_fwd.hip", "mw_ntt_w2_inv.hip", "mw_ntt_ablation.hip",
           "mw_exec.hip", "mw_resident.hip", "mw_blas.hip", "mw_ntt.hip", "mw_serve.hip", "mw_validate.hip",
           "mw_capi.cpp"]
# Sources whose kernels are scheduled for instruction-level parallelism: the
# multi-word carry chains otherwise serialize on VCC with hazard wait states.
ILP_SOURCES = {"mw_ntt_w8_fwd.hip", "mw_ntt_w8_inv.hip", "mw_ntt_w4_fwd.hip", "mw_ntt_w4_inv.hip",
               "mw_ntt_w2_fwd.hip", "mw_ntt_w2_inv.hip", "mw_ntt_ablation.hip", "mw_exec.hip", "mw_resident.hip"}
ILP_FLAGS = ["-mllvm", "-amdgpu-sched-strategy=max-ilp", "-DMWNTT_MIN_WAVES_PER_EU=3"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include")]
# device-code flags: every HIP source goes through hipcc for gfx950
HIP_FLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


# Host-only sanitizer instrumentation (device code untouched): the flags go to
# the host pass of every compile and to the link.
SANITIZE = {
    "address": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"],
    "undefined": ["-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined"],
}


def _compile(src, verbose, build_dir=BUILD_DIR, san=()):
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    extra = ILP_FLAGS if src in ILP_SOURCES else []
    cmd = [HIPCC] + COMMON + HIP_FLAGS + extra + list(san) + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the device-only feature flag; drop that note
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    if verbose and err.strip():
        print(err)
    return obj


PYCALL = os.path.join(HERE, "_mwcall" + sysconfig.get_config_var("EXT_SUFFIX"))


def build_pycall(verbose: bool = False) -> str:
    """The binding's direct-call shim (a CPython extension, no device code)."""
    tmp = PYCALL + ".tmp"
    cmd = ["gcc", "-O2", "-shared", "-fPIC", "-Wall", "-I" + sysconfig.get_paths()["include"],
           os.path.join(CSRC, "mw_pycall.c"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("mw_pycall.c failed:\n" + r.stderr)
    os.replace(tmp, PYCALL)
    return PYCALL


def build(verbose: bool = False, sanitize: str = "") -> str:
    """Builds the library; with sanitize ("address" or "undefined") a
    host-instrumented copy under _build/sanitize-<kind>/ instead, for running
    the host code's tests with the sanitizer runtime preloaded (the library
    is then selected with MWNTT_LIB)."""
    san = SANITIZE[sanitize] if sanitize else []
    build_dir = os.path.join(BUILD_DIR, "sanitize-" + sanitize) if sanitize else BUILD_DIR
    out = os.path.join(build_dir, "libmwntt.so") if sanitize else LIB
    os.makedirs(build_dir, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, build_dir, san), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + san + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, out)
    if not sanitize:
        build_pycall(verbose)
    return out


if __name__ == "__main__":
    kind = sys.argv[sys.argv.index("--sanitize") + 1] if "--sanitize" in sys.argv else ""
    print(build(verbose="-v" in sys.argv, sanitize=kind))

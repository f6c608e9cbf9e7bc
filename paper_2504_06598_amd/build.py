"""Compile libsrt.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libsrt.so")

SOURCES = ["build.hip", "trace.hip", "backward.hip", "batched.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# -ffp-contract=off: the canonical FP32 ray constructions (camera, secondary
# rays) must be single rounded operations; the hot FP64 arithmetic spells out
# its fused multiply-adds explicitly.
# -packed-fp32-ops: no packed FP32 VALU instructions are generated.
CFLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics", "-Wall", "-Wno-unused-result", f"-I{INCLUDE}", f"-I{CSRC}"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs,
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libsrt.so failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_host_sanitized(out_dir: str) -> str:
    """The host code of libsrt (argument validation, workspace arithmetic, the
    block cache, the memory limit) compiled with AddressSanitizer and
    UndefinedBehaviorSanitizer and without device code, for CPU tests: no
    kernel exists in it, so only calls that return before launching anything
    may be made. Load it with clang's ASan runtime preloaded. Returns its path."""
    os.makedirs(out_dir, exist_ok=True)
    flags = ["--offload-host-only", "-x", "hip", "-O1", "-g", "-fPIC", "-std=c++17",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
             "-fno-omit-frame-pointer", f"-I{INCLUDE}", f"-I{CSRC}"]

    def one(src):
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".host.o")
        r = subprocess.run([HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"host-only sanitizer compile failed on {src}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(one, SOURCES))
    # each object's module constructor registers its device-code bundle; a
    # host-only compile leaves that symbol undefined, so give it an empty
    # offload bundle (no code objects: nothing can be launched)
    names = set()
    for o in objs:
        out = subprocess.run(["nm", "-u", o], capture_output=True, text=True, check=True).stdout
        names.update(w for w in out.split() if w.startswith("__hip_fatbin_"))
    stub_c = os.path.join(out_dir, "empty_bundles.c")
    with open(stub_c, "w") as fh:
        for n in sorted(names):
            fh.write(f'__attribute__((aligned(4096))) const char {n}[4096] = '
                     f'"__CLANG_OFFLOAD_BUNDLE__";\n')
    stub_o = os.path.join(out_dir, "empty_bundles.o")
    subprocess.run(["gcc", "-c", "-fPIC", stub_c, "-o", stub_o], check=True)
    objs.append(stub_o)
    lib = os.path.join(out_dir, "libsrt_host_asan.so")
    clangxx = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin",
                           "clang++")
    if not os.path.exists(clangxx):
        clangxx = "/opt/rocm/llvm/bin/clang++"
    r = subprocess.run([clangxx, "-shared", "-fPIC", "-fsanitize=address,undefined",
                        "-shared-libsan", "-o", lib, *objs, "-L/opt/rocm/lib", "-lamdhip64",
                        "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of the sanitized host library failed")
    return lib


def asan_runtime() -> str:
    """clang's shared ASan runtime (to preload for build_host_sanitized's library)."""
    import glob
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise RuntimeError("clang ASan runtime not found")
    return found[-1]


if __name__ == "__main__":
    build(verbose=True)

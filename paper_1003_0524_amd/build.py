"""Build the gfx950 shared libraries in-tree with hipcc.

    python -m paper_1003_0524_amd.build          # libexchange.so (+ synth/libsynth.so)

The packed-FP32 target feature is switched off for all device code: the
compiler otherwise forms v_pk_* FP32 instructions from ordinary float code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ARCH = os.environ.get("EXC_OFFLOAD_ARCH", "gfx950")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

COMMON = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-result", "-Wno-unused-value", "-I" + os.path.join(ROOT, "include")]

TARGETS = [
    (os.path.join(HERE, "csrc", "exchange.hip"), os.path.join(HERE, "libexchange.so")),
    (os.path.join(ROOT, "synth", "csrc", "synth.hip"), os.path.join(ROOT, "synth", "libsynth.so")),
]


def build(verbose: bool = False, only=None) -> None:
    for src, out in TARGETS:
        if only and os.path.basename(out) not in only:
            continue
        if not os.path.exists(src):
            continue
        tmp = out + ".tmp"
        cmd = [HIPCC, *COMMON, src, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        errs = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l]
        if r.returncode != 0:
            sys.stderr.write("\n".join(errs) + "\n")
            raise RuntimeError(f"hipcc failed for {src}")
        if verbose and errs:
            sys.stderr.write("\n".join(errs) + "\n")
        os.replace(tmp, out)


ASAN_LIB = os.path.join(HERE, "libexchange_asan.so")


def asan_runtime() -> str:
    """The compiler's AddressSanitizer runtime (to preload into a host process)."""
    import glob
    root = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    hits = sorted(glob.glob(os.path.join(root, "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")) +
                  glob.glob(os.path.join(root, "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise RuntimeError("no libclang_rt.asan-x86_64.so next to hipcc")
    return hits[-1]


def build_asan(out: str = ASAN_LIB) -> str:
    """The exchange library with its host code under AddressSanitizer (device code as usual),
    for running the ABI's argument checks under the sanitizer on a machine without a GPU."""
    src = os.path.join(HERE, "csrc", "exchange.hip")
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-result", "-Wno-unused-value", "-I" + os.path.join(ROOT, "include"), src, "-o", out + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError("hipcc failed for the sanitizer build")
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    if sys.argv[1:] == ["--asan"]:
        print(build_asan())
    else:
        build(verbose=True, only=sys.argv[1:] or None)

"""Build the HIP library ``libfth.so`` in-tree for gfx950.

Every translation unit under ``csrc/`` is compiled by hipcc into
``_build/`` (in parallel) and linked into ``paper_1402_2095_amd/libfth.so``.

Device code is compiled with FP contraction off (every fused multiply-add
in the kernels is written explicitly) and without packed-FP32 instructions.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libfth.so")
ARCH = os.environ.get("FTH_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-fPIC", "-std=c++17", "-ffp-contract=off", "-Wall", "-Wno-unused-function"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _deps_mtime(path: str, seen=None) -> float:
    """Newest modification time of a source and the local headers it
    includes (quoted includes, followed recursively)."""
    import re
    seen = set() if seen is None else seen
    if path in seen or not os.path.exists(path):
        return 0.0
    seen.add(path)
    t = os.path.getmtime(path)
    with open(path) as fh:
        for inc in re.findall(r'^\s*#\s*include\s+"([^"]+)"', fh.read(), re.M):
            t = max(t, _deps_mtime(os.path.normpath(os.path.join(os.path.dirname(path), inc)), seen))
    return t


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj) and os.path.getmtime(obj) > _deps_mtime(src):
        return obj
    cmd = [hipcc(), *COMMON, *DEVICE, "-I", CSRC, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [hipcc(), *COMMON, "-x", "hip", *DEVICE, "-I", CSRC, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def build(verbose: bool = True, jobs: int | None = None, incremental: bool = False) -> str:
    """Compile every source (incremental=True skips objects newer than their
    source and every header) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)), 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, incremental), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources", flush=True)
    return LIB


# Host translation units (no kernels): the part a CPU sanitizer build covers.
HOST_SOURCES = ["fth_api.cpp", "fth_linalg.cpp", "fth_scale.cpp", "fth_server.cpp", "noalloc.hip"]
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_sanitized(out: str) -> str:
    """A copy of the library whose host code is built with AddressSanitizer
    and UndefinedBehaviorSanitizer (device code as in the normal build; the
    sanitizers apply to the host side only).  Load it with the compiler's
    shared ASan runtime preloaded."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in sources():
        base = os.path.basename(src)
        if base in HOST_SOURCES:
            obj = os.path.join(os.path.dirname(out), base + ".san.o")
            cmd = [hipcc(), *COMMON, "-g", "-x", "hip", *DEVICE, *SANITIZE, "-I", CSRC, "-c", src, "-o", obj]
            res = subprocess.run(cmd, capture_output=True, text=True)
            if res.returncode != 0:
                raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
            objs.append(obj)
        else:
            objs.append(_compile(src, incremental=True))
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *SANITIZE, "-Xarch_host", "-shared-libasan",
           *objs, "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return out


def asan_runtime() -> str:
    """The shared ASan runtime of the compiler that builds the library."""
    res = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = res.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        import glob
        cands = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        path = cands[0] if cands else ""
    return path


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv)
    sys.exit(0)

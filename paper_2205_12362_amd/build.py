"""Compile libarts.so (HIP for gfx950 + host C++) in place, next to this file.

    python -m paper_2205_12362_amd.build        # or __graft_entry__.build()

Every call recompiles.  Objects go to _build/ inside the package (git-ignored)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libarts.so")
ARCH = os.environ.get("ARTS_OFFLOAD_ARCH", "gfx950")

# Packed-FP32 instructions are disabled for all device code (some of their forms have been
# unreliable on this hardware); hipcc's host pass warns that it does not know the feature.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          f"-I{os.path.join(PKG, '..', 'include')}"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; install ROCm or set HIPCC")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    return out


def sources():
    srcs = sorted(os.listdir(CSRC))
    return ([os.path.join(CSRC, s) for s in srcs if s.endswith(".hip")],
            [os.path.join(CSRC, s) for s in srcs if s.endswith(".cpp")])


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    hip_srcs, cpp_srcs = sources()
    jobs = []
    for src in hip_srcs:
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        jobs.append([hipcc, "-c", "-x", "hip", f"--offload-arch={ARCH}", *COMMON, *DEVICE_FLAGS,
                     src, "-o", obj])
    for src in cpp_srcs:
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        # host-only C++ (no device pass)
        rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
        jobs.append([hipcc, "-c", "-x", "c++", *COMMON, "-D__HIP_PLATFORM_AMD__",
                     f"-I{rocm}/include", src, "-o", obj])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    objs = [j[-1] for j in jobs]
    tmp = LIB + ".tmp"
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    _run([hipcc, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp,
          "-Wl,-soname,libarts.so", f"-L{rocm}/lib", "-lrocprofiler-sdk-roctx",
          f"-Wl,-rpath,{rocm}/lib"])
    os.replace(tmp, LIB)
    return LIB


def build_sanitized_host(driver_src: str, out_exe: str) -> str:
    """A CPU executable of `driver_src` linked with the library's host code built under
    AddressSanitizer and UndefinedBehaviorSanitizer (the .cpp host sources recompiled with the
    sanitizers; the .hip objects of the normal build, whose device code is never run on the
    CPU, linked as they are).  Used by the CPU test suite."""
    hipcc = _hipcc()
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    hip_srcs, cpp_srcs = sources()
    hip_objs = [os.path.join(BUILD, os.path.basename(x) + ".o") for x in hip_srcs]
    if not all(os.path.exists(o) for o in hip_objs):
        build()
    work = os.path.dirname(os.path.abspath(out_exe))
    san = ["-g", "-O1", "-fno-omit-frame-pointer"]
    jobs = []
    for src in cpp_srcs:
        obj = os.path.join(work, os.path.basename(src) + ".asan.o")
        # host-only compilation (-x c++): the sanitizers instrument host code only
        jobs.append([hipcc, "-c", "-x", "c++", *COMMON, *san, "-Xarch_host", "-fsanitize=address",
                     "-Xarch_host", "-fsanitize=undefined", "-D__HIP_PLATFORM_AMD__",
                     f"-I{rocm}/include", src, "-o", obj])
    # the driver and the link use ROCm's host clang (the sanitizer runtimes must match the
    # compiler that instrumented the objects)
    clang = os.path.join(rocm, "llvm", "bin", "clang++")
    drv_obj = os.path.join(work, "driver.asan.o")
    jobs.append([clang, "-c", "-std=c++17", *san, "-fsanitize=address,undefined",
                 f"-I{os.path.join(PKG, '..', 'include')}", driver_src, "-o", drv_obj])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        list(ex.map(_run, jobs))
    objs = [j[-1] for j in jobs]
    _run([clang, "-fsanitize=address,undefined", *objs, *hip_objs, f"-L{rocm}/lib",
          "-lamdhip64", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{rocm}/lib", "-o", out_exe])
    return out_exe


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

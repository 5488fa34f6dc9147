"""Build libspnet.so in-tree: host C++ with g++ (-ffp-contract=off, so the
floating-point steps that decide the network structure round exactly as
written) and the gfx950 kernels with hipcc, linked by hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libspnet.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HOST_SOURCES = ["network.cpp", "assemble.cpp", "spaces.cpp", "factor.cpp", "diagnostics.cpp", "api.cpp", "serve.cpp"]
DEVICE_SOURCES = ["device.hip"]
# the star kernel launcher, once per factor precision and column count
STAR_VARIANTS = [(t, kc) for t in ("float", "double") for kc in (1, 2, 4, 8, 16)]

HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function", "-pthread"]
DEVICE_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops", "-ffp-contract=off", "-Wno-unused-result"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[0]} {cmd[-1]}")
    return r


def _stale(obj, src):
    """obj is missing or older than its source or any header of csrc/ or include/."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    hdrs = ["internal.hpp"]
    if src.endswith(".cpp"):
        hdrs.append("handles.hpp")
    else:
        hdrs.append("device_common.hpp")
    if src.endswith("star_inst.hip"):
        hdrs += ["star_band.hpp", "star_sn.hpp"]
    deps = [src] + [os.path.join(CSRC, h) for h in hdrs]
    deps.append(os.path.join(os.path.dirname(HERE), "include", "spnet.h"))
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, force: bool = True) -> str:
    """Compile and link libspnet.so; force=False skips objects newer than their sources."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
    objs = [os.path.join(BUILD, s + ".o") for s in HOST_SOURCES + DEVICE_SOURCES]
    for src in DEVICE_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append([HIPCC, *DEVICE_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
    for t, kc in STAR_VARIANTS:
        obj = os.path.join(BUILD, f"star_{t}_{kc}.o")
        objs.append(obj)
        jobs.append([HIPCC, *DEVICE_FLAGS, f"-DSTAR_T={t}", f"-DSTAR_KC={kc}", "-c",
                     os.path.join(CSRC, "star_inst.hip"), "-o", obj])
    # the widest variants first: they take longest
    jobs.sort(key=lambda j: -max([int(a.split("=")[1]) for a in j if a.startswith("-DSTAR_KC=")] or [0]))
    if not force:
        jobs = [j for j in jobs if _stale(j[-1], [a for a in j if a.endswith((".cpp", ".hip"))][0])]
    if jobs:
        with ThreadPoolExecutor(max_workers=min(int(os.environ.get("MAX_JOBS", "8")), len(jobs))) as ex:
            list(ex.map(_run, jobs))
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "--offload-arch=gfx950", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


SAN_LIB = os.path.join(HERE, "libspnet_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


def build_sanitized(verbose: bool = False) -> str:
    """libspnet_san.so: the host sources with AddressSanitizer and
    UndefinedBehaviorSanitizer (g++), linked with the device objects of the
    normal build (built first if missing) and gcc's sanitizer runtimes. Load it
    with SPNET_LIB=<path> and LD_PRELOAD=$(gcc -print-file-name=libasan.so);
    host code only (network, assembly, spaces, factorisation, ABI, server)."""
    dev_objs = [os.path.join(BUILD, s + ".o") for s in DEVICE_SOURCES]
    dev_objs += [os.path.join(BUILD, f"star_{t}_{kc}.o") for t, kc in STAR_VARIANTS]
    if not all(os.path.exists(o) for o in dev_objs):
        build(verbose=verbose, force=False)
    san = os.path.join(BUILD, "san")
    os.makedirs(san, exist_ok=True)
    jobs, objs = [], []
    for src in HOST_SOURCES:
        obj = os.path.join(san, src + ".o")
        objs.append(obj)
        jobs.append(["g++", *HOST_FLAGS, *SAN_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=min(int(os.environ.get("MAX_JOBS", "8")), len(jobs))) as ex:
        list(ex.map(_run, jobs))
    tmp = SAN_LIB + ".tmp"
    _run([HIPCC, "-shared", "--offload-arch=gfx950", "-o", tmp, *objs, *dev_objs, "-lpthread", "-lasan", "-lubsan"])
    os.replace(tmp, SAN_LIB)
    if verbose:
        print("built", SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        build_sanitized(verbose=True)
    else:
        build(verbose=True, force="--incremental" not in sys.argv)

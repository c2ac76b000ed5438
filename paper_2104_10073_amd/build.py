"""Build the gfx950 library (libzmc.so) in-tree with hipcc.

Three translation units: the batched kernels, the other kernels and the host
runtime.  Flags:
* --offload-arch=gfx950 only;
* -ffp-contract=off: every fused multiply-add in the kernels is written out,
  so the FP64 path keeps the reference operation order;
* packed FP32 instructions disabled (the FP32 path is written as scalar code).
"""

from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(os.path.dirname(PKG), "include")
LIB = os.path.join(PKG, "libzmc.so")
BUILD = os.path.join(PKG, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-ffp-contract=off",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + INCLUDE, "-I" + CSRC, "-Wall", "-Wno-unused-result"]
SOURCES = ["zmc_batched.hip", "zmc_kernels.hip", "zmc_host.hip"]


def _run(cmd):
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return proc


def _newer(a: str, b: str) -> bool:
    return os.path.exists(b) and os.path.getmtime(b) >= os.path.getmtime(a)


def _rtc_headers_object() -> str:
    """Object holding the device headers as strings, for run-time compiled families."""
    parts = ["namespace zmc {"]
    for var, name in (("kRtcHeaderDevice", "zmc_device.hpp"), ("kRtcHeaderCode", "zmc_device_code.hpp")):
        text = open(os.path.join(CSRC, name)).read()
        assert ")zmcrtc\"" not in text
        parts.append(f'extern const char* const {var};\nconst char* const {var} = R"zmcrtc({text})zmcrtc";')
    parts.append("}  // namespace zmc\n")
    src = os.path.join(BUILD, "zmc_rtc_headers.cpp")
    with open(src, "w") as f:
        f.write("\n".join(parts))
    obj = os.path.join(BUILD, "zmc_rtc_headers.o")
    _run(["g++", "-O1", "-fPIC", "-c", src, "-o", obj])
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile the translation units (in parallel) and link libzmc.so.

    incremental=True skips an object that is newer than its source and the
    shared headers (for development; the default always recompiles)."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    procs = []
    headers = [os.path.join(CSRC, "zmc_device.hpp"), os.path.join(CSRC, "zmc_device_code.hpp"),
               os.path.join(CSRC, "zmc_pack.hpp"),
               os.path.join(INCLUDE, "zmc.h")]
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        objs.append(obj)
        if incremental and all(_newer(x, obj) for x in [os.path.join(CSRC, src), *headers]):
            continue
        cmd = [HIPCC, *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    for cmd, p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out + err)
            raise RuntimeError("build step failed: " + " ".join(cmd))
    objs.append(_rtc_headers_object())
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs,
          "-L/opt/rocm/lib", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))

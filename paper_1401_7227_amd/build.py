"""Builds libasm_mi355x.so (HIP kernels for gfx950 + host C++ setup) in-tree."""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libasm_mi355x.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["kernels.hip", "dense.hip", "setup.cpp", "capi.cpp", "batch.cpp"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-Wall", "-Wno-unused-result",
          f"-I{os.path.join(ROOT, 'include')}"]
# Device code: gfx950 only; packed-FP32 instructions disabled (the compiler
# must not form v_pk_* FP32 ops).
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


# The compiler's resource-usage remarks of the device code: every kernel
# must run without private (scratch) memory and without register spills.
# A spill reload the register allocator placed under an empty execution
# mask once read garbage in the batched sweep; this keeps any scratch use
# from coming back unnoticed.
REMARKS = "-Rpass-analysis=kernel-resource-usage"
_REMARK = re.compile(r"remark: +(Function Name|ScratchSize \[bytes/lane\]|VGPRs Spill|SGPRs Spill|VGPRs|AGPRs"
                     r"|LDS Size \[bytes/block\]): (\S+)")


def parse_resources(text: str) -> dict:
    """kernel name -> {remark: value} from the compiler's remark output."""
    out, cur = {}, None
    for line in text.splitlines():
        m = _REMARK.search(line)
        if not m:
            continue
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = out.setdefault(val, {})
        elif cur is not None:
            cur[key] = int(val)
    return out


def check_resources(res: dict, src: str) -> None:
    bad = {k: v for k, v in res.items()
           if v.get("ScratchSize [bytes/lane]", 0) or v.get("VGPRs Spill", 0) or v.get("SGPRs Spill", 0)}
    if bad:
        raise RuntimeError(f"{src}: kernels with scratch memory or spills: {bad}")


def _compile(src: str, obj: str) -> dict:
    path = os.path.join(CSRC, src)
    cmd = [HIPCC, *COMMON]
    dev = src.endswith(".hip")
    if dev:
        cmd += ["-x", "hip", *DEVICE, REMARKS]
    else:  # host-only C++: no device compilation pass
        cmd += ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
    cmd += ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"compile failed: {src}")
    res = parse_resources(r.stderr) if dev else {}
    if dev:
        check_resources(res, src)
    noise = [l for l in r.stderr.splitlines()
             if "packed-fp32-ops" not in l and "kernel-resource-usage" not in l and l.strip()
             and not l.lstrip().startswith(("|", "^")) and not re.match(r"^\s*\d+ \|", l)]
    if any(noise):
        sys.stderr.write("\n".join(noise) + "\n")
    return res


RESOURCES: dict = {}  # of the last build: kernel -> resource-usage remarks


def build() -> str:
    """Compiles every source and links the shared library (always rebuilds)."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, s.rsplit(".", 1)[0] + ".o") for s in SOURCES]
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        res = list(ex.map(_compile, SOURCES, objs))
    global RESOURCES
    RESOURCES = {k: v for r in res for k, v in r.items()}
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fopenmp", f"--offload-arch={ARCH}", "-o", tmp, *objs,
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx",
           "-Wl,-rpath,/opt/rocm/llvm/lib", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())

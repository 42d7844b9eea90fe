"""CPU-side safety nets: the host planner and the oracle under AddressSanitizer
and UndefinedBehaviorSanitizer, and the device code's resource usage.

* The planner (the library's host setup, setup.cpp) is built together with
  tests/native/planner_check.cpp by g++ with -fsanitize=address,undefined
  and run on the 10x10x5 configuration, mid-size grids and a case whose
  coarse rows are split into pieces; the driver checks the plan's internal
  consistency, and its sizes are compared with the oracle's.
* The oracle (oracle.c) is built with the same sanitizers and the oracle
  pins run against it in a child process (AddressSanitizer preloaded).
* Every HIP kernel is compiled for gfx950 with the compiler's
  resource-usage remarks: none may use scratch memory or spill registers.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import gen
import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1401_7227_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def _gxx_ok():
    try:
        subprocess.run(["g++", "--version"], check=True, capture_output=True)
        return True
    except (OSError, subprocess.CalledProcessError):
        return False


@pytest.fixture(scope="module")
def planner(tmp_path_factory):
    if not _gxx_ok():
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("san") / "planner_check")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fopenmp", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           f"-I{os.path.join(ROOT, 'include')}", os.path.join(ROOT, "tests", "native", "planner_check.cpp"),
           os.path.join(CSRC, "setup.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


@pytest.fixture(scope="module")
def planner_nb4(tmp_path_factory):
    """The planner check built for four record buffers (no sanitizers)."""
    if not _gxx_ok():
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("nb4") / "planner_check_nb4")
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-DASM_REC_BUFS=4", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           f"-I{os.path.join(ROOT, 'include')}", os.path.join(ROOT, "tests", "native", "planner_check.cpp"),
           os.path.join(CSRC, "setup.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


PLANS = [
    # grid, kind, combine, sx, sy, overlap, near, far, precision, field
    ((10, 10, 5), 1, 0, 4, 1, 1, (2, 2, 2), (5, 5, 5), 0, 0),
    ((10, 10, 5), 1, 1, 4, 1, 1, (2, 2, 2), (5, 5, 5), 0, 0),
    ((10, 10, 5), 2, 1, 4, 1, 1, (2, 2, 2), (5, 5, 5), 0, 0),
    ((13, 11, 7), 2, 1, 4, 3, 2, (2, 3, 2), (5, 4, 3), 0, 0),
    ((13, 11, 7), 2, 0, 3, 3, 0, (1, 1, 1), (3, 3, 3), 1, 0),
    ((40, 36, 20), 2, 1, 5, 4, 1, (4, 4, 4), (8, 8, 8), 1, 0),
    ((40, 36, 20), 2, 1, 5, 4, 1, (4, 4, 4), (8, 8, 8), 0, 1),
    ((40, 36, 20), 2, 1, 5, 4, 1, (4, 4, 4), (8, 8, 8), 0, 2),
    ((48, 48, 16), 1, 0, 6, 6, 2, (2, 2, 2), (4, 4, 4), 0, 0),
    # near boxes spanning a whole y-z face: coarse rows too long for one record
    ((24, 16, 64), 2, 1, 3, 1, 1, (1, 16, 64), (8, 8, 8), 0, 0),
]


def _run_planner(exe, case):
    grid, kind, comb, sx, sy, ov, near, far, prec, field = case
    args = [exe, *map(str, grid), str(kind), str(comb), str(sx), str(sy), str(ov), *map(str, near), *map(str, far),
            str(prec), str(field)]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="4")
    r = subprocess.run(args, capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, f"{case}: {r.stderr[-4000:]}"
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


@pytest.mark.parametrize("case", PLANS, ids=[f"{c[0][0]}x{c[0][1]}x{c[0][2]}-k{c[1]}c{c[2]}-{c[3]}x{c[4]}d{c[5]}"
                                             f"-p{c[8]}f{c[9]}" for c in PLANS])
def test_planner_under_sanitizers(planner, case):
    st = _run_planner(planner, case)
    assert st["fails"] == 0
    grid, kind, comb, sx, sy, ov, near, far, prec, field = case
    s = gen.generate(*grid, seed=1)
    Bo = O.Precond(O.Matrix.from_system(s), kind=kind, combine=comb, sx=sx, sy=sy, overlap=ov, near=near, far=far,
                   field=field)
    subs = [Bo.sub(i) for i in range(Bo.nsub)]
    assert st["nsub"] == Bo.nsub
    assert st["ext_rows"] == sum(u.n for u in subs)
    assert st["factor_blocks"] == sum(int(u.rp[-1]) for u in subs)
    if grid == (24, 16, 64):
        assert st["split_rows"] > 0


def test_config1_plan_sizes(planner):
    """The 10x10x5 two-level plan: 915 extended rows (800 fine + 115
    coarse) and 5,931 stored blocks."""
    st = _run_planner(planner, PLANS[2])
    assert (st["ext_rows"], st["coarse_rows"], st["factor_blocks"]) == (915, 115, 5931)


def test_oracle_pins_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    r = subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-Wall", "-shared", "-fPIC", *SAN,
                        os.path.join(ROOT, "oracle", "oracle.c"), "-o", lib, "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("libasan not found")
    env = dict(os.environ, ASM_ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_comparators.py")],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=1200)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "ERROR: AddressSanitizer" not in out, out[-4000:]


def test_device_code_uses_no_scratch(tmp_path):
    """Every kernel of the library, compiled for gfx950 as the build does:
    no scratch memory, no spilled registers; the sweep kernel is among them."""
    sys.path.insert(0, ROOT)
    from paper_1401_7227_amd import build as B
    allres = {}
    for src in ("kernels.hip", "dense.hip"):
        cmd = [B.HIPCC, *B.COMMON, "-x", "hip", *B.DEVICE, B.REMARKS, "--cuda-device-only", "-c",
               os.path.join(CSRC, src), "-o", str(tmp_path / (src + ".o"))]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        res = B.parse_resources(r.stderr)
        assert res, "no resource remarks"
        allres.update(res)
    bad = {k: v for k, v in allres.items()
           if v.get("ScratchSize [bytes/lane]", 0) or v.get("VGPRs Spill", 0) or v.get("SGPRs Spill", 0)}
    assert not bad, bad
    sweeps = [k for k in allres if "ilu_apply" in k]
    assert sweeps and all(allres[k]["ScratchSize [bytes/lane]"] == 0 for k in sweeps)


def test_four_buffer_sweep_builds(tmp_path, planner_nb4):
    """The sweep's other compile-time shape (four 27,584-byte record buffers,
    ASM_REC_BUFS=4): the kernels compile for gfx950 without scratch or
    spills, and two-level plans of 48x48x32 cells (FP64 and FP32 factors)
    pass every check (the records fit the smaller buffers, each head names
    the step five ahead)."""
    sys.path.insert(0, ROOT)
    from paper_1401_7227_amd import build as B
    cmd = [B.HIPCC, *B.COMMON, "-DASM_REC_BUFS=4", "-x", "hip", *B.DEVICE, B.REMARKS, "--cuda-device-only", "-c",
           os.path.join(CSRC, "kernels.hip"), "-o", str(tmp_path / "kernels4.o")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    res = B.parse_resources(r.stderr)
    sweeps = [k for k in res if "apply_kernel" in k]
    assert sweeps and all(res[k]["ScratchSize [bytes/lane]"] == 0 and res[k].get("VGPRs Spill", 0) == 0
                          for k in sweeps)
    for prec in (0, 1):
        st = _run_planner(planner_nb4, ((48, 48, 32), 2, 1, 6, 6, 1, (4, 4, 4), (16, 16, 16), prec, 0))
        assert st["fails"] == 0

"""AddressSanitizer + UndefinedBehaviorSanitizer runs of the host code (CPU only).

* The oracle (oracle.c) built by gcc with ASan and UBSan (UB is fatal),
  loaded in a child process that preloads gcc's ASan runtime, runs every
  oracle pin (tests/test_oracle_pins.py: hand cases, brute force, borders,
  culling, NaN/Inf positions, empty inputs, termination, adjoints).
* The HIP library with its host code built by clang with ASan and UBSan
  (device code unchanged), loaded in a child process that preloads clang's
  ASan runtime, runs the host-validation tests of the C ABI
  (tests/test_abi.py: every entry point with null, misaligned, oversized and
  inconsistent arguments, sizes queries, the tuning records), none of which
  reaches the device.

Both builds go to separate files (liborc_san.so, libinpc_raster_san.so) and
are selected in the child through INPC_ORACLE_LIB / INPC_RASTER_LIB.  A
sanitizer report makes the child fail.
"""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

ORC_SAN = os.path.join(ROOT, "oracle", "liborc_san.so")
RASTER_SAN = os.path.join(ROOT, "paper_2403_16862_amd", "libinpc_raster_san.so")
GCC_SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
HOST_SAN_COMPILE = ["-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined"]
HOST_SAN_LINK = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def _runtime(compiler, name):
    p = subprocess.run([compiler, f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not p or not os.path.isabs(p) or not os.path.exists(p):
        pytest.skip(f"{name} not found for {compiler}")
    return p


def _stale(target, sources):
    return not os.path.exists(target) or any(os.path.getmtime(s) > os.path.getmtime(target) for s in sources)


def _child(env_extra, test_file):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", test_file, "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu"], cwd="/tmp", env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    return out


def test_oracle_under_asan_ubsan():
    from oracle import build as ob
    if _stale(ORC_SAN, [ob.SRC]):
        ob.build(lib_path=ORC_SAN, opt_flags=GCC_SAN)
    asan = _runtime("gcc", "libasan.so")
    assert b"__asan_report" in open(ORC_SAN, "rb").read() and b"__ubsan_handle" in open(ORC_SAN, "rb").read()
    probe = "import oracle; assert oracle.LIB_PATH.endswith('liborc_san.so'); oracle.lib()"
    env = {"LD_PRELOAD": asan, "INPC_ORACLE_LIB": ORC_SAN, "PYTHONPATH": ROOT}
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env={**os.environ, **env,
                       "ASAN_OPTIONS": "detect_leaks=0"}, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    out = _child(env, os.path.join(ROOT, "tests", "test_oracle_pins.py"))
    assert " passed" in out


def test_host_validation_under_asan_ubsan():
    from paper_2403_16862_amd import build as hb
    hipcc = hb.HIPCC
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    srcs = [os.path.join(hb.CSRC, s) for s in hb.SOURCES] + glob.glob(os.path.join(hb.CSRC, "*.h")) + \
        [os.path.join(ROOT, "include", "inpc_raster.h")]
    if _stale(RASTER_SAN, srcs):
        hb.build(objdir=os.path.join(hb.HERE, "_build_san"), lib_path=RASTER_SAN, extra_flags=HOST_SAN_COMPILE,
                 link_flags=HOST_SAN_LINK)
    asan = _runtime(hipcc, "libclang_rt.asan-x86_64.so")
    env = {"LD_PRELOAD": asan, "INPC_RASTER_LIB": RASTER_SAN, "PYTHONPATH": ROOT}
    blob = open(RASTER_SAN, "rb").read()
    assert b"__asan_report" in blob and b"__ubsan_handle" in blob
    probe = ("import paper_2403_16862_amd as pr; assert pr.LIB_PATH.endswith('libinpc_raster_san.so'); "
             "assert pr.lib().inpc_version() >= 1")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env={**os.environ, **env,
                       "ASAN_OPTIONS": "detect_leaks=0"}, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    out = _child(env, os.path.join(ROOT, "tests", "test_abi.py"))
    assert " passed" in out

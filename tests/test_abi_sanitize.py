"""The C ABI's host-side paths under AddressSanitizer (with leak detection)
and UndefinedBehaviorSanitizer: tests/sanitize/abi_driver.cpp calls every
entry point with NULL handles and pointers, bad configurations, empty
batches and (with no device visible) the create calls.  The library sources
are compiled with the sanitizers on their host code only (device code as
usual) into tests/sanitize/_build; the driver must print "done" and exit 0
with no sanitizer report."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1607_07624_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
BUILD = os.path.join(HERE, "_build")
DRIVER = os.path.join(BUILD, "abi_driver")
SOURCES = [os.path.join(CSRC, f) for f in ("pwfs_kernels.hip", "pwfs_kernels16.hip", "pwfs_detector.hip",
                                           "pwfs_psf.hip", "pwfs_sh.hip", "pwfs_fstop.hip", "pwfs_static.hip",
                                           "cnn_kernels.hip", "pwfs_api.cpp", "cnn_api.cpp")]
SOURCES.append(os.path.join(HERE, "abi_driver.cpp"))
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]
FLAGS = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include")] + SANITIZE


def _hipcc():
    p = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(p):
        pytest.skip("hipcc not available")
    return p


def _build():
    deps = SOURCES + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")] + \
        [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    if os.path.exists(DRIVER) and os.path.getmtime(DRIVER) > max(os.path.getmtime(d) for d in deps):
        return
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        objs.append(obj)
        procs.append(subprocess.Popen([hipcc, *FLAGS, "-c", src, "-o", obj], stdout=subprocess.PIPE,
                                      stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out = p.communicate(timeout=600)[0]
        assert p.returncode == 0, out
    r = subprocess.run([hipcc, *SANITIZE, *objs, "-o", DRIVER], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr


@pytest.mark.parametrize("mode", ["no-device", "default"])
def test_abi_host_paths_clean_under_sanitizers(mode):
    _build()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    if mode == "no-device":
        env.update(HIP_VISIBLE_DEVICES="-1", ROCR_VISIBLE_DEVICES="-1")
    args = [DRIVER] + (["no-device"] if mode == "no-device" else [])
    r = subprocess.run(args, env=env, capture_output=True, text=True, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "done:" in r.stdout and "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out

"""Host-side checks of the C ABI: exports, argument validation, error codes.

These run without a GPU: every check here returns before any device work.
"""
import ctypes
import os
import re
import subprocess
import sys

import pytest

import paper_1607_07624_amd as pw
from paper_1607_07624_amd._lib import make_config
from synth.configs import CFG1, CFG2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\**\s*([a-z_][a-z_0-9]*)\s*\(",
                                txt, flags=re.M)
    return names


def test_library_exports_every_declared_symbol():
    lib = pw.load_library()
    names = _declared_functions()
    assert {"pwfs_plan", "pwfs_measure", "recon_apply", "pwfs_destroy"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", pw.library_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\s[TW]\s+(\S+)$", out, flags=re.M))
    for n in names:
        assert n in exported, n
        assert getattr(lib, n) is not None


def _plan_status(**over):
    lib = pw.load_library()
    c = make_config(CFG2, 4)
    for k, v in over.items():
        setattr(c, k, v)
    h = ctypes.c_void_p()
    st = lib.pwfs_plan(ctypes.byref(c), None, ctypes.byref(h))
    return st, lib.pwfs_last_error().decode()


@pytest.mark.parametrize("over,status", [
    (dict(n_pupil=0), -1), (dict(n_bin=3), -1), (dict(batch_max=0), -1),
    (dict(wavelength_m=0.0), -1), (dict(mod_radius_lod=-1.0), -1), (dict(obstruction=1.0), -1),
    (dict(norm_mode=2), -1), (dict(flags=4), -1), (dict(face_shift=-3), -1),
    (dict(n_fft=600), -2), (dict(face_shift=100), -2), (dict(n_pupil=96, n_fft=384), -2),
    (dict(n_bin=5), -2), (dict(n_mod=2000), -2),
    (dict(n_pupil=480, n_fft=1920, n_bin=3), -2), (dict(n_pupil=480, n_fft=1920, n_bin=6), -2),
    (dict(n_pupil=128, n_fft=512, n_bin=5), -1), (dict(n_pupil=320, n_fft=1280), -2),
    (dict(det_window=36), -1), (dict(n_bin=1, det_window=1), -1), (dict(n_bin=1, det_window=161), -1),
    (dict(n_bin=1, det_window=-2), -1), (dict(reserved=1), -1),
    (dict(field_stop_lod=-1.0), -1), (dict(field_stop_lod=float("nan")), -1),
    (dict(n_pupil=480, n_fft=1920, n_bin=5, field_stop_lod=100.0), -2),
])
def test_plan_rejects_bad_config_before_touching_a_device(over, status):
    st, msg = _plan_status(**over)
    assert st == status and msg


def test_null_arguments_rejected():
    lib = pw.load_library()
    assert lib.pwfs_plan(None, None, None) == -1
    h = ctypes.c_void_p()
    assert lib.pwfs_plan(None, None, ctypes.byref(h)) == -1
    assert lib.pwfs_measure(None, None, 1, None, None, None) == -1
    assert lib.pwfs_measure_static(None, None, 1, None, None, None) == -1
    assert lib.pwfs_plan_info(None, None, None, None) == -1
    assert lib.pwfs_get_valid(None, None) == -1
    assert lib.pwfs_set_valid(None, None, 1) == -1
    assert lib.recon_apply(None, 0, 10, None, 1, 1.0, 0.0, None, None) == -1
    assert lib.recon_apply(None, 10, 10, None, -1, 1.0, 0.0, None, None) == -1
    # B == 0 is an empty batch: nothing to do, nothing dereferenced.
    assert lib.recon_apply(None, 10, 10, None, 0, 1.0, 0.0, None, None) == 0
    lib.pwfs_destroy(None)
    assert lib.pwfs_strerror(-4) == b"out of device memory"


def test_no_device_is_an_error_not_a_fallback():
    code = ("import ctypes, sys; sys.path.insert(0, %r)\n"
            "import paper_1607_07624_amd as pw\n"
            "from paper_1607_07624_amd._lib import make_config\n"
            "from synth.configs import CFG1\n"
            "lib = pw.load_library(); h = ctypes.c_void_p()\n"
            "print(lib.pwfs_plan(ctypes.byref(make_config(CFG1, 2)), None, ctypes.byref(h)))\n") % ROOT
    env = dict(os.environ, HIP_VISIBLE_DEVICES="-1", ROCR_VISIBLE_DEVICES="-1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.stdout.strip().splitlines()[-1] == "-3", out.stdout + out.stderr


def test_cnn_abi_validation_and_no_device():
    from paper_1607_07624_amd.cnn import _lib, cnn_config
    lib = _lib()
    h = ctypes.c_void_p()
    assert lib.pwfs_cnn_create(None, ctypes.byref(h)) == -1
    bad = cnn_config(n_sub=2, c1=32, c2=64, c3=64, hidden=2048, n_out=600, batch_max=4, reserved=0)
    assert lib.pwfs_cnn_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    bad.n_sub, bad.reserved = 40, 7
    assert lib.pwfs_cnn_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    assert lib.pwfs_cnn_forward(None, None, 1, None, None) == -1
    assert lib.pwfs_cnn_prepare(None, None, None, 0, 1, 40, None, None) == -1
    assert lib.pwfs_cnn_prepare(None, None, None, 10, 0, 40, None, None) == 0      # empty batch
    step = ctypes.c_int64()
    assert lib.pwfs_cnn_get_optimizer(None, None, None, ctypes.byref(step), None) == -1
    assert lib.pwfs_cnn_set_optimizer(None, None, None, 0, None) == -1
    lib.pwfs_cnn_destroy(None)
    code = ("import ctypes, sys; sys.path.insert(0, %r)\n"
            "from paper_1607_07624_amd.cnn import _lib, cnn_config\n"
            "lib = _lib(); h = ctypes.c_void_p()\n"
            "c = cnn_config(n_sub=40, c1=32, c2=64, c3=64, hidden=2048, n_out=600, batch_max=4, reserved=0)\n"
            "print(lib.pwfs_cnn_create(ctypes.byref(c), ctypes.byref(h)))\n") % ROOT
    env = dict(os.environ, HIP_VISIBLE_DEVICES="-1", ROCR_VISIBLE_DEVICES="-1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.stdout.strip().splitlines()[-1] == "-3", out.stdout + out.stderr


@pytest.mark.parametrize("over,status", [
    (dict(n_pupil=128), -2), (dict(pad=3), -2), (dict(wavelength_m=0.0), -1), (dict(reserved=1), -1),
    (dict(batch_max=0), -1), (dict(obstruction=1.0), -1),
])
def test_psf_camera_rejects_bad_config_before_touching_a_device(over, status):
    from paper_1607_07624_amd._lib import psf_config_struct
    lib = pw.load_library()
    c = psf_config_struct(160, 8, 4, 0, 1.65e-6, 0.0)
    for k, v in over.items():
        setattr(c, k, v)
    h = ctypes.c_void_p()
    assert lib.pwfs_psf_create(ctypes.byref(c), None, ctypes.byref(h)) == status
    assert lib.pwfs_last_error().decode()


@pytest.mark.parametrize("over,status", [
    (dict(n_sub=7), -1), (dict(n_sub=4), -2), (dict(pad=3), -2), (dict(wavelength_m=-1.0), -1),
    (dict(batch_max=0), -1),
])
def test_sh_rejects_bad_config_before_touching_a_device(over, status):
    from paper_1607_07624_amd._lib import sh_config_struct
    lib = pw.load_library()
    c = sh_config_struct(160, 40, 4, 4, 750e-9, 0.0)
    for k, v in over.items():
        setattr(c, k, v)
    h = ctypes.c_void_p()
    assert lib.pwfs_sh_create(ctypes.byref(c), None, ctypes.byref(h)) == status
    assert lib.pwfs_last_error().decode()

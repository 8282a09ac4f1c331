"""ctypes binding of libpwfs.so: same names as the C ABI, marshalling only.

Device buffers are torch tensors on the current HIP device; the HIP stream
is torch's current stream.  torch is used for memory and streams only.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB = None

STATUS_NAMES = {0: "PWFS_OK", -1: "PWFS_ERR_INVALID_ARG", -2: "PWFS_ERR_UNSUPPORTED",
                -3: "PWFS_ERR_NO_DEVICE", -4: "PWFS_ERR_OUT_OF_MEMORY", -5: "PWFS_ERR_HIP"}


class PwfsError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} ({detail})")


class sh_config_struct(ctypes.Structure):
    _fields_ = [("n_pupil", ctypes.c_int32), ("n_sub", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("batch_max", ctypes.c_int32), ("wavelength_m", ctypes.c_double), ("obstruction", ctypes.c_double)]


class psf_config_struct(ctypes.Structure):
    _fields_ = [("n_pupil", ctypes.c_int32), ("pad", ctypes.c_int32), ("batch_max", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("wavelength_m", ctypes.c_double), ("obstruction", ctypes.c_double)]


class detector_struct(ctypes.Structure):
    _fields_ = [("electrons_per_frame", ctypes.c_double), ("readout_noise_e", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class config_struct(ctypes.Structure):
    _fields_ = [("n_fft", ctypes.c_int32), ("n_pupil", ctypes.c_int32), ("n_bin", ctypes.c_int32),
                ("n_mod", ctypes.c_int32), ("face_shift", ctypes.c_int32), ("norm_mode", ctypes.c_int32),
                ("batch_max", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("diameter_m", ctypes.c_double), ("wavelength_m", ctypes.c_double),
                ("mod_radius_lod", ctypes.c_double), ("obstruction", ctypes.c_double),
                ("det_window", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("field_stop_lod", ctypes.c_double)]


def library_path() -> str:
    return os.path.join(_PKG, "libpwfs.so")


def load_library():
    """Load libpwfs.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1607_07624_amd/build.py")
    lib = ctypes.CDLL(path)
    vp, i32, f32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float, ctypes.c_size_t
    lib.pwfs_plan.argtypes = [ctypes.POINTER(config_struct), vp, ctypes.POINTER(vp)]
    lib.pwfs_plan_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(sz)]
    lib.pwfs_get_valid.argtypes = [vp, vp]
    lib.pwfs_set_valid.argtypes = [vp, vp, i32]
    lib.pwfs_get_reference.argtypes = [vp, vp]
    lib.pwfs_set_reference.argtypes = [vp, vp, vp]
    lib.pwfs_measure.argtypes = [vp, vp, i32, vp, vp, vp]
    lib.pwfs_measure_static.argtypes = [vp, vp, i32, vp, vp, vp]
    lib.recon_apply.argtypes = [vp, i32, i32, vp, i32, f32, f32, vp, vp]
    lib.pwfs_get_pupil.argtypes = [vp, vp]
    lib.pwfs_timing_enable.argtypes = [vp, ctypes.c_int]
    lib.pwfs_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.pwfs_get_schedule.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.pwfs_set_schedule.argtypes = [vp, i32, i32, i32]
    lib.pwfs_get_schedule_lanes.argtypes = [vp, i32, ctypes.POINTER(i32)]
    lib.pwfs_set_schedule_lanes.argtypes = [vp, i32, i32]
    lib.pwfs_autotune.argtypes = [vp, i32, i32, vp, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]
    lib.pwfs_set_detector.argtypes = [vp, ctypes.POINTER(detector_struct)]
    lib.pwfs_get_detector.argtypes = [vp, ctypes.POINTER(f32), ctypes.POINTER(ctypes.c_uint64)]
    lib.pwfs_set_frame_counter.argtypes = [vp, ctypes.c_uint64]
    lib.pwfs_detect.argtypes = [vp, vp, i32, ctypes.c_uint64, vp, vp]
    lib.pwfs_sh_create.argtypes = [ctypes.POINTER(sh_config_struct), vp, ctypes.POINTER(vp)]
    lib.pwfs_sh_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.pwfs_sh_get_valid.argtypes = [vp, vp]
    lib.pwfs_sh_get_reference.argtypes = [vp, vp]
    lib.pwfs_sh_measure.argtypes = [vp, vp, i32, vp, vp, vp]
    lib.pwfs_sh_destroy.argtypes = [vp]
    lib.pwfs_sh_destroy.restype = None
    lib.pwfs_psf_create.argtypes = [ctypes.POINTER(psf_config_struct), vp, ctypes.POINTER(vp)]
    lib.pwfs_psf_info.argtypes = [vp, ctypes.POINTER(i32)]
    lib.pwfs_psf_compute.argtypes = [vp, vp, i32, i32, vp, vp, vp]
    lib.pwfs_psf_destroy.argtypes = [vp]
    lib.pwfs_psf_destroy.restype = None
    lib.pwfs_destroy.argtypes = [vp]
    lib.pwfs_destroy.restype = None
    lib.pwfs_strerror.argtypes = [ctypes.c_int]
    lib.pwfs_strerror.restype = ctypes.c_char_p
    lib.pwfs_last_error.argtypes = []
    lib.pwfs_last_error.restype = ctypes.c_char_p
    for name in ("pwfs_plan", "pwfs_plan_info", "pwfs_get_valid", "pwfs_set_valid", "pwfs_get_reference",
                 "pwfs_set_reference", "pwfs_measure", "recon_apply", "pwfs_get_pupil",
                 "pwfs_timing_enable", "pwfs_timing_read", "pwfs_get_schedule", "pwfs_set_schedule",
                 "pwfs_get_schedule_lanes", "pwfs_set_schedule_lanes",
                 "pwfs_autotune", "pwfs_set_detector", "pwfs_get_detector", "pwfs_set_frame_counter",
                 "pwfs_detect", "pwfs_psf_create", "pwfs_psf_info", "pwfs_psf_compute", "pwfs_sh_create",
                 "pwfs_sh_info", "pwfs_sh_get_valid", "pwfs_sh_get_reference", "pwfs_sh_measure"):
        getattr(lib, name).restype = ctypes.c_int
    _LIB = lib
    return lib


def _check(status: int, where: str):
    if status != 0:
        detail = load_library().pwfs_last_error().decode(errors="replace")
        raise PwfsError(status, where, detail)


def _stream_handle(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _need(t, torch, dtype, numel, name):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and t.numel() == numel):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor with {numel} elements")


FLAG_FP32_TABLES = 1
FLAG_FP32_PHASE = 2


def make_config(cfg, batch_max: int, flags: int = 0) -> config_struct:
    """Lower a sensor configuration record (attributes as in synth.configs.SensorConfig)."""
    return config_struct(n_fft=cfg.n_fft, n_pupil=cfg.n_pupil, n_bin=cfg.n_bin, n_mod=cfg.n_mod,
                         face_shift=cfg.face_shift, norm_mode=cfg.norm_mode, batch_max=batch_max,
                         flags=flags, diameter_m=cfg.diameter_m, wavelength_m=cfg.wavelength_m,
                         mod_radius_lod=cfg.mod_radius_lod, obstruction=cfg.obstruction,
                         det_window=getattr(cfg, "det_window", 0), reserved=0,
                         field_stop_lod=getattr(cfg, "field_stop_lod", 0.0))


class Plan:
    """pwfs_plan / pwfs_measure / pwfs_destroy for one sensor geometry."""

    def __init__(self, cfg, batch_max: int = 16, pupil_amp: np.ndarray | None = None, flags: int = 0):
        import torch
        self._torch = torch
        self.lib = load_library()
        self.cfg = cfg
        self.device = torch.cuda.current_device()
        c = make_config(cfg, batch_max, flags)
        amp = None
        if pupil_amp is not None:
            amp = np.ascontiguousarray(pupil_amp, dtype=np.float32)
            if amp.shape != (cfg.n_pupil, cfg.n_pupil):
                raise ValueError("pupil_amp must be P x P")
        h = ctypes.c_void_p()
        _check(self.lib.pwfs_plan(ctypes.byref(c), amp.ctypes.data if amp is not None else None,
                                  ctypes.byref(h)), "pwfs_plan")
        self.handle = h
        nv, ns, ws = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
        _check(self.lib.pwfs_plan_info(h, ctypes.byref(nv), ctypes.byref(ns), ctypes.byref(ws)),
               "pwfs_plan_info")
        self.n_valid, self.n_sub, self.workspace_bytes = nv.value, ns.value, ws.value
        self.batch_max = batch_max

    @property
    def valid(self) -> np.ndarray:
        out = np.empty(self.n_valid, np.int32)
        _check(self.lib.pwfs_get_valid(self.handle, out.ctypes.data), "pwfs_get_valid")
        return out

    def set_valid(self, idx) -> None:
        """Replace the valid-subaperture list (pwfs_set_valid); the reference
        slopes are measured again."""
        a = np.ascontiguousarray(idx, dtype=np.int32)
        _check(self.lib.pwfs_set_valid(self.handle, a.ctypes.data, int(a.size)), "pwfs_set_valid")
        nv, ns, ws = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
        _check(self.lib.pwfs_plan_info(self.handle, ctypes.byref(nv), ctypes.byref(ns), ctypes.byref(ws)),
               "pwfs_plan_info")
        self.n_valid, self.workspace_bytes = nv.value, ws.value

    @property
    def s_ref(self) -> np.ndarray:
        out = np.empty(2 * self.n_valid, np.float32)
        _check(self.lib.pwfs_get_reference(self.handle, out.ctypes.data), "pwfs_get_reference")
        return out

    @property
    def pupil(self) -> np.ndarray:
        P = self.cfg.n_pupil
        out = np.empty((P, P), np.float32)
        _check(self.lib.pwfs_get_pupil(self.handle, out.ctypes.data), "pwfs_get_pupil")
        return out

    def timing_enable(self, enable: bool = True):
        _check(self.lib.pwfs_timing_enable(self.handle, int(enable)), "pwfs_timing_enable")

    def timing_read(self) -> dict:
        r, c, s, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        _check(self.lib.pwfs_timing_read(self.handle, ctypes.byref(r), ctypes.byref(c), ctypes.byref(s),
                                         ctypes.byref(n)), "pwfs_timing_read")
        return {"row_ms": r.value, "col_ms": c.value, "slopes_ms": s.value, "slices": n.value}

    def set_detector(self, electrons_per_frame: float, readout_noise_e: float = 0.0, seed: int = 0):
        """Photon + readout noise on the binned images (electrons_per_frame = 0: noiseless)."""
        d = detector_struct(float(electrons_per_frame), float(readout_noise_e), int(seed))
        _check(self.lib.pwfs_set_detector(self.handle, ctypes.byref(d)), "pwfs_set_detector")

    def detector(self) -> dict:
        g, f = ctypes.c_float(), ctypes.c_uint64()
        _check(self.lib.pwfs_get_detector(self.handle, ctypes.byref(g), ctypes.byref(f)), "pwfs_get_detector")
        return {"gain": g.value, "next_frame": f.value}

    def set_frame_counter(self, frame: int):
        _check(self.lib.pwfs_set_frame_counter(self.handle, int(frame)), "pwfs_set_frame_counter")

    def detect(self, intensity, frame0: int, pixels=None):
        """pwfs_detect: detector pixels from noiseless images [B, 4, S, S] (device tensors)."""
        torch = self._torch
        B = intensity.shape[0]
        S = self.n_sub
        _need(intensity, torch, torch.float32, B * 4 * S * S, "intensity")
        if pixels is None:
            pixels = torch.empty_like(intensity)
        _need(pixels, torch, torch.float32, B * 4 * S * S, "pixels")
        _check(self.lib.pwfs_detect(self.handle, _ptr(intensity), int(B), int(frame0), _ptr(pixels),
                                    _stream_handle(torch, self.device)), "pwfs_detect")
        return pixels

    def get_schedule(self, B: int) -> tuple:
        """(a_chunk, k_chunk) pwfs_measure uses for slices of B frames."""
        a, k = ctypes.c_int32(), ctypes.c_int32()
        _check(self.lib.pwfs_get_schedule(self.handle, int(B), ctypes.byref(a), ctypes.byref(k)), "pwfs_get_schedule")
        return a.value, k.value

    def set_schedule(self, B: int, a_chunk: int, k_chunk: int):
        """Fix the schedule for slices of B frames ((0, 0): back to the default)."""
        _check(self.lib.pwfs_set_schedule(self.handle, int(B), int(a_chunk), int(k_chunk)), "pwfs_set_schedule")

    def autotune(self, B: int, reps: int = 5) -> dict:
        """Run the library's autotuner for slices of B frames (waits for the stream)."""
        d0, d1 = ctypes.c_double(), ctypes.c_double()
        _check(self.lib.pwfs_autotune(self.handle, int(B), int(reps), _stream_handle(self._torch, self.device),
                                       ctypes.byref(d0), ctypes.byref(d1)), "pwfs_autotune")
        a, k = self.get_schedule(B)
        return {"B": int(B), "a_chunk": a, "k_chunk": k, "lanes": self.get_lanes(B), "ms_default": d0.value,
                "ms_tuned": d1.value}

    def get_lanes(self, B: int) -> int:
        """Lane form (8 or 32 lanes per line) pwfs_measure uses for slices of B frames."""
        n = ctypes.c_int32()
        _check(self.lib.pwfs_get_schedule_lanes(self.handle, int(B), ctypes.byref(n)), "pwfs_get_schedule_lanes")
        return n.value

    def set_lanes(self, B: int, lanes: int):
        _check(self.lib.pwfs_set_schedule_lanes(self.handle, int(B), int(lanes)), "pwfs_set_schedule_lanes")

    def set_reference(self, sref=None):
        t = self._torch
        if sref is not None:
            _need(sref, t, t.float32, 2 * self.n_valid, "sref")
        _check(self.lib.pwfs_set_reference(self.handle, _ptr(sref), _stream_handle(t, self.device)),
               "pwfs_set_reference")

    def measure_into(self, opd, pupils=None, slopes=None):
        """pwfs_measure on caller-owned tensors (asynchronous on torch's current stream)."""
        t = self._torch
        P, S = self.cfg.n_pupil, self.n_sub
        B = opd.shape[0] if opd.dim() == 3 else 1
        _need(opd, t, t.float32, B * P * P, "opd")
        if pupils is not None:
            _need(pupils, t, t.float32, B * 4 * S * S, "pupils")
        if slopes is not None:
            _need(slopes, t, t.float32, B * 2 * self.n_valid, "slopes")
        _check(self.lib.pwfs_measure(self.handle, _ptr(opd), B, _ptr(pupils), _ptr(slopes),
                                     _stream_handle(t, self.device)), "pwfs_measure")
        return pupils, slopes

    def measure_static_into(self, opd, pupils=None, slopes=None):
        """pwfs_measure_static (no allocation: the workspace is the library's
        static device array) on caller-owned tensors."""
        t = self._torch
        P, S = self.cfg.n_pupil, self.n_sub
        B = opd.shape[0] if opd.dim() == 3 else 1
        _need(opd, t, t.float32, B * P * P, "opd")
        if pupils is not None:
            _need(pupils, t, t.float32, B * 4 * S * S, "pupils")
        if slopes is not None:
            _need(slopes, t, t.float32, B * 2 * self.n_valid, "slopes")
        _check(self.lib.pwfs_measure_static(self.handle, _ptr(opd), B, _ptr(pupils), _ptr(slopes),
                                            _stream_handle(t, self.device)), "pwfs_measure_static")
        return pupils, slopes

    def measure(self, opd, want_pupils: bool = True):
        """(pupils [B,4,S,S] or None, slopes [B, 2 n_valid]) for opd [B,P,P] float32 nm."""
        t = self._torch
        opd = opd.contiguous()
        B = opd.shape[0] if opd.dim() == 3 else 1
        S = self.n_sub
        pupils = t.empty((B, 4, S, S), dtype=t.float32, device=opd.device) if want_pupils else None
        slopes = t.empty((B, 2 * self.n_valid), dtype=t.float32, device=opd.device)
        return self.measure_into(opd, pupils, slopes)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pwfs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def recon_apply(R, s, alpha: float = 1.0, beta: float = 0.0, m=None):
    """m = alpha R s + beta m for each row of s ([B, n_s]); returns m [B, M]."""
    import torch
    lib = load_library()
    M, ns = R.shape
    s2 = s.reshape(-1, ns)
    B = s2.shape[0]
    _need(R, torch, torch.float32, M * ns, "R")
    _need(s2, torch, torch.float32, B * ns, "s")
    if m is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs an existing m")
        m = torch.empty((B, M), dtype=torch.float32, device=R.device)
    _need(m, torch, torch.float32, B * M, "m")
    _check(lib.recon_apply(_ptr(R), M, ns, _ptr(s2), B, float(alpha), float(beta), _ptr(m),
                           _stream_handle(torch, R.device)), "recon_apply")
    return m


class PsfCamera:
    """pwfs_psf_create / pwfs_psf_compute / pwfs_psf_destroy."""

    def __init__(self, n_pupil: int, pad: int, wavelength_m: float, batch_max: int = 16,
                 obstruction: float = 0.0, pupil_amp: np.ndarray | None = None):
        import torch
        self._torch = torch
        self.lib = load_library()
        self.device = torch.cuda.current_device()
        c = psf_config_struct(int(n_pupil), int(pad), int(batch_max), 0, float(wavelength_m), float(obstruction))
        amp = None
        if pupil_amp is not None:
            amp = np.ascontiguousarray(pupil_amp, dtype=np.float32)
            if amp.shape != (n_pupil, n_pupil):
                raise ValueError("pupil_amp must be P x P")
        h = ctypes.c_void_p()
        _check(self.lib.pwfs_psf_create(ctypes.byref(c), amp.ctypes.data if amp is not None else None,
                                        ctypes.byref(h)), "pwfs_psf_create")
        self.handle = h
        n = ctypes.c_int32()
        _check(self.lib.pwfs_psf_info(h, ctypes.byref(n)), "pwfs_psf_info")
        self.n_image = n.value
        self.n_pupil = n_pupil

    def compute(self, opd, psf=None, strehl=None, accumulate: bool = False, want_psf: bool = True):
        torch = self._torch
        B = opd.shape[0]
        P, N = self.n_pupil, self.n_image
        _need(opd, torch, torch.float32, B * P * P, "opd")
        if want_psf and psf is None:
            psf = torch.zeros((N, N) if accumulate else (B, N, N), device=opd.device)
        if psf is not None:
            _need(psf, torch, torch.float32, N * N if accumulate else B * N * N, "psf")
        if strehl is None:
            strehl = torch.empty(B, device=opd.device)
        _check(self.lib.pwfs_psf_compute(self.handle, _ptr(opd), int(B), 1 if accumulate else 0,
                                         _ptr(psf) if psf is not None else None, _ptr(strehl),
                                         _stream_handle(torch, self.device)), "pwfs_psf_compute")
        return psf, strehl

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pwfs_psf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ShPlan:
    """pwfs_sh_create / pwfs_sh_measure / pwfs_sh_destroy, with the same
    measure_into / n_valid / batch_max interface as Plan (so calibration and
    the closed loops drive either sensor)."""

    def __init__(self, n_pupil: int, n_sub: int, pad: int, wavelength_m: float, batch_max: int = 16,
                 obstruction: float = 0.0, pupil_amp: np.ndarray | None = None):
        import torch
        self._torch = torch
        self.lib = load_library()
        self.device = torch.cuda.current_device()
        c = sh_config_struct(int(n_pupil), int(n_sub), int(pad), int(batch_max), float(wavelength_m),
                             float(obstruction))
        amp = None
        if pupil_amp is not None:
            amp = np.ascontiguousarray(pupil_amp, dtype=np.float32)
        h = ctypes.c_void_p()
        _check(self.lib.pwfs_sh_create(ctypes.byref(c), amp.ctypes.data if amp is not None else None,
                                       ctypes.byref(h)), "pwfs_sh_create")
        self.handle = h
        nv, m = ctypes.c_int32(), ctypes.c_int32()
        _check(self.lib.pwfs_sh_info(h, ctypes.byref(nv), ctypes.byref(m)), "pwfs_sh_info")
        self.n_valid, self.spot_side = nv.value, m.value
        self.n_pupil, self.n_sub, self.batch_max = n_pupil, n_sub, batch_max

    @property
    def valid(self) -> np.ndarray:
        out = np.empty(self.n_valid, np.int32)
        _check(self.lib.pwfs_sh_get_valid(self.handle, out.ctypes.data), "pwfs_sh_get_valid")
        return out

    @property
    def s_ref(self) -> np.ndarray:
        out = np.empty(2 * self.n_valid, np.float32)
        _check(self.lib.pwfs_sh_get_reference(self.handle, out.ctypes.data), "pwfs_sh_get_reference")
        return out

    def measure_into(self, opd, spots=None, slopes=None):
        torch = self._torch
        B = opd.shape[0]
        P, nv, M = self.n_pupil, self.n_valid, self.spot_side
        _need(opd, torch, torch.float32, B * P * P, "opd")
        if spots is not None:
            _need(spots, torch, torch.float32, B * nv * M * M, "spots")
        if slopes is not None:
            _need(slopes, torch, torch.float32, B * 2 * nv, "slopes")
        _check(self.lib.pwfs_sh_measure(self.handle, _ptr(opd), int(B), _ptr(spots) if spots is not None else None,
                                        _ptr(slopes) if slopes is not None else None,
                                        _stream_handle(torch, self.device)), "pwfs_sh_measure")

    def measure(self, opd, want_spots: bool = True):
        torch = self._torch
        B = opd.shape[0]
        spots = torch.empty((B, self.n_valid, self.spot_side, self.spot_side), device=opd.device) if want_spots else None
        slopes = torch.empty((B, 2 * self.n_valid), device=opd.device)
        self.measure_into(opd, spots, slopes)
        return spots, slopes

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pwfs_sh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

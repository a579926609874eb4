"""Python binding of libevis (ctypes): argument marshalling only.

Every function here has the name of the C entry point it calls and passes
device pointers of torch tensors plus the current HIP stream; all
arithmetic happens in the library's HIP kernels.  torch provides device
memory and streams, nothing else.  The library must have been built
(``python -m paper_2607_08098_amd.build``); without it every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libevis.so")

EVIS_OK = 0
EVIS_ERR_INVALID = -1
EVIS_ERR_UNSUPPORTED = -2
EVIS_ERR_HIP = -3
EVIS_ERR_NOMEM = -4
EVIS_BLEND_TIME = 0
EVIS_BLEND_B_PRIMARY = 1
EVIS_WARP_GATHER = 0x00       # or'ed with an EVIS_BLEND_* into the mode word
EVIS_WARP_SPLAT = 0x10
EVIS_WARP_JOINT = 0x20
EVIS_FLAG_RESET_CURSOR = 1
EVIS_T_LAST_INIT = -(2 ** 30)
EVIS_MAX_CROSSINGS = 65535

_c_float_p = ctypes.POINTER(ctypes.c_float)


class EvisPair(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("L_A", ctypes.c_void_p), ("L_B", ctypes.c_void_p),
                ("m_A", ctypes.c_void_p), ("m_B", ctypes.c_void_p),
                ("Z_A", ctypes.c_void_p), ("Z_B", ctypes.c_void_p),
                ("t0_us", ctypes.c_int64), ("t1_us", ctypes.c_int64)]


class EvisSensor(ctypes.Structure):
    _fields_ = [("C_on", ctypes.c_float), ("C_off", ctypes.c_float),
                ("theta_on", ctypes.c_void_p), ("theta_off", ctypes.c_void_p),
                ("refractory_us", ctypes.c_int32), ("K", ctypes.c_int32),
                ("K_max", ctypes.c_int32), ("blend_mode", ctypes.c_int32)]


class EvisState(ctypes.Structure):
    _fields_ = [("L_ref", ctypes.c_void_p), ("t_last", ctypes.c_void_p)]


class EvisNoise(ctypes.Structure):
    _fields_ = [("leak_rate_hz", ctypes.c_float), ("shot_rate_hz", ctypes.c_float),
                ("hot_rate_hz", ctypes.c_float), ("hot_fraction", ctypes.c_float),
                ("shot_L0", ctypes.c_float), ("shot_inv_range", ctypes.c_float),
                ("seed", ctypes.c_uint64), ("pair_index", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class EvisFrames(ctypes.Structure):
    _fields_ = [("L_seq", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("K", ctypes.c_int32), ("env_id", ctypes.c_int32), ("t0_us", ctypes.c_int64),
                ("t1_us", ctypes.c_int64), ("sensor", EvisSensor), ("state", EvisState)]


class EvisEnv(ctypes.Structure):
    _fields_ = [("pair", EvisPair), ("sensor", EvisSensor), ("state", EvisState),
                ("env_id", ctypes.c_int32), ("crop_margin", ctypes.c_int32),
                ("noise", ctypes.POINTER(EvisNoise))]


class EvisSoftEnv(ctypes.Structure):
    _fields_ = [("pair", EvisPair), ("L_ref", ctypes.c_void_p), ("S", ctypes.c_void_p),
                ("gS", ctypes.c_void_p), ("gL_A", ctypes.c_void_p), ("gL_B", ctypes.c_void_p),
                ("gm_A", ctypes.c_void_p), ("gm_B", ctypes.c_void_p)]


class EvisTuning(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("grid_mult", ctypes.c_int32), ("list_cap", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("static_tiles", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class EvisTuneTrial(ctypes.Structure):
    _fields_ = [("tuning", EvisTuning), ("ms", ctypes.c_float), ("reserved", ctypes.c_int32)]


# Every symbol include/evis.h declares, with its ctypes signature.
_VP = ctypes.c_void_p
SIGNATURES = {
    "evis_abi_version": (ctypes.c_int, []),
    "evis_create": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int]),
    "evis_destroy": (None, [_VP]),
    "evis_last_error": (ctypes.c_char_p, [_VP]),
    "evis_log_luminance": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                                          _VP, _VP]),
    "evis_log_channels": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_float, _VP, _VP]),
    "evis_voxel_grid": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                       _VP, _VP]),
    "evis_defocus_batch": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, _VP]),
    "evis_defocus": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_float, _VP, _VP]),
    "evis_state_init": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(EvisState), _VP]),
    "evis_substep_count": (ctypes.c_int, [_VP, ctypes.POINTER(EvisPair), ctypes.c_int32, _VP, _VP]),
    "evis_interpolate": (ctypes.c_int, [_VP, ctypes.POINTER(EvisPair), ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, _VP, _VP, _VP]),
    "evis_generate_events": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(EvisSensor),
                                            ctypes.POINTER(EvisState), ctypes.c_int32, _VP,
                                            ctypes.c_int64, _VP, ctypes.c_int32, _VP]),
    "evis_generate_events_noise": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                                  ctypes.POINTER(EvisSensor), ctypes.POINTER(EvisState),
                                                  ctypes.c_int32, ctypes.POINTER(EvisNoise), _VP,
                                                  ctypes.c_int64, _VP, ctypes.c_int32, _VP]),
    "evis_generate_events_batch": (ctypes.c_int, [_VP, ctypes.POINTER(EvisFrames), ctypes.c_int32, _VP,
                                                  ctypes.c_int64, _VP, ctypes.c_int32, _VP]),
    "evis_step_batch": (ctypes.c_int, [_VP, ctypes.POINTER(EvisEnv), ctypes.c_int32, _VP, ctypes.c_int64,
                                       _VP, _VP, ctypes.c_int32, _VP]),
    "evis_step_batch_noalloc": (ctypes.c_int, [_VP, ctypes.POINTER(EvisEnv), ctypes.c_int32, _VP,
                                               ctypes.c_int64, _VP, _VP, ctypes.c_int32, _VP]),
    "evis_get_tuning": (ctypes.c_int, [_VP, ctypes.POINTER(EvisTuning)]),
    "evis_set_tuning": (ctypes.c_int, [_VP, ctypes.POINTER(EvisTuning)]),
    "evis_soft_count_forward": (ctypes.c_int, [_VP, ctypes.POINTER(EvisSoftEnv), ctypes.c_int32,
                                               ctypes.c_int32, ctypes.c_float, ctypes.c_int32, _VP, _VP]),
    "evis_soft_count_backward": (ctypes.c_int, [_VP, ctypes.POINTER(EvisSoftEnv), ctypes.c_int32,
                                                ctypes.c_int32, ctypes.c_float, ctypes.c_int32, _VP, _VP,
                                                ctypes.c_int32, _VP]),
    "evis_profile_enable": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "evis_profile_read": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64)]),
    "evis_autotune": (ctypes.c_int, [_VP, ctypes.POINTER(EvisEnv), ctypes.c_int32, _VP, ctypes.c_int64,
                                     _VP, ctypes.c_int32, ctypes.POINTER(EvisTuning),
                                     ctypes.POINTER(ctypes.c_float), _VP]),
    "evis_autotune_ex": (ctypes.c_int, [_VP, ctypes.POINTER(EvisEnv), ctypes.c_int32, _VP,
                                        ctypes.c_int64, _VP, ctypes.c_int32, ctypes.c_char_p,
                                        ctypes.POINTER(EvisTuning), ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(EvisTuneTrial), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                        _VP]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libevis.so and bind every declared symbol; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libevis.so not built ({path}); run python -m paper_2607_08098_amd.build")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class EvisError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"evis error {code}: {msg}")
        self.code = code


def _is_device(t: torch.Tensor) -> bool:
    return t.is_cuda


def _ptr(t: Optional[torch.Tensor], name: str = "tensor", dtype: Optional[torch.dtype] = None,
         numel: Optional[int] = None, device=None, min_numel: Optional[int] = None):
    """Device pointer of a contiguous tensor, after checking what the kernel
    will assume of it: dtype, exact (numel) or least (min_numel) element
    count, and device.  A mismatch raises ValueError before anything is
    enqueued (a wrong size would otherwise become an out-of-bounds access)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements (shape {tuple(t.shape)}), expected {numel}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name}: {t.numel()} elements (shape {tuple(t.shape)}), "
                         f"expected at least {min_numel}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: libevis takes contiguous tensors")
    if not _is_device(t):
        raise ValueError(f"{name}: libevis takes device tensors")
    if device is not None and t.device != torch.device(device):
        raise ValueError(f"{name}: on {t.device}, expected {device}")
    return ctypes.c_void_p(t.data_ptr())


def _hw(t: torch.Tensor, name: str):
    """(H, W) of a [..., H, W] plane."""
    if not isinstance(t, torch.Tensor) or t.dim() < 2:
        raise ValueError(f"{name}: expected a tensor of shape [..., H, W]")
    return int(t.shape[-2]), int(t.shape[-1])


def _events_ptrs(out: torch.Tensor, n_total: torch.Tensor, device=None):
    """Event buffer [capacity, 2] int32 and its int64 cursor (8-byte atomics)."""
    if not isinstance(out, torch.Tensor) or out.dim() != 2 or out.shape[1] != 2:
        raise ValueError("out: expected an event buffer of shape [capacity, 2]")
    dev = device if device is not None else out.device
    return (_ptr(out, "out", torch.int32, device=dev),
            _ptr(n_total, "n_total", torch.int64, min_numel=1, device=dev))


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """Owns one evis_ctx on one device."""

    def __init__(self, device: int = 0):
        lib = load_library()
        h = ctypes.c_void_p()
        rc = lib.evis_create(ctypes.byref(h), int(device))
        if rc != EVIS_OK:
            raise EvisError(rc, "evis_create failed")
        self.handle = h
        self.device = device
        self.lib = lib

    def close(self):
        if self.handle:
            self.lib.evis_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc: int):
        if rc != EVIS_OK:
            raise EvisError(rc, self.lib.evis_last_error(self.handle).decode())
        return rc

    def last_error(self) -> str:
        return self.lib.evis_last_error(self.handle).decode()


def make_pair(d: dict) -> EvisPair:
    """L_A, L_B, Z_A, Z_B float32 [H, W]; m_A, m_B float32 [H, W, 2]; one device."""
    H, W = _hw(d["L_A"], "L_A")
    dev = d["L_A"].device
    f32 = torch.float32
    plane = lambda k: _ptr(d[k], k, f32, numel=H * W, device=dev)
    field = lambda k: _ptr(d[k], k, f32, numel=H * W * 2, device=dev)
    for k in ("m_A", "m_B"):
        if d[k].shape[-1] != 2:
            raise ValueError(f"{k}: expected shape [H, W, 2], got {tuple(d[k].shape)}")
    return EvisPair(H, W, plane("L_A"), plane("L_B"), field("m_A"), field("m_B"),
                    plane("Z_A"), plane("Z_B"), int(d.get("t0", 0)), int(d.get("t1", 16667)))


def make_sensor(d: dict, H: Optional[int] = None, W: Optional[int] = None, device=None) -> EvisSensor:
    """theta_on / theta_off (optional): float32 [H, W] per-pixel thresholds."""
    n = None if H is None else H * W
    return EvisSensor(float(d.get("C_on", 0.2)), float(d.get("C_off", 0.2)),
                      _ptr(d.get("theta_on"), "theta_on", torch.float32, numel=n, device=device),
                      _ptr(d.get("theta_off"), "theta_off", torch.float32, numel=n, device=device),
                      int(d.get("refractory_us", 0)), int(d.get("K", 0)), int(d.get("K_max", 64)),
                      int(d.get("blend_mode", EVIS_BLEND_TIME)))


def make_state(d: dict, H: Optional[int] = None, W: Optional[int] = None, device=None) -> EvisState:
    """L_ref float32 [H, W]; t_last (optional) int32 [H, W]."""
    n = None if H is None else H * W
    return EvisState(_ptr(d["L_ref"], "L_ref", torch.float32, numel=n, device=device),
                     _ptr(d.get("t_last"), "t_last", torch.int32, numel=n, device=device))


def make_noise(nz: dict) -> EvisNoise:
    """Sensor noise of one env: keys leak_rate_hz, shot_rate_hz, hot_rate_hz,
    hot_fraction, shot_L0, shot_inv_range, seed, pair_index (missing = 0,
    shot_inv_range 1)."""
    return EvisNoise(float(nz.get("leak_rate_hz", 0.0)), float(nz.get("shot_rate_hz", 0.0)),
                     float(nz.get("hot_rate_hz", 0.0)), float(nz.get("hot_fraction", 0.0)),
                     float(nz.get("shot_L0", 0.0)), float(nz.get("shot_inv_range", 1.0)),
                     int(nz.get("seed", 0)) & 0xFFFF_FFFF_FFFF_FFFF,
                     int(nz.get("pair_index", 0)) & 0xFFFF_FFFF, 0)


def make_env(d: dict, keep: Optional[list] = None) -> EvisEnv:
    """d["noise"] (optional) is a make_noise dict; the EvisNoise it becomes
    is appended to `keep`, which must outlive every call that uses the env."""
    pair = make_pair(d)
    dev = d["L_A"].device
    env = EvisEnv(pair, make_sensor(d, pair.H, pair.W, dev), make_state(d, pair.H, pair.W, dev),
                  int(d.get("env_id", 0)), int(d.get("crop_margin", 0)))
    if d.get("noise") is not None:
        nz = make_noise(d["noise"])
        if keep is None:
            raise ValueError("make_env: an env with noise needs a keep list")
        keep.append(nz)
        env.noise = ctypes.pointer(nz)
    return env


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def evis_abi_version() -> int:
    return load_library().evis_abi_version()


def evis_log_luminance(ctx: Context, x: torch.Tensor, eps: float = 1e-3, out=None, stream=None):
    channels = 3 if (x.dim() >= 1 and x.shape[-1] == 3) else 1
    n = x.numel() // channels
    shape = x.shape[:-1] if channels == 3 else x.shape
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=x.device)
    xp = _ptr(x, "x", torch.float32)
    op = _ptr(out, "out", torch.float32, numel=n, device=x.device)
    ctx.check(ctx.lib.evis_log_luminance(ctx.handle, xp, channels, n, eps, op, _stream(stream)))
    return out


def evis_log_channels(ctx: Context, x: torch.Tensor, eps: float = 1e-3, out=None, stream=None):
    """x: [..., 3] linear RGB on the device -> [3, ...] per-channel log."""
    if x.dim() < 1 or x.shape[-1] != 3:
        raise ValueError("x: expected linear RGB of shape [..., 3]")
    n = x.numel() // 3
    if out is None:
        out = torch.empty((3,) + tuple(x.shape[:-1]), dtype=torch.float32, device=x.device)
    xp = _ptr(x, "x", torch.float32)
    op = _ptr(out, "out", torch.float32, numel=3 * n, device=x.device)
    ctx.check(ctx.lib.evis_log_channels(ctx.handle, xp, n, eps, op, _stream(stream)))
    return out


def evis_voxel_grid(ctx: Context, out_events: torch.Tensor, n_total: torch.Tensor, env_id: int,
                    H: int, W: int, t0_us: int, t1_us: int, bins: int = 128, out=None, stream=None):
    """Normalised per-polarity voxel grid [2, bins, H, W] of one env's events."""
    if out is None:
        out = torch.empty((2, bins, H, W), dtype=torch.float32, device=out_events.device)
    ep, npt = _events_ptrs(out_events, n_total)
    op = _ptr(out, "out", torch.float32, numel=2 * bins * H * W, device=out_events.device)
    ctx.check(ctx.lib.evis_voxel_grid(ctx.handle, ep, npt, out_events.shape[0],
                                      env_id, H, W, t0_us, t1_us, bins, op, _stream(stream)))
    return out


class EvisImage(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("out", ctypes.c_void_p), ("H", ctypes.c_int32),
                ("W", ctypes.c_int32)]


def evis_defocus_batch(ctx: Context, pairs, sigma: float, stream=None):
    """pairs: sequence of (x, out) device tensors, each [H, W] or [H, W, 3]
    (all with the same channel count)."""
    arr = (EvisImage * len(pairs))()
    channels = None
    for i, (x, out) in enumerate(pairs):
        c = 3 if (x.dim() == 3 and x.shape[-1] == 3) else 1
        if x.dim() != (3 if c == 3 else 2):
            raise ValueError(f"image {i}: expected [H, W] or [H, W, 3], got {tuple(x.shape)}")
        if channels is not None and c != channels:
            raise ValueError("evis_defocus_batch: every image needs the same channel count")
        channels = c
        xp = _ptr(x, f"x[{i}]", torch.float32)
        op = _ptr(out, f"out[{i}]", torch.float32, numel=x.numel(), device=x.device)
        arr[i] = EvisImage(xp.value, op.value, x.shape[0], x.shape[1])
    channels = channels or 1
    ctx.check(ctx.lib.evis_defocus_batch(ctx.handle, arr, len(pairs), channels, float(sigma),
                                         _stream(stream)))


def evis_defocus(ctx: Context, x: torch.Tensor, sigma: float, out=None, stream=None):
    """x: [H, W] or [H, W, 3] float32 linear intensity on the device."""
    channels = 3 if (x.dim() == 3 and x.shape[-1] == 3) else 1
    if x.dim() != (3 if channels == 3 else 2):
        raise ValueError(f"x: expected [H, W] or [H, W, 3], got {tuple(x.shape)}")
    H, W = x.shape[0], x.shape[1]
    if out is None:
        out = torch.empty_like(x)
    xp = _ptr(x, "x", torch.float32)
    op = _ptr(out, "out", torch.float32, numel=x.numel(), device=x.device)
    ctx.check(ctx.lib.evis_defocus(ctx.handle, xp, H, W, channels, float(sigma), op,
                                   _stream(stream)))
    return out


def evis_state_init(ctx: Context, L_first: torch.Tensor, L_ref: torch.Tensor,
                    t_last: Optional[torch.Tensor] = None, stream=None):
    H, W = _hw(L_first, "L_first")
    dev = L_first.device
    lp = _ptr(L_first, "L_first", torch.float32, numel=H * W)
    st = EvisState(_ptr(L_ref, "L_ref", torch.float32, numel=H * W, device=dev),
                   _ptr(t_last, "t_last", torch.int32, numel=H * W, device=dev))
    ctx.check(ctx.lib.evis_state_init(ctx.handle, lp, H, W, ctypes.byref(st), _stream(stream)))


def evis_substep_count(ctx: Context, pair: dict, K_max: int, K_out: Optional[torch.Tensor] = None,
                       stream=None) -> torch.Tensor:
    if K_out is None:
        K_out = torch.zeros(1, dtype=torch.int32, device=pair["L_A"].device)
    p = make_pair(pair)
    kp = _ptr(K_out, "K_out", torch.int32, min_numel=1, device=pair["L_A"].device)
    ctx.check(ctx.lib.evis_substep_count(ctx.handle, ctypes.byref(p), K_max, kp, _stream(stream)))
    return K_out


def evis_interpolate(ctx: Context, pair: dict, K: int, j_begin: int, j_end: int,
                     blend_mode: int = EVIS_BLEND_TIME, L_out=None, hole_mask=None,
                     want_holes: bool = True, stream=None):
    H, W = _hw(pair["L_A"], "L_A")
    dev = pair["L_A"].device
    if L_out is None:
        L_out = torch.empty((j_end - j_begin, H, W), dtype=torch.float32, device=dev)
    if hole_mask is None and want_holes:
        hole_mask = torch.empty((j_end - j_begin, H, W), dtype=torch.uint8, device=dev)
    p = make_pair(pair)
    n = max(0, j_end - j_begin) * H * W
    lo = _ptr(L_out, "L_out", torch.float32, min_numel=n, device=dev)
    hm = _ptr(hole_mask, "hole_mask", torch.uint8, min_numel=n, device=dev)
    ctx.check(ctx.lib.evis_interpolate(ctx.handle, ctypes.byref(p), K, j_begin, j_end, blend_mode,
                                       lo, hm, _stream(stream)))
    return L_out, hole_mask


def evis_generate_events(ctx: Context, L_seq: torch.Tensor, t0: int, t1: int, sensor: dict,
                         state: dict, env_id: int, out: torch.Tensor, n_total: torch.Tensor,
                         flags: int = EVIS_FLAG_RESET_CURSOR, stream=None, noise: Optional[dict] = None):
    """noise: a make_noise dict (evis_generate_events_noise), or None."""
    if not isinstance(L_seq, torch.Tensor) or L_seq.dim() != 3:
        raise ValueError("L_seq: expected float32 samples of shape [K + 1, H, W]")
    K = L_seq.shape[0] - 1
    H, W = _hw(L_seq, "L_seq")
    dev = L_seq.device
    lp = _ptr(L_seq, "L_seq", torch.float32)
    s = make_sensor(sensor, H, W, dev)
    st = make_state(state, H, W, dev)
    op, npt = _events_ptrs(out, n_total, dev)
    if noise is None:
        ctx.check(ctx.lib.evis_generate_events(ctx.handle, lp, H, W, K, int(t0), int(t1),
                                               ctypes.byref(s), ctypes.byref(st), env_id, op,
                                               out.shape[0], npt, flags, _stream(stream)))
    else:
        nz = make_noise(noise)
        ctx.check(ctx.lib.evis_generate_events_noise(ctx.handle, lp, H, W, K, int(t0),
                                                     int(t1), ctypes.byref(s), ctypes.byref(st),
                                                     env_id, ctypes.byref(nz), op,
                                                     out.shape[0], npt, flags,
                                                     _stream(stream)))
    return n_total


def evis_generate_events_batch(ctx: Context, items: Sequence[dict], out: torch.Tensor,
                               n_total: torch.Tensor, flags: int = EVIS_FLAG_RESET_CURSOR, stream=None):
    """items: dicts with L_seq ([K + 1, H, W] float32), t0, t1, env_id, the
    sensor keys of make_sensor and the state keys of make_state."""
    arr = (EvisFrames * len(items))()
    for i, d in enumerate(items):
        L_seq = d["L_seq"]
        if not isinstance(L_seq, torch.Tensor) or L_seq.dim() != 3:
            raise ValueError(f"items[{i}].L_seq: expected float32 samples of shape [K + 1, H, W]")
        H, W = _hw(L_seq, "L_seq")
        dev = L_seq.device
        arr[i] = EvisFrames(_ptr(L_seq, "L_seq", torch.float32), H, W, L_seq.shape[0] - 1,
                            int(d.get("env_id", i)), int(d.get("t0", 0)), int(d.get("t1", 16667)),
                            make_sensor(d, H, W, dev), make_state(d, H, W, dev))
    op, npt = _events_ptrs(out, n_total)
    ctx.check(ctx.lib.evis_generate_events_batch(ctx.handle, arr, len(arr), op, out.shape[0], npt,
                                                 flags, _stream(stream)))
    return n_total


def env_array(envs: Sequence[dict]):
    """Host array of env descriptors; noise structs stay alive with it."""
    arr = (EvisEnv * len(envs))()
    arr._keep = []
    for i, d in enumerate(envs):
        arr[i] = make_env(d, arr._keep)
    return arr


def evis_step_batch(ctx: Context, envs, out: torch.Tensor, n_total: torch.Tensor,
                    K_used: Optional[torch.Tensor] = None, flags: int = EVIS_FLAG_RESET_CURSOR,
                    stream=None):
    """envs: a sequence of env dicts or a prebuilt env_array()."""
    arr = envs if isinstance(envs, ctypes.Array) else env_array(envs)
    op, npt = _events_ptrs(out, n_total)
    kp = _ptr(K_used, "K_used", torch.int32, min_numel=len(arr), device=out.device)
    ctx.check(ctx.lib.evis_step_batch(ctx.handle, arr, len(arr), op, out.shape[0],
                                      npt, kp, flags, _stream(stream)))
    return n_total


def evis_step_batch_noalloc(ctx: Context, envs, out: torch.Tensor, n_total: torch.Tensor,
                            K_used: Optional[torch.Tensor] = None, flags: int = EVIS_FLAG_RESET_CURSOR,
                            stream=None):
    """evis_step_batch with the library's static scratch (allocates nothing)."""
    arr = envs if isinstance(envs, ctypes.Array) else env_array(envs)
    op, npt = _events_ptrs(out, n_total)
    kp = _ptr(K_used, "K_used", torch.int32, min_numel=len(arr), device=out.device)
    ctx.check(ctx.lib.evis_step_batch_noalloc(ctx.handle, arr, len(arr), op, out.shape[0],
                                              npt, kp, flags, _stream(stream)))
    return n_total


def evis_get_tuning(ctx: Context) -> EvisTuning:
    t = EvisTuning()
    ctx.check(ctx.lib.evis_get_tuning(ctx.handle, ctypes.byref(t)))
    return t


def evis_set_tuning(ctx: Context, **kw) -> EvisTuning:
    t = evis_get_tuning(ctx)
    for k, v in kw.items():
        setattr(t, k, int(v))
    ctx.check(ctx.lib.evis_set_tuning(ctx.handle, ctypes.byref(t)))
    return t


def evis_autotune(ctx: Context, envs, out: torch.Tensor, n_total: torch.Tensor, reps: int = 3,
                  stream=None):
    arr = envs if isinstance(envs, ctypes.Array) else env_array(envs)
    best = EvisTuning()
    ms = ctypes.c_float()
    op, npt = _events_ptrs(out, n_total)
    ctx.check(ctx.lib.evis_autotune(ctx.handle, arr, len(arr), op, out.shape[0], npt,
                                    reps, ctypes.byref(best), ctypes.byref(ms), _stream(stream)))
    return best, ms.value


def evis_autotune_ex(ctx: Context, envs, out: torch.Tensor, n_total: torch.Tensor, reps: int = 3,
                     cache_path: Optional[str] = None, max_trials: int = 32, stream=None):
    """(best EvisTuning, its ms, [(tuning dict, ms) per trial in search order],
    from_cache) of the library's schedule search (see include/evis.h)."""
    arr = envs if isinstance(envs, ctypes.Array) else env_array(envs)
    best = EvisTuning()
    ms = ctypes.c_float()
    trials = (EvisTuneTrial * max_trials)()
    n_tr = ctypes.c_int32()
    hit = ctypes.c_int32()
    op, npt = _events_ptrs(out, n_total)
    path = None if cache_path is None else os.fsencode(cache_path)
    ctx.check(ctx.lib.evis_autotune_ex(ctx.handle, arr, len(arr), op, out.shape[0], npt, reps, path,
                                       ctypes.byref(best), ctypes.byref(ms), trials, max_trials,
                                       ctypes.byref(n_tr), ctypes.byref(hit), _stream(stream)))
    got = [(trials[i].tuning.as_dict(), trials[i].ms) for i in range(min(n_tr.value, max_trials))]
    return best, ms.value, got, bool(hit.value)


def soft_env_array(L_A, L_B, m_A, m_B, Z_A, Z_B, L_ref, S=None, gS=None, gL_A=None, gL_B=None,
                   gm_A=None, gm_B=None):
    """evis_soft_env[n] from batched tensors [n, H, W] (m: [n, H, W, 2])."""
    if not isinstance(L_A, torch.Tensor) or L_A.dim() != 3:
        raise ValueError("L_A: expected float32 planes of shape [n, H, W]")
    n, H, W = (int(v) for v in L_A.shape)
    dev = L_A.device
    arr = (EvisSoftEnv * n)()
    for name, t, per in (("L_ref", L_ref, H * W), ("S", S, H * W), ("gS", gS, H * W),
                         ("gL_A", gL_A, H * W), ("gL_B", gL_B, H * W), ("gm_A", gm_A, 2 * H * W),
                         ("gm_B", gm_B, 2 * H * W)):
        _ptr(t, name, torch.float32, numel=n * per, device=dev)
    for e in range(n):
        pair = make_pair(dict(L_A=L_A[e], L_B=L_B[e], m_A=m_A[e], m_B=m_B[e], Z_A=Z_A[e], Z_B=Z_B[e],
                              t0=0, t1=1))
        pick = lambda t: None if t is None else _ptr(t[e])
        arr[e] = EvisSoftEnv(pair, pick(L_ref), pick(S), pick(gS), pick(gL_A), pick(gL_B), pick(gm_A),
                             pick(gm_B))
    return arr


def evis_soft_count_forward(ctx: Context, envs, K: int, tau: float, blend_mode: int,
                            C: torch.Tensor, stream=None):
    cp = _ptr(C, "C", torch.float32, min_numel=len(envs))
    ctx.check(ctx.lib.evis_soft_count_forward(ctx.handle, envs, len(envs), K, tau, blend_mode, cp,
                                              _stream(stream)))


def evis_soft_count_backward(ctx: Context, envs, K: int, tau: float, blend_mode: int,
                             C: torch.Tensor, gC: torch.Tensor, flags: int = 0, stream=None):
    cp = _ptr(C, "C", torch.float32, min_numel=len(envs))
    gp = _ptr(gC, "gC", torch.float32, min_numel=len(envs), device=C.device)
    ctx.check(ctx.lib.evis_soft_count_backward(ctx.handle, envs, len(envs), K, tau, blend_mode, cp,
                                               gp, flags, _stream(stream)))


EVIS_SOFT_HOLD_REF = 1

EVIS_KERNEL_STEP = 0
EVIS_KERNEL_INTERP = 1
EVIS_KERNEL_EVENTS = 2


def evis_profile_enable(ctx: Context, enable: bool = True):
    ctx.check(ctx.lib.evis_profile_enable(ctx.handle, 1 if enable else 0))


def evis_profile_read(ctx: Context, kernel: int):
    """(summed milliseconds, launches) of the recorded launches of one kernel."""
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    ctx.check(ctx.lib.evis_profile_read(ctx.handle, kernel, ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


# ---------------------------------------------------------------------------
# event buffers
# ---------------------------------------------------------------------------

def event_buffer(capacity: int, device="cuda"):
    """(events [capacity, 2] int32 of (xyp, t_us), n_total [1] int64)."""
    return (torch.empty((capacity, 2), dtype=torch.int32, device=device),
            torch.zeros(1, dtype=torch.int64, device=device))


def decode_events(out: torch.Tensor, n_total: torch.Tensor):
    """Host int64 [N, 5] of (x, y, t, p, env) from the first min(n, capacity) records."""
    import numpy as np
    n = int(n_total.item())
    n = min(n, out.shape[0])
    rec = out[:n].cpu().numpy()
    word = rec[:, 0].astype(np.int64) & 0xFFFFFFFF
    x = word & 0x7FF
    y = (word >> 11) & 0x7FF
    p = (word >> 22) & 1
    env = (word >> 23) & 0x1FF
    return np.stack([x, y, rec[:, 1].astype(np.int64), p, env], axis=1)

"""Seeded synthetic scenes: the inputs that the event path consumes.

This module stands in for the renderer of the paper (Sec. "Problem
Formulation", Eq. 2): it produces linear radiance, backward motion vectors and
depth for keyframe pairs.  It holds none of the event path's own arithmetic
(no luminance/log transform, no splat, no gather, no crossing count); both the
CPU oracle and the GPU path take their inputs from here, so nothing in this
file may be shared with either of them beyond these arrays.

Conventions (shared contract, not method arithmetic):
  * images are row-major [H][W]; pixel centres sit at integer (x, y);
  * motion vectors are [H][W][2] float32 (dx, dy) in pixels, backward
    pointing: pixel p of keyframe B sits at p + m_B(p) in keyframe A
    (Sec. "Bidirectional Motion Vector Warping");
  * depth is float32 metres, > 0;
  * every generator takes an explicit numpy Generator (PCG64) seed.

Scene recipes (stand-ins for the paper's unavailable Isaac Sim scenes):
  * ``blob_pair``: a log-linear ramp spanning 1e-2..1e3 along a random
    direction plus 32 Gaussian blobs, depth U[0.5, 5] i.i.d.; a flow field
    (constant translation or a rotation about the image centre) plus
    N(0, 0.3^2) px noise; frame B is frame A resampled along that flow
    (bilinear, edge-clamped, in linear radiance).
  * ``disc_pair``: an 8-sector textured disc rotating in front of a static
    random-plane background (the sim-to-real disc workload, Sec.
    "Sim-to-Real Rotational Speed Estimation").
"""
from __future__ import annotations

import math

import numpy as np
from scipy import ndimage

F32 = np.float32

# Per-resolution classes of the 64-environment mixed batch.
MIXED_CLASSES = ((24, 260, 346), (24, 480, 640), (16, 720, 1280))


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _grid(H: int, W: int):
    yy, xx = np.mgrid[0:H, 0:W]
    return xx.astype(np.float64), yy.astype(np.float64)


def blob_radiance(H: int, W: int, rng: np.random.Generator, n_blobs: int = 32) -> np.ndarray:
    """Linear radiance: log-linear ramp over [1e-2, 1e3] plus Gaussian blobs.

    The ramp runs along a seeded random direction; blob amplitudes are
    log-uniform in [1e-2, 1e3], widths U[2, 12] * min(H, W) / 128 px and
    centres uniform over the image.  Returns float64 [H][W].
    """
    xx, yy = _grid(H, W)
    ang = rng.uniform(0.0, 2.0 * math.pi)
    proj = xx * math.cos(ang) + yy * math.sin(ang)
    t = (proj - proj.min()) / max(proj.max() - proj.min(), 1e-12)
    img = 10.0 ** (-2.0 + 5.0 * t)
    scale = min(H, W) / 128.0
    for _ in range(n_blobs):
        amp = 10.0 ** rng.uniform(-2.0, 3.0)
        sig = rng.uniform(2.0, 12.0) * scale
        cx = rng.uniform(0.0, W - 1.0)
        cy = rng.uniform(0.0, H - 1.0)
        r = int(math.ceil(5.0 * sig))
        x0, x1 = max(0, int(cx) - r), min(W, int(cx) + r + 2)
        y0, y1 = max(0, int(cy) - r), min(H, int(cy) + r + 2)
        if x0 >= x1 or y0 >= y1:
            continue
        dx = xx[y0:y1, x0:x1] - cx
        dy = yy[y0:y1, x0:x1] - cy
        img[y0:y1, x0:x1] += amp * np.exp(-(dx * dx + dy * dy) / (2.0 * sig * sig))
    return img


def translation_displacement(H, W, rng, mean=(2.5, -1.25), noise=0.3):
    """Content displacement A->B: a constant translation plus i.i.d. noise."""
    d = np.empty((H, W, 2), np.float64)
    d[..., 0] = mean[0]
    d[..., 1] = mean[1]
    if noise > 0:
        d += rng.normal(0.0, noise, size=(H, W, 2))
    return d


def rotation_displacement(H, W, rng, angle, noise=0.3):
    """Content displacement A->B of a rotation by ``angle`` rad about the centre."""
    xx, yy = _grid(H, W)
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    c, s = math.cos(angle), math.sin(angle)
    rx, ry = xx - cx, yy - cy
    d = np.empty((H, W, 2), np.float64)
    d[..., 0] = c * rx - s * ry - rx
    d[..., 1] = s * rx + c * ry - ry
    if noise > 0:
        d += rng.normal(0.0, noise, size=(H, W, 2))
    return d


def _resample(img: np.ndarray, sx: np.ndarray, sy: np.ndarray) -> np.ndarray:
    """Bilinear, edge-clamped resampling of a float64 image (scene synthesis)."""
    return ndimage.map_coordinates(img, [sy, sx], order=1, mode="nearest")


def blob_pair(H: int, W: int, seed: int, *, flow: str = "translate",
              omega: float | None = None, frame_rate: float = 60.0,
              noise: float = 0.3, mean=(2.5, -1.25)) -> dict:
    """One keyframe pair of the blob scene.

    ``flow='translate'``: constant ``mean`` px translation plus noise.
    ``flow='rotate'``: rotation about the image centre by omega/frame_rate rad
    (omega in rad/s, drawn U[0.5, 20] when None) plus noise.

    Both keyframes carry the same backward field m_A = m_B = -displacement
    (keyframe A reuses its own backward motion as a forward velocity).
    Frame B is frame A resampled at p + m_B(p).
    """
    rng = rng_for(seed)
    I_A = blob_radiance(H, W, rng)
    Z_A = rng.uniform(0.5, 5.0, size=(H, W))
    if flow == "translate":
        disp = translation_displacement(H, W, rng, mean=mean, noise=noise)
    elif flow == "rotate":
        if omega is None:
            omega = rng.uniform(0.5, 20.0)
        disp = rotation_displacement(H, W, rng, omega / frame_rate, noise=noise)
    else:
        raise ValueError(flow)
    m = (-disp).astype(F32)
    xx, yy = _grid(H, W)
    sx = xx + m[..., 0].astype(np.float64)
    sy = yy + m[..., 1].astype(np.float64)
    I_B = _resample(I_A, sx, sy)
    Z_B = _resample(Z_A, sx, sy)
    return dict(H=H, W=W, I_A=I_A.astype(F32), I_B=I_B.astype(F32),
                m_A=m.copy(), m_B=m.copy(),
                Z_A=Z_A.astype(F32), Z_B=Z_B.astype(F32), omega=omega)


def mixed_batch_specs(seed_base: int = 3000):
    """The 64-environment mixed-resolution batch: list of (H, W, seed)."""
    out = []
    e = 0
    for count, H, W in MIXED_CLASSES:
        for _ in range(count):
            out.append((H, W, seed_base + e))
            e += 1
    return out


def mixed_env(H: int, W: int, seed: int) -> dict:
    """One environment of the mixed batch: rotating blob scene, omega U[0.5, 20]."""
    return blob_pair(H, W, seed, flow="rotate")


def mismatch_thresholds(H: int, W: int, C: float, sigma: float, theta_min: float,
                        rng: np.random.Generator):
    """Per-pixel ON/OFF thresholds max(N(C, sigma^2), theta_min), drawn once
    (Eq. 8).  The draw is an input to the event path, not part of it."""
    on = np.maximum(rng.normal(C, sigma, size=(H, W)), theta_min).astype(F32)
    off = np.maximum(rng.normal(C, sigma, size=(H, W)), theta_min).astype(F32)
    return on, off


# ---------------------------------------------------------------------------
# Rotating disc in front of a static background.
# ---------------------------------------------------------------------------

def _value_noise(H, W, rng, cell=16.0):
    """Smooth value noise (bilinear interpolation of a random lattice)."""
    gh, gw = int(H / cell) + 3, int(W / cell) + 3
    lat = rng.uniform(0.0, 1.0, size=(gh, gw))
    xx, yy = _grid(H, W)
    return ndimage.map_coordinates(lat, [yy / cell, xx / cell], order=1, mode="nearest")


def disc_scene_params(H: int, W: int, seed: int):
    rng = rng_for(seed)
    albedo = 10.0 ** rng.uniform(math.log10(0.05), 0.0, size=8)
    omega = rng.uniform(1.0, 40.0)
    phase = rng.uniform(0.0, 2.0 * math.pi)
    bg = 0.05 + 0.95 * _value_noise(H, W, rng)
    return dict(albedo=albedo, omega=omega, phase=phase, bg=bg)


def disc_frame(H: int, W: int, params: dict, t: float, frame_rate: float = 60.0,
               irradiance: float = 100.0):
    """Radiance, backward MV and depth of the disc scene at time t (seconds).

    Disc: radius 0.6 * min(H, W) / 2 px, centred, 8 equal sectors, depth 1 m,
    rotating at omega rad/s.  Background: static value-noise plane at 3 m.
    The backward MV of a disc pixel rotates it back by omega/frame_rate.
    """
    xx, yy = _grid(H, W)
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    rad = 0.6 * min(H, W) / 2.0
    rx, ry = xx - cx, yy - cy
    inside = rx * rx + ry * ry <= rad * rad
    ang = np.arctan2(ry, rx) - (params["phase"] + params["omega"] * t)
    sector = np.floor(np.mod(ang, 2.0 * math.pi) / (2.0 * math.pi / 8.0)).astype(np.int64) % 8
    img = np.where(inside, params["albedo"][sector], params["bg"]) * irradiance
    Z = np.where(inside, 1.0, 3.0)
    th = -params["omega"] / frame_rate
    c, s = math.cos(th), math.sin(th)
    mx = np.where(inside, c * rx - s * ry - rx, 0.0)
    my = np.where(inside, s * rx + c * ry - ry, 0.0)
    m = np.stack([mx, my], axis=-1).astype(F32)
    return img.astype(F32), m, Z.astype(F32)


def disc_pair(H: int, W: int, seed: int, step: int = 0, frame_rate: float = 60.0) -> dict:
    p = disc_scene_params(H, W, seed)
    I_A, m_A, Z_A = disc_frame(H, W, p, step / frame_rate, frame_rate)
    I_B, m_B, Z_B = disc_frame(H, W, p, (step + 1) / frame_rate, frame_rate)
    return dict(H=H, W=W, I_A=I_A, I_B=I_B, m_A=m_A, m_B=m_B, Z_A=Z_A, Z_B=Z_B,
                omega=p["omega"])


def frame_time_us(i: int, frame_rate: float = 60.0) -> int:
    """Keyframe i's timestamp in integer microseconds: round(i * 1e6 / rate)."""
    return int(round(i * 1e6 / frame_rate))

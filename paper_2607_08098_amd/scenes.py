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


class RotatingSequence:
    """A sequence of keyframes of the rotating blob scene (the benchmark's
    mixed batch advanced frame by frame).

    Keyframe 0 draws its radiance and depth exactly as ``blob_pair(flow=
    'rotate')`` draws keyframe A (same seed, same draws in the same order,
    then omega); keyframe i is that content turned by i * omega / frame_rate
    rad about the image centre, resampled from keyframe 0 once (bilinear,
    edge-clamped, float64), so no resampling error accumulates along the
    sequence.  Each keyframe carries its own backward motion field towards
    keyframe i - 1: the exact rotation back by one frame plus fresh
    N(0, noise^2) px noise per keyframe (the renderer's motion-vector error),
    drawn from PCG64 seeded with (seed, i).  A pair (i, i + 1) uses
    m_A = keyframe i's field and m_B = keyframe i + 1's.
    """

    def __init__(self, H: int, W: int, seed: int, frame_rate: float = 60.0, noise: float = 0.3,
                 theta: float | None = None):
        rng = rng_for(seed)
        self.H, self.W, self.seed, self.noise = H, W, seed, noise
        self.base = blob_radiance(H, W, rng)
        self.Z0 = rng.uniform(0.5, 5.0, size=(H, W))
        self.omega = float(rng.uniform(0.5, 20.0))
        # theta: the turn per keyframe (rad); by default omega / frame_rate
        self.theta = self.omega / frame_rate if theta is None else float(theta)

    def _turned(self, img: np.ndarray, angle: float) -> np.ndarray:
        """img turned by `angle` rad about the centre: out(p) = img(R(-angle)(p - c) + c)."""
        xx, yy = _grid(self.H, self.W)
        cx, cy = (self.W - 1) / 2.0, (self.H - 1) / 2.0
        c, s = math.cos(angle), math.sin(angle)
        rx, ry = xx - cx, yy - cy
        return _resample(img, c * rx + s * ry + cx, -s * rx + c * ry + cy)

    def keyframe(self, i: int):
        """(radiance float32 [H][W], backward motion float32 [H][W][2] towards
        keyframe i - 1, depth float32 [H][W]) of keyframe i."""
        a = i * self.theta
        I = self._turned(self.base, a)
        Z = self._turned(self.Z0, a)
        xx, yy = _grid(self.H, self.W)
        cx, cy = (self.W - 1) / 2.0, (self.H - 1) / 2.0
        c, s = math.cos(self.theta), math.sin(self.theta)
        rx, ry = xx - cx, yy - cy
        m = np.empty((self.H, self.W, 2), np.float64)
        m[..., 0] = c * rx + s * ry - rx
        m[..., 1] = -s * rx + c * ry - ry
        if self.noise > 0:
            m += np.random.Generator(np.random.PCG64([self.seed, i])).normal(
                0.0, self.noise, size=(self.H, self.W, 2))
        return I.astype(F32), m.astype(F32), Z.astype(F32)


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


class DiscScene:
    """The disc scene of one env with its time-independent parts computed
    once (pixel angles, disc mask, motion, depth); ``frame(t)`` gives the
    radiance at time t.  ``disc_frame`` is the one-call form."""

    def __init__(self, H: int, W: int, params: dict, frame_rate: float = 60.0,
                 irradiance: float = 100.0):
        self.H, self.W, self.params, self.irradiance = H, W, params, irradiance
        xx, yy = _grid(H, W)
        cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
        rad = 0.6 * min(H, W) / 2.0
        rx, ry = xx - cx, yy - cy
        self.inside = rx * rx + ry * ry <= rad * rad
        self.ang0 = np.arctan2(ry, rx)
        th = -params["omega"] / frame_rate
        c, s = math.cos(th), math.sin(th)
        mx = np.where(self.inside, c * rx - s * ry - rx, 0.0)
        my = np.where(self.inside, s * rx + c * ry - ry, 0.0)
        self.m = np.stack([mx, my], axis=-1).astype(F32)
        self.Z = np.where(self.inside, 1.0, 3.0).astype(F32)

    def frame(self, t: float) -> np.ndarray:
        p = self.params
        ang = self.ang0 - (p["phase"] + p["omega"] * t)
        sector = np.floor(np.mod(ang, 2.0 * math.pi) / (2.0 * math.pi / 8.0)).astype(np.int64) % 8
        img = np.where(self.inside, p["albedo"][sector], p["bg"]) * self.irradiance
        return img.astype(F32)


def disc_frame(H: int, W: int, params: dict, t: float, frame_rate: float = 60.0,
               irradiance: float = 100.0):
    """Radiance, backward MV and depth of the disc scene at time t (seconds).

    Disc: radius 0.6 * min(H, W) / 2 px, centred, 8 equal sectors, depth 1 m,
    rotating at omega rad/s.  Background: static value-noise plane at 3 m.
    The backward MV of a disc pixel rotates it back by omega/frame_rate.
    """
    sc = DiscScene(H, W, params, frame_rate, irradiance)
    return sc.frame(t), sc.m, sc.Z


def disc_pair(H: int, W: int, seed: int, step: int = 0, frame_rate: float = 60.0) -> dict:
    p = disc_scene_params(H, W, seed)
    I_A, m_A, Z_A = disc_frame(H, W, p, step / frame_rate, frame_rate)
    I_B, m_B, Z_B = disc_frame(H, W, p, (step + 1) / frame_rate, frame_rate)
    return dict(H=H, W=W, I_A=I_A, I_B=I_B, m_A=m_A, m_B=m_B, Z_A=Z_A, Z_B=Z_B,
                omega=p["omega"])


def frame_time_us(i: int, frame_rate: float = 60.0) -> int:
    """Keyframe i's timestamp in integer microseconds: round(i * 1e6 / rate)."""
    return int(round(i * 1e6 / frame_rate))


# ---------------------------------------------------------------------------
# Textured planes seen by a moving pinhole camera (exact flow and depth).
# ---------------------------------------------------------------------------

def _perlin_table(rng: np.random.Generator) -> np.ndarray:
    p = rng.permutation(256).astype(np.int64)
    return np.concatenate([p, p])


def _perlin2(u: np.ndarray, v: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """2-D gradient noise after Perlin's improved noise (quintic fade, hashed
    gradient directions); about [-1, 1]."""
    fu, fv = np.floor(u), np.floor(v)
    xi = fu.astype(np.int64) & 255
    yi = fv.astype(np.int64) & 255
    xf, yf = u - fu, v - fv
    fade = lambda t: t * t * t * (t * (t * 6.0 - 15.0) + 10.0)
    dirs = np.array([[1, 1], [-1, 1], [1, -1], [-1, -1], [1, 0], [-1, 0], [0, 1], [0, -1]], np.float64)

    def grad(h, x, y):
        g = dirs[h & 7]
        return g[..., 0] * x + g[..., 1] * y

    aa = perm[perm[xi] + yi]
    ba = perm[perm[xi + 1] + yi]
    ab = perm[perm[xi] + yi + 1]
    bb = perm[perm[xi + 1] + yi + 1]
    wu, wv = fade(xf), fade(yf)
    x1 = grad(aa, xf, yf) + wu * (grad(ba, xf - 1.0, yf) - grad(aa, xf, yf))
    x2 = grad(ab, xf, yf - 1.0) + wu * (grad(bb, xf - 1.0, yf - 1.0) - grad(ab, xf, yf - 1.0))
    return x1 + wv * (x2 - x1)


def _rodrigues(w: np.ndarray) -> np.ndarray:
    th = float(np.linalg.norm(w))
    if th < 1e-12:
        return np.eye(3)
    k = w / th
    Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(th) * Kx + (1 - math.cos(th)) * (Kx @ Kx)


class PlaneScene:
    """Twelve textured planes (one background plane at 8 m plus 11 rectangles
    at depth U[0.3, 8] m, normals within 30 degrees of the optical axis),
    each with its own gradient-noise albedo in [0.05, 1] and irradiance
    10^U[-3, 3] (six decades), seen by a pinhole camera (f = 500 px, centre
    at the image middle) on a 6-DoF random walk (angular-velocity steps
    N(0, 0.5^2) rad/s and linear-velocity steps N(0, 0.2^2) m/s per frame);
    three of the rectangles also move rigidly on random walks of their own.
    Depth is the camera-space z of the first hit; motion vectors project
    the same material point at the other keyframe exactly."""

    def __init__(self, H: int, W: int, seed: int, n_frames: int, frame_rate: float = 60.0,
                 focal: float = 500.0):
        rng = rng_for(seed)
        self.H, self.W, self.f = H, W, focal
        self.cx, self.cy = (W - 1) / 2.0, (H - 1) / 2.0
        self.frame_rate = frame_rate
        dt = 1.0 / frame_rate
        planes = []
        for i in range(12):
            if i == 0:
                c, n, half = np.array([0.0, 0.0, 8.0]), np.array([0.0, 0.0, -1.0]), (1e9, 1e9)
            else:
                z = rng.uniform(0.3, 8.0)
                x = rng.uniform(-0.5, 0.5) * z * W / focal
                y = rng.uniform(-0.5, 0.5) * z * H / focal
                c = np.array([x, y, z])
                tilt = math.radians(rng.uniform(0.0, 30.0))
                az = rng.uniform(0.0, 2.0 * math.pi)
                n = np.array([math.sin(tilt) * math.cos(az), math.sin(tilt) * math.sin(az), -math.cos(tilt)])
                s = z * min(H, W) / focal
                half = (rng.uniform(0.1, 0.4) * s, rng.uniform(0.1, 0.4) * s)
            u = np.cross(n, [0.0, 1.0, 0.0])
            u /= np.linalg.norm(u)
            v = np.cross(n, u)
            planes.append(dict(c=c, R=np.stack([u, v, n], axis=1), half=half,
                               perm=_perlin_table(rng), freq=rng.uniform(4.0, 12.0),
                               irr=10.0 ** rng.uniform(-3.0, 3.0), moving=i in (1, 2, 3)))
        self.planes = planes
        # poses per frame: camera (R, o) and the moving planes (R, c)
        Rc, oc = np.eye(3), np.zeros(3)
        wc, vc = np.zeros(3), np.zeros(3)
        self.cam = []
        pl_state = {i: (planes[i]["R"].copy(), planes[i]["c"].copy(), np.zeros(3), np.zeros(3))
                    for i in range(12) if planes[i]["moving"]}
        self.pl_pose = []
        for k in range(n_frames + 1):
            self.cam.append((Rc.copy(), oc.copy()))
            self.pl_pose.append({i: (s[0].copy(), s[1].copy()) for i, s in pl_state.items()})
            wc = wc + rng.normal(0.0, 0.5, 3)
            vc = vc + rng.normal(0.0, 0.2, 3)
            Rc = Rc @ _rodrigues(wc * dt)
            oc = oc + Rc @ (vc * dt)
            for i, (Rp, cp, wp, vp) in list(pl_state.items()):
                wp = wp + rng.normal(0.0, 0.5, 3)
                vp = vp + rng.normal(0.0, 0.2, 3)
                pl_state[i] = (_rodrigues(wp * dt) @ Rp, cp + vp * dt, wp, vp)

    def _plane_pose(self, i: int, k: int):
        p = self.planes[i]
        if p["moving"]:
            return self.pl_pose[k][i]
        return p["R"], p["c"]

    def _hit(self, k: int):
        """First hit per pixel at frame k: plane index, local (u, v), depth."""
        H, W = self.H, self.W
        yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
        d_cam = np.stack([(xx - self.cx) / self.f, (yy - self.cy) / self.f, np.ones_like(xx)], -1)
        Rc, oc = self.cam[k]
        d = d_cam @ Rc.T
        best = np.full((H, W), np.inf)
        idx = np.zeros((H, W), np.int64)
        uu = np.zeros((H, W))
        vv = np.zeros((H, W))
        for i, p in enumerate(self.planes):
            Rp, cp = self._plane_pose(i, k)
            n = Rp[:, 2]
            den = d @ n
            with np.errstate(divide="ignore", invalid="ignore"):
                t = ((cp - oc) @ n) / den
            X = oc + t[..., None] * d
            lu = (X - cp) @ Rp[:, 0]
            lv = (X - cp) @ Rp[:, 1]
            ok = (t > 1e-3) & (np.abs(lu) <= p["half"][0]) & (np.abs(lv) <= p["half"][1]) & (t < best)
            best = np.where(ok, t, best)
            idx = np.where(ok, i, idx)
            uu = np.where(ok, lu, uu)
            vv = np.where(ok, lv, vv)
        return idx, uu, vv, best

    def _project(self, i, uu, vv, k):
        """Pixel position at frame k of material point (u, v) of plane i."""
        Rp, cp = self._plane_pose(i, k)
        X = cp + uu[..., None] * Rp[:, 0] + vv[..., None] * Rp[:, 1]
        Rc, oc = self.cam[k]
        Xc = (X - oc) @ Rc
        z = np.maximum(Xc[..., 2], 1e-3)
        return self.f * Xc[..., 0] / z + self.cx, self.f * Xc[..., 1] / z + self.cy

    def frame(self, k: int, other: int):
        """Radiance, motion vectors towards keyframe `other` and depth of frame k.

        With other = k + 1 the field is A's m_A(p) = p - p_B; with
        other = k - 1 it is B's backward m_B(p) = p_A - p.
        """
        idx, uu, vv, Z = self._hit(k)
        img = np.zeros((self.H, self.W))
        px = np.zeros((self.H, self.W))
        py = np.zeros((self.H, self.W))
        for i, p in enumerate(self.planes):
            sel = idx == i
            if not sel.any():
                continue
            n = _perlin2(uu[sel] * p["freq"], vv[sel] * p["freq"], p["perm"])
            alb = np.clip(0.525 + 0.475 * n, 0.05, 1.0)
            img[sel] = alb * p["irr"]
            qx, qy = self._project(i, uu[sel], vv[sel], other)
            px[sel], py[sel] = qx, qy
        yy, xx = np.mgrid[0:self.H, 0:self.W].astype(np.float64)
        if other > k:
            m = np.stack([xx - px, yy - py], -1)
        else:
            m = np.stack([px - xx, py - yy], -1)
        return img.astype(F32), m.astype(F32), np.where(np.isfinite(Z), Z, 8.0).astype(F32)

    def pair(self, k: int) -> dict:
        """Keyframes k (A) and k + 1 (B)."""
        I_A, m_A, Z_A = self.frame(k, k + 1)
        I_B, m_B, Z_B = self.frame(k + 1, k)
        return dict(H=self.H, W=self.W, I_A=I_A, I_B=I_B, m_A=m_A, m_B=m_B, Z_A=Z_A, Z_B=Z_B)

    def keyframe(self, k: int):
        """Keyframe k with both of its fields, one ray cast: (radiance, the
        field towards k + 1 (its m_A as keyframe A; None at the last
        keyframe), the field towards k - 1 (its m_B as keyframe B; None at
        k = 0), depth), each equal to what frame(k, k + 1) and
        frame(k, k - 1) return."""
        idx, uu, vv, Z = self._hit(k)
        img = np.zeros((self.H, self.W))
        nxt = [np.zeros((self.H, self.W)), np.zeros((self.H, self.W))]
        prv = [np.zeros((self.H, self.W)), np.zeros((self.H, self.W))]
        for i, p in enumerate(self.planes):
            sel = idx == i
            if not sel.any():
                continue
            n = _perlin2(uu[sel] * p["freq"], vv[sel] * p["freq"], p["perm"])
            img[sel] = np.clip(0.525 + 0.475 * n, 0.05, 1.0) * p["irr"]
            if k + 1 < len(self.cam):
                qx, qy = self._project(i, uu[sel], vv[sel], k + 1)
                nxt[0][sel], nxt[1][sel] = qx, qy
            if k > 0:
                qx, qy = self._project(i, uu[sel], vv[sel], k - 1)
                prv[0][sel], prv[1][sel] = qx, qy
        yy, xx = np.mgrid[0:self.H, 0:self.W].astype(np.float64)
        m_next = np.stack([xx - nxt[0], yy - nxt[1]], -1).astype(F32) if k + 1 < len(self.cam) else None
        m_prev = np.stack([prv[0] - xx, prv[1] - yy], -1).astype(F32) if k > 0 else None
        return img.astype(F32), m_next, m_prev, np.where(np.isfinite(Z), Z, 8.0).astype(F32)


def render_keyframes(scene: "PlaneScene", ks, threads: int = 16) -> list:
    """scene.keyframe(k) for every k of ks, on `threads` Python threads.

    The ray casts are small matrix products.  Multithreaded OpenBLAS called
    from several Python threads at once has returned different motion
    fields from one call to the next, so the threads run with BLAS held to
    one thread each (a product's elements are the same dot products at any
    thread count, so the frames equal those of a sequential rendering)."""
    from concurrent.futures import ThreadPoolExecutor
    ks = list(ks)
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:   # without it: one at a time
        return [scene.keyframe(k) for k in ks]
    with threadpool_limits(1), ThreadPoolExecutor(max(1, threads)) as pool:
        return list(pool.map(scene.keyframe, ks))

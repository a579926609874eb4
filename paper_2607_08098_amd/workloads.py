"""Device-resident synthetic workloads for the benchmark and the tests.

Every environment's frames live in packed device buffers (one per field),
so that the log front end runs as a single launch over all environments and
each env's tensors are contiguous views.  Scene content comes from
``scenes``; log intensity comes either from ``log_fn`` (a host function,
used by tests so both sides see the same numbers) or from the library's own
``evis_log_luminance`` on the device.
"""
from __future__ import annotations

import math
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import evis, scenes


class Batch:
    """Packed device frames of n environments plus their per-env views."""

    def __init__(self, shapes: Sequence[Tuple[int, int]], device="cuda"):
        self.shapes = list(shapes)
        self.device = device
        self.offsets = [0]
        for H, W in self.shapes:
            self.offsets.append(self.offsets[-1] + H * W)
        n = self.offsets[-1]
        f32 = dict(dtype=torch.float32, device=device)
        self.I_A = torch.empty(n, **f32)
        self.I_B = torch.empty(n, **f32)
        self.L_A = torch.empty(n, **f32)
        self.L_B = torch.empty(n, **f32)
        self.m_A = torch.empty((n, 2), **f32)
        self.m_B = torch.empty((n, 2), **f32)
        self.Z_A = torch.empty(n, **f32)
        self.Z_B = torch.empty(n, **f32)
        self.L_ref = torch.empty(n, **f32)
        self.t_last: Optional[torch.Tensor] = None
        self.omega: List[float] = []

    @property
    def n_px(self) -> int:
        return self.offsets[-1]

    def view(self, buf: torch.Tensor, e: int) -> torch.Tensor:
        H, W = self.shapes[e]
        a, b = self.offsets[e], self.offsets[e + 1]
        return buf[a:b].view(H, W, *buf.shape[1:])

    def env_dicts(self, sensor: dict, t0: int = 0, t1: int = 16667, env_ids=None) -> List[dict]:
        out = []
        for e in range(len(self.shapes)):
            d = dict(L_A=self.view(self.L_A, e), L_B=self.view(self.L_B, e),
                     m_A=self.view(self.m_A, e), m_B=self.view(self.m_B, e),
                     Z_A=self.view(self.Z_A, e), Z_B=self.view(self.Z_B, e),
                     L_ref=self.view(self.L_ref, e), t0=t0, t1=t1,
                     env_id=e if env_ids is None else env_ids[e])
            if self.t_last is not None:
                d["t_last"] = self.view(self.t_last, e)
            d.update(sensor)
            out.append(d)
        return out


def mixed_batch(ctx: evis.Context, seed_base: int = 3000, device="cuda",
                log_fn: Optional[Callable[[np.ndarray], np.ndarray]] = None,
                specs=None) -> Batch:
    """The 64-environment mixed-resolution batch (24 x 346x260, 24 x 640x480,
    16 x 1280x720) of rotating blob scenes, omega U[0.5, 20] rad/s at 60 Hz.
    L_ref starts at L_A."""
    specs = specs if specs is not None else scenes.mixed_batch_specs(seed_base)
    b = Batch([(H, W) for H, W, _ in specs], device)
    for e, (H, W, seed) in enumerate(specs):
        sc = scenes.mixed_env(H, W, seed)
        b.omega.append(float(sc["omega"]))
        put = lambda buf, arr: b.view(buf, e).copy_(torch.from_numpy(np.ascontiguousarray(arr)))
        put(b.I_A, sc["I_A"])
        put(b.I_B, sc["I_B"])
        put(b.m_A, sc["m_A"])
        put(b.m_B, sc["m_B"])
        put(b.Z_A, sc["Z_A"])
        put(b.Z_B, sc["Z_B"])
        if log_fn is not None:
            put(b.L_A, log_fn(sc["I_A"]).astype(np.float32))
            put(b.L_B, log_fn(sc["I_B"]).astype(np.float32))
    if log_fn is None:
        evis.evis_log_luminance(ctx, b.I_A, 1e-3, out=b.L_A)
        evis.evis_log_luminance(ctx, b.I_B, 1e-3, out=b.L_B)
    for e in range(len(b.shapes)):
        H, W = b.shapes[e]
        evis.evis_state_init(ctx, b.view(b.L_A, e), b.view(b.L_ref, e))
    return b


class DiscBatch(Batch):
    """n copies of the rotating-disc scene (``scenes.disc_scene_params``, one
    seed per env) at one resolution, advanced frame by frame on the device.

    Motion vectors and depth of this scene do not change over time; only
    the radiance does (the sector pattern turns), so each step generates
    the next keyframe's radiance with torch on the device and takes its log
    intensity with the library's own front end.  Frame i is at i / 60 s.
    """

    def __init__(self, ctx: evis.Context, n_envs: int = 512, H: int = 260, W: int = 346,
                 seed_base: int = 4000, device="cuda", frame_rate: float = 60.0):
        super().__init__([(H, W)] * n_envs, device)
        self.ctx = ctx
        self.frame_rate = frame_rate
        self.H, self.W, self.n = H, W, n_envs
        f64 = dict(dtype=torch.float64, device=device)
        albedo, omega, phase, bg = [], [], [], []
        for e in range(n_envs):
            p = scenes.disc_scene_params(H, W, seed_base + e)
            albedo.append(p["albedo"])
            omega.append(p["omega"])
            phase.append(p["phase"])
            bg.append(p["bg"])
        self.omega = [float(w) for w in omega]
        self.albedo = torch.tensor(np.stack(albedo), **f64)             # [n, 8]
        self.w = torch.tensor(omega, **f64).view(n_envs, 1, 1)
        self.phase = torch.tensor(phase, **f64).view(n_envs, 1, 1)
        self.bg = torch.tensor(np.stack(bg), **f64)                      # [n, H, W]
        yy, xx = torch.meshgrid(torch.arange(H, **f64), torch.arange(W, **f64), indexing="ij")
        rx, ry = xx - (W - 1) / 2.0, yy - (H - 1) / 2.0
        rad = 0.6 * min(H, W) / 2.0
        self.inside = (rx * rx + ry * ry <= rad * rad)
        self.ang0 = torch.atan2(ry, rx)
        # static motion (the backward rotation of one frame) and depth, per env
        for e in range(n_envs):
            _, m, Z = scenes.disc_frame(H, W, dict(albedo=albedo[e], omega=omega[e], phase=phase[e],
                                                   bg=bg[e]), 0.0, frame_rate)
            mt = torch.from_numpy(np.ascontiguousarray(m))
            zt = torch.from_numpy(np.ascontiguousarray(Z))
            self.view(self.m_A, e).copy_(mt)
            self.view(self.m_B, e).copy_(mt)
            self.view(self.Z_A, e).copy_(zt)
            self.view(self.Z_B, e).copy_(zt)
        self.frame = -1

    def radiance(self, i: int, out: torch.Tensor) -> None:
        """Linear radiance of every env at frame i into out [n * H * W]."""
        t = i / self.frame_rate
        ang = self.ang0.unsqueeze(0) - (self.phase + self.w * t)
        two_pi = 2.0 * math.pi
        sector = torch.floor(torch.remainder(ang, two_pi) / (two_pi / 8.0)).long() % 8
        a = torch.gather(self.albedo, 1, sector.view(self.n, -1)).view(self.n, self.H, self.W)
        img = torch.where(self.inside.unsqueeze(0), a, self.bg) * 100.0
        out.view(self.n, self.H, self.W).copy_(img.to(torch.float32))

    def start(self, i: int = 0) -> None:
        """Keyframes i, i + 1 as L_A, L_B; L_ref = L_A; no refractory state."""
        self.radiance(i, self.I_A)
        self.radiance(i + 1, self.I_B)
        evis.evis_log_luminance(self.ctx, self.I_A, 1e-3, out=self.L_A)
        evis.evis_log_luminance(self.ctx, self.I_B, 1e-3, out=self.L_B)
        for e in range(self.n):
            evis.evis_state_init(self.ctx, self.view(self.L_A, e), self.view(self.L_ref, e))
        self.frame = i

    def advance(self) -> None:
        """Move one keyframe on: L_A <- L_B, L_B <- log of the next frame
        (buffers keep their addresses, so descriptors stay the same)."""
        self.frame += 1
        self.L_A.copy_(self.L_B)
        self.radiance(self.frame + 1, self.I_B)
        evis.evis_log_luminance(self.ctx, self.I_B, 1e-3, out=self.L_B)

    def times(self) -> Tuple[int, int]:
        return scenes.frame_time_us(self.frame, self.frame_rate), \
            scenes.frame_time_us(self.frame + 1, self.frame_rate)


class MixedSequence:
    """The 64-environment mixed batch as a sequence of keyframes resident in
    device memory: keyframe i of env e is ``scenes.RotatingSequence``'s
    keyframe i (radiance, its own backward motion field, depth), so a step
    takes the pair (i, i + 1) of every env, at times i / 60 s and
    (i + 1) / 60 s, and the reference level carries over from one pair to
    the next as in a rendered sequence.

    Layout: one packed allocation per field and keyframe ([n_kf][n_px] for
    radiance, log intensity and depth, [n_kf][n_px][2] for motion), so the
    log front end of one keyframe is one launch over all envs and every
    env's planes are contiguous views.  Keyframes are generated on the host
    by a thread pool and copied once; log intensity comes either from
    ``log_fn`` (a host function: tests feed both sides the same numbers) or
    from the library's own front end (``log_keyframe``).
    """

    def __init__(self, ctx: evis.Context, n_keyframes: int, specs=None, device="cuda",
                 log_fn: Optional[Callable[[np.ndarray], np.ndarray]] = None, threads: int = 16,
                 seq_kw: Optional[Callable[[int, int, int], dict]] = None):
        """seq_kw(e, H, W) (optional): extra RotatingSequence arguments of env e."""
        from concurrent.futures import ThreadPoolExecutor
        self.ctx = ctx
        self.specs = specs if specs is not None else scenes.mixed_batch_specs(3000)
        self.shapes = [(H, W) for H, W, _ in self.specs]
        self.n_envs = len(self.specs)
        self.n_kf = int(n_keyframes)
        self.offsets = [0]
        for H, W in self.shapes:
            self.offsets.append(self.offsets[-1] + H * W)
        n = self.offsets[-1]
        f32 = dict(dtype=torch.float32, device=device)
        self.I = torch.empty((self.n_kf, n), **f32)
        self.L = torch.empty((self.n_kf, n), **f32)
        self.m = torch.empty((self.n_kf, n, 2), **f32)
        self.Z = torch.empty((self.n_kf, n), **f32)
        self.L_ref = torch.empty(n, **f32)
        self.t_last: Optional[torch.Tensor] = None
        seqs = [scenes.RotatingSequence(H, W, seed, **(seq_kw(e, H, W) if seq_kw else {}))
                for e, (H, W, seed) in enumerate(self.specs)]
        self.omega = [s.omega for s in seqs]

        def make(task):
            e, i = task
            I, m, Z = seqs[e].keyframe(i)
            L = log_fn(I).astype(np.float32) if log_fn is not None else None
            return e, i, I, m, Z, L

        tasks = [(e, i) for i in range(self.n_kf) for e in range(self.n_envs)]
        with ThreadPoolExecutor(max(1, threads)) as ex:
            for e, i, I, m, Z, L in ex.map(make, tasks):
                a, b = self.offsets[e], self.offsets[e + 1]
                self.I[i, a:b].copy_(torch.from_numpy(I.reshape(-1)))
                self.m[i, a:b].copy_(torch.from_numpy(m.reshape(-1, 2)))
                self.Z[i, a:b].copy_(torch.from_numpy(Z.reshape(-1)))
                if L is not None:
                    self.L[i, a:b].copy_(torch.from_numpy(L.reshape(-1)))
        if log_fn is None:
            for i in range(self.n_kf):
                self.log_keyframe(i)

    @property
    def n_px(self) -> int:
        return self.offsets[-1]

    def view(self, buf: torch.Tensor, e: int) -> torch.Tensor:
        H, W = self.shapes[e]
        a, b = self.offsets[e], self.offsets[e + 1]
        return buf[..., a:b, :].view(H, W, 2) if buf.dim() == 2 and buf.shape[-1] == 2 \
            else buf[a:b].view(H, W)

    def log_keyframe(self, i: int) -> None:
        """Log intensity of keyframe i of every env: one launch of the library's a1."""
        evis.evis_log_luminance(self.ctx, self.I[i], 1e-3, out=self.L[i])

    def reset_state(self, i: int = 0) -> None:
        """L_ref = keyframe i's log intensity (every env)."""
        for e in range(self.n_envs):
            evis.evis_state_init(self.ctx, self.view(self.L[i], e), self.view(self.L_ref, e))

    def times(self, i: int) -> Tuple[int, int]:
        return scenes.frame_time_us(i), scenes.frame_time_us(i + 1)

    def env_dicts(self, i: int, sensor: dict) -> List[dict]:
        """Env dicts of the pair (i, i + 1)."""
        t0, t1 = self.times(i)
        out = []
        for e in range(self.n_envs):
            d = dict(L_A=self.view(self.L[i], e), L_B=self.view(self.L[i + 1], e),
                     m_A=self.view(self.m[i], e), m_B=self.view(self.m[i + 1], e),
                     Z_A=self.view(self.Z[i], e), Z_B=self.view(self.Z[i + 1], e),
                     L_ref=self.view(self.L_ref, e), t0=t0, t1=t1, env_id=e)
            if self.t_last is not None:
                d["t_last"] = self.view(self.t_last, e)
            d.update(sensor)
            out.append(d)
        return out

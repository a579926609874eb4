"""CPU oracle of EVIS's per-frame event-generation path.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The HIP library and its
Python binding never import, call or link anything here, and this file uses
nothing from them.

Paper: "EVIS: Real-Time Event Camera Simulation with Multimodal Supervision
in NVIDIA Isaac Sim".  Steps, in the paper's order:

  defocus                the optional defocus of Sec. "Sensor Calibration
                         and Non-idealities": a separable Gaussian blur of
                         the linear intensity before the log (R24)
  log_luminance          Sec. "HDR Event Formation Model", Eq. 3 and the
                         log-intensity definition that follows it
  log_channels           the colour-event variant: each of R, G, B in place
                         of the luminance (same section)
  adaptive_k             Sec. "Bidirectional Motion Vector Warping": K-1
                         intermediate frames per keyframe gap, K chosen so
                         that no pixel moves more than one px per substep
  endpoint_depth         Eq. 7, depth at the B-side endpoint of A's motion
  splat_forward          Eq. 5 (q_A), the bilinear footprint, Eq. 6 z-buffer,
                         Eq. 7 intermediate depth
  resolve_gather_blend   Eq. 5 (q_B) evaluated as a backward gather, the
                         hole-aware blend of A and B
  start_depth,           the two-splat warp: B splatted backward to Eq. 5's
  splat_backward,        q_B with its own z-buffer (or one z-buffer shared
  resolve_two_splat      with A's splat, Eq. 6 over both keyframes) and
                         the same hole-aware blend
  emit_events            Eq. 4 (crossing count, polarity, residual-keeping
                         reference update), Eq. 8 threshold mismatch, the
                         refractory period of Sec. "Sensor Calibration and
                         Non-idealities"
  noise_events           leak events, shot noise and hot pixels of Sec.
                         "Sensor Calibration and Non-idealities", drawn
                         from a Philox4x32-10 counter-based generator
  pack_events            the (x, y, t, p) event tuple of Sec. "Problem
                         Formulation" as an 8-byte record
  voxel_grid             the per-polarity event voxel grid of the speed
                         estimation experiment (128 temporal bins, linear
                         interpolation in time, each bin divided by its
                         maximum; R26)
  step / interpolate     the whole per-pair path

Precision.  Everything from the log intensity onwards is float32, every
operation rounded to nearest in the order written: numpy float32 ufuncs and
float32 scalars do exactly that and never fuse a multiply with an add.  The
splat winner, the footprint corners and the crossing count are discrete
decisions taken on those float32 values; the crossing count is the exact
floor of the real quotient of the two float32 numbers (``fractions``).
The log intensity is the one float64 step: it holds a transcendental and sits upstream of
the exact part, so it is compared within a tolerance.

Readings of the paper taken here (each is restated where it is used):
  R1  B is warped by a backward bilinear gather at s = q - (1-f) m_B(q);
      A by the depth-tested forward splat of Eq. 6.
  R2  blend: L = lerp(A^, B^, alpha) where both are valid, the valid one
      where only one is, lerp(L_A(q), L_B(q), alpha) where neither is;
      alpha = f (BLEND_TIME) or alpha = 1 (BLEND_B_PRIMARY: B primary,
      A only fills B's holes).
  R3  the splat value is the winner's own intensity (winner-take-all).
  R4  the footprint of a target position holds only the corners of its
      containing cell whose bilinear weight is strictly positive.
  R5  equal depths: the smaller source index wins.
  R6  Eq. 7 endpoints: p_A = p, p_B = p - m_A(p); Z_B is sampled bilinearly
      with the position clamped into the image.
  R7  a source is invisible unless its intermediate depth is > 0 (NaN too).
  R8  crossing count n = floor(|dL| / C) of the exact real quotient, with
      no upper bound; an infinite |dL| has no count (ValueError).  An
      implementation that bounds the crossings of one pixel-substep states
      its bound, and a test of that bound passes it as ``count_limit``.
  R9  the reference moves by fl(n * C) after all n crossings, also for
      crossings the refractory period suppresses.
  R10 crossing k of a substep is timed by linear interpolation of L between
      the previous and the current sample; integer microseconds, floor.
  R11 lerp(a, b, w) = a + w * (b - a); bilinear = two lerps along x, one
      along y; x1 = min(x0 + 1, W - 1).
  R18 two-splat warp (WARP_SPLAT): B is splatted backward to
      q_B = p + (1 - f) m_B(p) with Eq. 7 endpoints p_A = p + m_B(p),
      p_B = p (Z_A sampled bilinearly at p_A, clamped into the image), the
      same footprint, tie rule and visibility as A's splat, into a z-buffer
      of its own; B^ is L_B at B's winner (valid where a B source landed)
      and the blend is R2's.  With BLEND_B_PRIMARY this is the paper's
      fusion: B's splat is the result and A fills only B's holes.
  R20 noise draws: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
      random numbers: as easy as 1, 2, 3", SC 2011), key = the 64-bit
      seed (low word first), counter = (x | y << 11, j, pair index, kind);
      kind 0 gives the three decisions of pixel-substep (x, y, j), kinds
      1-3 the time (and polarity) of a leak / shot / hot event there,
      kind 4 with j = pair = 0 the pixel's hot-pixel membership.  A word
      w becomes the float32 uniform (w >> 8) 2^-24 in [0, 1).
  R21 per substep of length Dt (float32 us; Dt_s = Dt * 1e-6 in float32):
      P_leak = r_l Dt_s, P_shot = (r_s Dt_s)(1 - I), P_hot = r_h Dt_s; an
      event fires when its uniform is < P (float32 compare).  I, the
      normalised intensity, is clamp((L_j - L0) * inv_range) into [0, 1]
      (NaN -> 0) of the current log sample: a per-camera affine map of log
      intensity (the library carries log intensity only).
  R22 a noise event's time is t0 + min(floor((j - 1 + u) Dt), span) with its
      own uniform u; leak events are ON, shot and hot events take the
      polarity bit 0 of their second word (1 = ON).
  R24 defocus: taps k = -r..r with r = ceil(3 sigma), weights
      exp(-k^2 / (2 sigma^2)) normalised to sum 1, edge pixels repeated,
      along x then along y (per channel of RGB input); float64 here.
  R25 over-render margin (the paper's optional border handling): with a
      crop margin m the warp runs on the whole rendered frame and only the
      inner pixels reach the event model (and the noise), in the cropped
      frame's coordinates; the margin keeps its state untouched.
  R26 voxel grid: events of one env with t0 <= t < t1 sit at the real
      position tau = (t - t0) (B - 1) / (t1 - t0) on the axis of the B bin
      centres; linear interpolation in time gives bin b the weight
      max(0, 1 - |tau - b|), i.e. 1 - (tau - floor(tau)) to floor(tau) and
      tau - floor(tau) to the bin after it.  Sums and the division of each
      (polarity, bin) plane by its maximum (all zero when empty) are
      float64 with no bound on the events per voxel.  Layout
      [2][B][H][W], polarity 0 = OFF first.
  R23 noise events are extra: they do not move L_ref, ignore the
      refractory period and leave t_last alone.
  R19 joint warp (WARP_JOINT): one z-buffer over the sources of both
      splats (Eq. 6 with X in {A, B}); at equal depth B wins (B is the
      primary keyframe), then the smaller index.  The winner's own
      intensity is the sub-frame; where nothing lands, R2's hole value.
      The hole mask marks A invalid unless an A source won, B invalid
      unless a B source won.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction
from typing import Iterable, Optional

import numpy as np

F32 = np.float32
EMPTY_KEY = np.uint64(0xFFFF_FFFF_FFFF_FFFF)
ENUMERATE_MAX = 10 ** 7       # more crossings than this in one pixel-substep: refuse to list them
T_LAST_INIT = -(2 ** 30)      # "never fired": far enough back for any refractory period
BLEND_TIME = 0
BLEND_B_PRIMARY = 1
# Warp of B, or'ed into the mode word next to the blend: R1, R18, R19.
WARP_GATHER = 0x00
WARP_SPLAT = 0x10
WARP_JOINT = 0x20
WARP_MASK = 0x30
A_TAG = np.uint64(0x8000_0000)    # R19: marks an A source in a joint key (B wins ties)
REC709 = (0.2126, 0.7152, 0.0722)


# ---------------------------------------------------------------------------
# Small float32 building blocks (R11)
# ---------------------------------------------------------------------------

def lerp(a, b, w):
    """a + w * (b - a), three float32 roundings."""
    return a + w * (b - a)


def pixel_coords(H: int, W: int):
    """Float32 x (column) and y (row) of every pixel centre, shape [H][W]."""
    yy, xx = np.mgrid[0:H, 0:W]
    return xx.astype(F32), yy.astype(F32)


def bilinear(img: np.ndarray, sx: np.ndarray, sy: np.ndarray) -> np.ndarray:
    """Bilinear sample of float32 ``img`` at positions inside [0,W-1]x[0,H-1]."""
    H, W = img.shape
    fx0 = np.floor(sx)
    fy0 = np.floor(sy)
    wx = sx - fx0
    wy = sy - fy0
    x0 = fx0.astype(np.int64)
    y0 = fy0.astype(np.int64)
    x1 = np.minimum(x0 + 1, W - 1)
    y1 = np.minimum(y0 + 1, H - 1)
    top = lerp(img[y0, x0], img[y0, x1], wx)
    bot = lerp(img[y1, x0], img[y1, x1], wx)
    return lerp(top, bot, wy)


def clamp_into(v: np.ndarray, hi: int) -> np.ndarray:
    """Clamp into [0, hi]; NaN becomes 0."""
    v = np.where(v > 0, v, F32(0))
    return np.where(v < hi, v, F32(hi)).astype(F32)


# ---------------------------------------------------------------------------
# defocus (float64; R24)
# ---------------------------------------------------------------------------

def defocus_radius(sigma: float) -> int:
    return int(math.ceil(3.0 * sigma))


def defocus_weights(sigma: float) -> np.ndarray:
    r = defocus_radius(sigma)
    k = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return w / w.sum()


def defocus(x, sigma: float) -> np.ndarray:
    """Separable Gaussian blur of linear intensity [H][W] or [H][W][3]:
    along x, then along y, edge pixels repeated (R24)."""
    x = np.asarray(x, np.float64)
    w = defocus_weights(sigma)
    r = len(w) // 2
    planes = x[..., None] if x.ndim == 2 else x
    out = np.empty_like(planes)
    H, W = planes.shape[:2]
    for c in range(planes.shape[2]):
        p = np.pad(planes[..., c], ((0, 0), (r, r)), mode="edge")
        h = sum(w[i] * p[:, i:i + W] for i in range(2 * r + 1))
        p = np.pad(h, ((r, r), (0, 0)), mode="edge")
        out[..., c] = sum(w[i] * p[i:i + H, :] for i in range(2 * r + 1))
    return out[..., 0] if x.ndim == 2 else out


# ---------------------------------------------------------------------------
# log luminance (float64)
# ---------------------------------------------------------------------------

def log_luminance(x, eps: float = 1e-3) -> np.ndarray:
    """Eq. 3 Rec.709 luminance of [..., 3] colour (a single channel is taken
    as luminance already), then L = ln(Y + eps).  float64."""
    x = np.asarray(x, np.float64)
    if x.ndim >= 1 and x.shape[-1] == 3:
        Y = REC709[0] * x[..., 0] + REC709[1] * x[..., 1] + REC709[2] * x[..., 2]
    else:
        Y = x
    return np.log(Y + eps)


def log_channels(x, eps: float = 1e-3) -> np.ndarray:
    """Colour events (Sec. "HDR Event Formation Model"): each of R, G, B in
    place of the luminance, L_c = ln(I_c + eps); [..., 3] -> [3, ...].
    float64."""
    x = np.asarray(x, np.float64)
    return np.stack([np.log(x[..., c] + eps) for c in range(3)])


# ---------------------------------------------------------------------------
# adaptive substep count
# ---------------------------------------------------------------------------

def adaptive_k(m_A: np.ndarray, m_B: np.ndarray, K_max: int) -> int:
    """Smallest K >= 1 with K^2 >= max |m|^2 over both motion fields, at most K_max.

    |m|^2 = dx^2 + dy^2 in float64 (both squares exact, one rounding in the
    sum).  Pixels whose |m|^2 is not finite are left out.  With K so chosen,
    no motion vector moves a pixel by more than one pixel per substep.
    """
    best = 0.0
    for m in (m_A, m_B):
        dx = m[..., 0].astype(np.float64)
        dy = m[..., 1].astype(np.float64)
        msq = dx * dx + dy * dy
        msq = msq[np.isfinite(msq)]
        if msq.size:
            best = max(best, float(msq.max()))
    need = math.ceil(Fraction(best))          # K^2 >= best  <=>  K^2 >= ceil(best)
    K = math.isqrt(need)
    if K * K < need:
        K += 1
    return int(min(max(K, 1), K_max))


# ---------------------------------------------------------------------------
# endpoint depth (Eq. 7)
# ---------------------------------------------------------------------------

def endpoint_depth(Z_B: np.ndarray, m_A: np.ndarray) -> np.ndarray:
    """Z_B at p_B = p - m_A(p), position clamped into the image (R6)."""
    H, W = Z_B.shape
    px, py = pixel_coords(H, W)
    sx = clamp_into(px - m_A[..., 0], W - 1)
    sy = clamp_into(py - m_A[..., 1], H - 1)
    return bilinear(Z_B, sx, sy)


# ---------------------------------------------------------------------------
# forward depth-tested splat of A (Eq. 5, Eq. 6, Eq. 7)
# ---------------------------------------------------------------------------

def substep_fraction(j: int, K: int):
    """f = j / K in float32 (one rounding)."""
    return F32(j) / F32(K)


def splat_keys(m_A, Z_A, Zend, f):
    """Per source: target q_A = p - f m_A(p), intermediate depth and the
    packed key (float32 depth bits << 32 | source index)."""
    H, W = Z_A.shape
    px, py = pixel_coords(H, W)
    qx = px - f * m_A[..., 0]
    qy = py - f * m_A[..., 1]
    zt = lerp(Z_A, Zend, f)
    src = np.arange(H * W, dtype=np.uint64).reshape(H, W)
    key = (np.ascontiguousarray(zt).view(np.uint32).astype(np.uint64) << np.uint64(32)) | src
    return qx, qy, zt, key


def footprint(qx, qy):
    """Corners of the cell holding (qx, qy) with strictly positive bilinear
    weight (R4): list of (cx, cy, selected) int64 arrays."""
    x0f = np.floor(qx)
    y0f = np.floor(qy)
    fx = qx - x0f
    fy = qy - y0f
    x0 = x0f.astype(np.int64)
    y0 = y0f.astype(np.int64)
    allv = np.ones(qx.shape, bool)
    return [(x0, y0, allv), (x0 + 1, y0, fx > 0), (x0, y0 + 1, fy > 0),
            (x0 + 1, y0 + 1, (fx > 0) & (fy > 0))]


def scatter_min(zbuf, qx, qy, zt, key):
    """Eq. 6: every visible source (R7 plus finite position) lowers the
    keys of its footprint cells inside the image to its own key; min over
    keys = nearest depth, then smallest source index (R5).  zbuf is a flat
    uint64 [H*W] array, updated in place."""
    H, W = zt.shape
    live = (zt > 0) & (np.abs(qx) < 2.0 ** 24) & (np.abs(qy) < 2.0 ** 24)
    qx = np.where(live, qx, F32(-8))
    qy = np.where(live, qy, F32(-8))
    for cx, cy, sel in footprint(qx, qy):
        sel = sel & live & (cx >= 0) & (cx < W) & (cy >= 0) & (cy < H)
        np.minimum.at(zbuf, (cy * W + cx)[sel], key[sel])


def splat_forward(m_A, Z_A, Zend, f) -> np.ndarray:
    """Eq. 6 z-buffer of A splatted to fraction f: uint64 key per target
    pixel, EMPTY_KEY where nothing lands."""
    H, W = Z_A.shape
    qx, qy, zt, key = splat_keys(m_A, Z_A, Zend, f)
    zbuf = np.full(H * W, EMPTY_KEY, dtype=np.uint64)
    scatter_min(zbuf, qx, qy, zt, key)
    return zbuf.reshape(H, W)


# ---------------------------------------------------------------------------
# backward splat of B (Eq. 5 q_B, Eq. 6, Eq. 7; R18, R19)
# ---------------------------------------------------------------------------

def start_depth(Z_A: np.ndarray, m_B: np.ndarray) -> np.ndarray:
    """Z_A at p_A = p + m_B(p), position clamped into the image (R18)."""
    H, W = Z_A.shape
    px, py = pixel_coords(H, W)
    sx = clamp_into(px + m_B[..., 0], W - 1)
    sy = clamp_into(py + m_B[..., 1], H - 1)
    return bilinear(Z_A, sx, sy)


def splat_keys_backward(m_B, Z_B, Zstart, f):
    """Per B source: target q_B = p + (1 - f) m_B(p), intermediate depth
    (1 - f) Z_A(p_A) + f Z_B(p) as lerp(Zstart, Z_B, f) and the packed key."""
    H, W = Z_B.shape
    px, py = pixel_coords(H, W)
    g = F32(1) - f
    qx = px + g * m_B[..., 0]
    qy = py + g * m_B[..., 1]
    zt = lerp(Zstart, Z_B, f)
    src = np.arange(H * W, dtype=np.uint64).reshape(H, W)
    key = (np.ascontiguousarray(zt).view(np.uint32).astype(np.uint64) << np.uint64(32)) | src
    return qx, qy, zt, key


def splat_backward(m_B, Z_B, Zstart, f) -> np.ndarray:
    """Eq. 6 z-buffer of B splatted back to fraction f (R18)."""
    H, W = Z_B.shape
    qx, qy, zt, key = splat_keys_backward(m_B, Z_B, Zstart, f)
    zbuf = np.full(H * W, EMPTY_KEY, dtype=np.uint64)
    scatter_min(zbuf, qx, qy, zt, key)
    return zbuf.reshape(H, W)


def splat_joint(m_A, Z_A, Zend, m_B, Z_B, Zstart, f) -> np.ndarray:
    """One z-buffer over the sources of both splats (R19): A keys carry
    A_TAG in their low word, so B wins at equal depth."""
    H, W = Z_A.shape
    zbuf = np.full(H * W, EMPTY_KEY, dtype=np.uint64)
    qx, qy, zt, key = splat_keys_backward(m_B, Z_B, Zstart, f)
    scatter_min(zbuf, qx, qy, zt, key)
    qx, qy, zt, key = splat_keys(m_A, Z_A, Zend, f)
    scatter_min(zbuf, qx, qy, zt, key | A_TAG)
    return zbuf.reshape(H, W)


# ---------------------------------------------------------------------------
# resolve, backward gather of B, hole-aware blend
# ---------------------------------------------------------------------------

def resolve_gather_blend(zbuf, L_A, L_B, m_B, f, alpha):
    """Intermediate log frame at fraction f.

    A^ = L_A at the z-buffer winner (valid where something landed);
    B^ = bilinear L_B at s = q - (1 - f) m_B(q) (valid where s is inside the
    image); blend per R2.  Returns (L_f, validA, validB).
    """
    H, W = L_A.shape
    g = F32(1) - f
    ux, uy = pixel_coords(H, W)
    key = zbuf.reshape(-1)
    vA = key != EMPTY_KEY
    src = np.where(vA, key & np.uint64(0xFFFF_FFFF), np.uint64(0)).astype(np.int64)
    Ah = np.where(vA, L_A.reshape(-1)[src], F32(0)).reshape(H, W)
    vA = vA.reshape(H, W)
    sx = ux - g * m_B[..., 0]
    sy = uy - g * m_B[..., 1]
    vB = (sx >= 0) & (sx <= W - 1) & (sy >= 0) & (sy <= H - 1)
    Bh = np.zeros((H, W), F32)
    Bh[vB] = bilinear(L_B, sx[vB], sy[vB])
    both = lerp(Ah, Bh, alpha)
    hole = lerp(L_A, L_B, alpha)
    out = np.where(vA & vB, both, np.where(vA, Ah, np.where(vB, Bh, hole)))
    return out.astype(F32), vA, vB


def resolve_two_splat(zA, zB, L_A, L_B, alpha):
    """Intermediate log frame from the winners of the two splats (R18):
    A^ = L_A at A's winner, B^ = L_B at B's winner, blend per R2.  Pass the
    joint z-buffer as zA and None as zB for R19.  Returns (L_f, validA,
    validB)."""
    H, W = L_A.shape
    low = np.uint64(0xFFFF_FFFF)
    if zB is None:
        key = zA.reshape(-1)
        hit = key != EMPTY_KEY
        isA = hit & ((key & A_TAG) != 0)
        vA, vB = isA, hit & ~isA
        sA = np.where(vA, key & (low ^ A_TAG), np.uint64(0)).astype(np.int64)
        sB = np.where(vB, key & low, np.uint64(0)).astype(np.int64)
    else:
        kA, kB = zA.reshape(-1), zB.reshape(-1)
        vA, vB = kA != EMPTY_KEY, kB != EMPTY_KEY
        sA = np.where(vA, kA & low, np.uint64(0)).astype(np.int64)
        sB = np.where(vB, kB & low, np.uint64(0)).astype(np.int64)
    Ah = np.where(vA, L_A.reshape(-1)[sA], F32(0)).reshape(H, W)
    Bh = np.where(vB, L_B.reshape(-1)[sB], F32(0)).reshape(H, W)
    vA, vB = vA.reshape(H, W), vB.reshape(H, W)
    both = lerp(Ah, Bh, alpha)
    hole = lerp(L_A, L_B, alpha)
    out = np.where(vA & vB, both, np.where(vA, Ah, np.where(vB, Bh, hole)))
    return out.astype(F32), vA, vB


def blend_alpha(f, blend_mode: int):
    return f if (blend_mode & ~WARP_MASK) == BLEND_TIME else F32(1)


@dataclass
class Pair:
    """One keyframe pair A (t0_us) -> B (t1_us) of one environment."""
    L_A: np.ndarray
    L_B: np.ndarray
    m_A: np.ndarray
    m_B: np.ndarray
    Z_A: np.ndarray
    Z_B: np.ndarray
    t0_us: int = 0
    t1_us: int = 16667

    @property
    def shape(self):
        return self.L_A.shape


def substep_frames(pair: Pair, K: int, js: Iterable[int], blend_mode: int = BLEND_TIME):
    """Yields (j, L_j, hole) for j in js; L_0 = L_A and L_K = L_B exactly;
    hole bit0 = A invalid, bit1 = B invalid (0 at j = 0 and j = K).
    blend_mode is the mode word: a BLEND_* value or'ed with a WARP_* value."""
    Zend = Zstart = None
    H, W = pair.shape
    warp = blend_mode & WARP_MASK
    for j in js:
        if j == 0 or j == K:
            yield j, (pair.L_A if j == 0 else pair.L_B).astype(F32), np.zeros((H, W), np.uint8)
            continue
        if Zend is None:
            Zend = endpoint_depth(pair.Z_B, pair.m_A)
            if warp != WARP_GATHER:
                Zstart = start_depth(pair.Z_A, pair.m_B)
        f = substep_fraction(j, K)
        alpha = blend_alpha(f, blend_mode)
        if warp == WARP_GATHER:
            zbuf = splat_forward(pair.m_A, pair.Z_A, Zend, f)
            L, vA, vB = resolve_gather_blend(zbuf, pair.L_A, pair.L_B, pair.m_B, f, alpha)
        elif warp == WARP_SPLAT:
            zA = splat_forward(pair.m_A, pair.Z_A, Zend, f)
            zB = splat_backward(pair.m_B, pair.Z_B, Zstart, f)
            L, vA, vB = resolve_two_splat(zA, zB, pair.L_A, pair.L_B, alpha)
        else:
            zj = splat_joint(pair.m_A, pair.Z_A, Zend, pair.m_B, pair.Z_B, Zstart, f)
            L, vA, vB = resolve_two_splat(zj, None, pair.L_A, pair.L_B, alpha)
        hole = ((~vA).astype(np.uint8) | ((~vB).astype(np.uint8) << 1))
        yield j, L, hole


def interpolate(pair: Pair, K: int, j_begin: int, j_end: int, blend_mode: int = BLEND_TIME):
    """Stacked L_j for j in [j_begin, j_end) and their hole masks."""
    Ls, holes = [], []
    for _, L, h in substep_frames(pair, K, range(j_begin, j_end), blend_mode):
        Ls.append(L)
        holes.append(h)
    return np.stack(Ls), np.stack(holes)


# ---------------------------------------------------------------------------
# event emission (Eq. 4, Eq. 8, refractory period)
# ---------------------------------------------------------------------------

@dataclass
class Sensor:
    C_on: float = 0.2
    C_off: float = 0.2
    theta_on: Optional[np.ndarray] = None     # [H][W] float32, Eq. 8
    theta_off: Optional[np.ndarray] = None
    refractory_us: int = 0
    K: int = 8                                # > 0 fixed, <= 0 adaptive
    K_max: int = 64
    blend_mode: int = BLEND_TIME
    noise: Optional["Noise"] = None           # leak / shot / hot-pixel events (R20-R23)

    def thresholds(self, H, W):
        on = self.theta_on if self.theta_on is not None else np.full((H, W), F32(self.C_on))
        off = self.theta_off if self.theta_off is not None else np.full((H, W), F32(self.C_off))
        return on.astype(F32), off.astype(F32)


def crossing_count(a, c, count_limit: Optional[int] = None) -> int:
    """Eq. 4: n = floor(a / c) of the exact real quotient of float32 a >= c > 0
    (R8).  An infinite a has no finite count and raises ValueError.

    ``count_limit`` is not the paper's: it models an implementation that
    bounds the crossings of one pixel-substep (n = min(n, limit), an infinite
    a counting as the limit); tests of such a bound pass it explicitly."""
    if not math.isfinite(float(a)):
        if count_limit is None:
            raise ValueError("Eq. 4 gives no finite crossing count for an infinite |dL|")
        return int(count_limit)
    n = int(Fraction(float(a)) // Fraction(float(c)))
    if count_limit is not None:
        n = min(n, int(count_limit))
    return n


def crossing_time_offset(j, k, R, c, positive, prev, cur, Dt, span) -> int:
    """R10: integer-microsecond offset from t0 of crossing k in substep j.

    The k-th crossing level is R +- k*c; its position between the previous
    sample ``prev`` and the current ``cur`` is phi = (level - prev) / (cur - prev),
    clamped to [0, 1] (1 when cur == prev, NaN -> 0); the offset is
    floor((j - 1 + phi) * Dt), at most ``span``.
    """
    kc = F32(k) * c
    lam = R + kc if positive else R - kc
    den = cur - prev
    if den == 0:
        phi = F32(1)
    else:
        phi = (lam - prev) / den
    if not phi >= 0:
        phi = F32(0)
    if phi > 1:
        phi = F32(1)
    v = (F32(j - 1) + phi) * Dt
    return min(int(np.floor(v)), span)


def substep_dt(t0_us: int, t1_us: int, K: int):
    """Dt = fl32(fl32(t1 - t0) / fl32(K)), microseconds per substep."""
    return F32(F32(t1_us - t0_us) / F32(K))


class EventLog:
    """Collects (x, y, t_us, p, env) tuples."""

    def __init__(self):
        self.rows = []

    def add(self, x, y, t, p, env):
        self.rows.append((x, y, t, p, env))

    def array(self) -> np.ndarray:
        if not self.rows:
            return np.zeros((0, 5), np.int64)
        return np.asarray(self.rows, np.int64)


def emit_substep(j, prev, cur, R, tl, on, off, refractory_us, t0_us, Dt, span,
                 env_id, log: EventLog, track_t_last: bool = True,
                 count_limit: Optional[int] = None):
    """Eq. 4 at substep j for every pixel; R and tl are updated in place
    (count_limit: see crossing_count)."""
    H, W = cur.shape
    d = cur - R
    positive = d > 0
    c = np.where(positive, on, off)
    a = np.abs(d)
    hit = (a >= c) & (c > 0)              # n = 0 otherwise (NaN never hits)
    for flat in np.flatnonzero(hit):
        y, x = divmod(int(flat), W)
        pos = bool(positive[y, x])
        cc = c[y, x]
        n = crossing_count(a[y, x], cc, count_limit)
        if n > ENUMERATE_MAX:
            raise ValueError(f"{n} crossings in one pixel-substep: too many to list")
        r0 = R[y, x]
        for k in range(1, n + 1):
            t = t0_us + crossing_time_offset(j, k, r0, cc, pos, prev[y, x], cur[y, x], Dt, span)
            if refractory_us == 0 or t - int(tl[y, x]) >= refractory_us:
                log.add(x, y, t, 1 if pos else 0, env_id)
                if track_t_last:
                    tl[y, x] = t
        nc = F32(n) * cc
        R[y, x] = r0 + nc if pos else r0 - nc


def emit_events(S_seq, t0_us, t1_us, sensor: Sensor, L_ref, t_last=None, env_id=0,
                count_limit: Optional[int] = None):
    """Events from caller-supplied frames S_seq[0..K] (S_seq[0] is the
    previous sample; events come from j = 1..K).  Returns (events[N,5] as
    x, y, t, p, env; L_ref'; t_last').  count_limit: see crossing_count."""
    S_seq = [np.asarray(s, F32) for s in S_seq]
    K = len(S_seq) - 1
    H, W = S_seq[0].shape
    on, off = sensor.thresholds(H, W)
    R = np.array(L_ref, F32, copy=True)
    track = t_last is not None
    tl = np.array(t_last, np.int64, copy=True) if track else np.full((H, W), T_LAST_INIT, np.int64)
    Dt = substep_dt(t0_us, t1_us, K)
    span = t1_us - t0_us
    log = EventLog()
    nz = sensor.noise
    hot = hot_pixels(H, W, nz) if nz is not None else None
    for j in range(1, K + 1):
        emit_substep(j, S_seq[j - 1], S_seq[j], R, tl, on, off, sensor.refractory_us,
                     t0_us, Dt, span, env_id, log, track, count_limit)
        if nz is not None:
            noise_events(j, S_seq[j], Dt, t0_us, span, nz, env_id, log, hot)
    return log.array(), R, (tl.astype(np.int32) if track else None)


# ---------------------------------------------------------------------------
# noise events (Sec. "Sensor Calibration and Non-idealities"; R20-R23)
# ---------------------------------------------------------------------------

PHILOX_M = (np.uint64(0xD2511F53), np.uint64(0xCD9E8D57))   # round multipliers
PHILOX_W = (np.uint64(0x9E3779B9), np.uint64(0xBB67AE85))   # key increments
_M32 = np.uint64(0xFFFF_FFFF)


def philox4x32(ctr, key, rounds: int = 10):
    """Philox4x32-R of Salmon et al. (SC 2011), elementwise over numpy
    arrays: ctr four uint32 words, key two; returns four uint32 arrays.
    Round: (hi(M0 c0), lo(M0 c0)) and (hi(M1 c2), lo(M1 c2)); the new
    counter is (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key grows by
    the Weyl increments before every round after the first."""
    c0, c1, c2, c3 = [np.asarray(c, np.uint64) & _M32 for c in ctr]
    k0, k1 = [np.asarray(k, np.uint64) & _M32 for k in key]
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + PHILOX_W[0]) & _M32
            k1 = (k1 + PHILOX_W[1]) & _M32
        p0 = PHILOX_M[0] * c0            # < 2^64: exact in uint64
        p1 = PHILOX_M[1] * c2
        c0, c1, c2, c3 = ((p1 >> np.uint64(32)) ^ c1 ^ k0, p1 & _M32,
                          (p0 >> np.uint64(32)) ^ c3 ^ k1, p0 & _M32)
    return [c.astype(np.uint32) for c in (c0, c1, c2, c3)]


def uniform24(w):
    """R20: the top 24 bits of a uint32 word as a float32 in [0, 1)."""
    return (np.asarray(w, np.uint32) >> np.uint32(8)).astype(F32) * F32(2.0 ** -24)


@dataclass
class Noise:
    """Per-camera noise parameters (rates in events per second)."""
    leak_rate_hz: float = 0.0
    shot_rate_hz: float = 0.0
    hot_rate_hz: float = 0.0
    hot_fraction: float = 0.0
    shot_L0: float = 0.0           # log intensity whose normalised intensity is 0
    shot_inv_range: float = 1.0    # normalised intensity per unit of log intensity
    seed: int = 0                  # 64-bit generator key
    pair_index: int = 0            # which keyframe pair (a counter word)


def hot_pixels(H, W, nz: Noise) -> np.ndarray:
    """R20: the fixed hot-pixel set, one draw per pixel."""
    ux, uy = pixel_coords(H, W)
    xy = ux.astype(np.uint64) | (uy.astype(np.uint64) << np.uint64(11))
    key = (nz.seed & 0xFFFF_FFFF, (nz.seed >> 32) & 0xFFFF_FFFF)
    w = philox4x32((xy, 0, 0, 4), key)[0]
    return uniform24(w) < F32(nz.hot_fraction)


def noise_events(j, cur, Dt, t0_us, span, nz: Noise, env_id, log: EventLog, hot=None):
    """Leak, shot and hot-pixel events of substep j (R20-R23); cur is the
    log sample L_j.  Appends to log; touches no state."""
    H, W = cur.shape
    ux, uy = pixel_coords(H, W)
    xy = ux.astype(np.uint64) | (uy.astype(np.uint64) << np.uint64(11))
    key = (nz.seed & 0xFFFF_FFFF, (nz.seed >> 32) & 0xFFFF_FFFF)
    w0, w1, w2, _ = philox4x32((xy, j, nz.pair_index, 0), key)
    dts = F32(Dt) * F32(1e-6)
    p_leak = F32(nz.leak_rate_hz) * dts
    ibar = (cur - F32(nz.shot_L0)) * F32(nz.shot_inv_range)
    ibar = np.where(ibar > 0, ibar, F32(0))
    ibar = np.where(ibar < 1, ibar, F32(1)).astype(F32)
    p_shot = (F32(nz.shot_rate_hz) * dts) * (F32(1) - ibar)
    p_hot = F32(nz.hot_rate_hz) * dts
    if hot is None:
        hot = hot_pixels(H, W, nz)
    fires = ((1, uniform24(w0) < p_leak), (2, uniform24(w1) < p_shot),
             (3, hot & (uniform24(w2) < p_hot)))
    for kind, fire in fires:
        for flat in np.flatnonzero(fire):
            y, x = divmod(int(flat), W)
            e0, e1, _, _ = philox4x32((np.uint64(x | (y << 11)), j, nz.pair_index, kind), key)
            v = (F32(j - 1) + uniform24(e0)) * F32(Dt)
            t = t0_us + min(int(np.floor(v)), span)
            pol = 1 if kind == 1 else int(e1) & 1
            log.add(x, y, t, pol, env_id)


# ---------------------------------------------------------------------------
# The whole per-pair path
# ---------------------------------------------------------------------------

def choose_k(pair: Pair, sensor: Sensor) -> int:
    if sensor.K > 0:
        return int(sensor.K)
    return adaptive_k(pair.m_A, pair.m_B, sensor.K_max)


def step(pair: Pair, sensor: Sensor, L_ref, t_last=None, env_id: int = 0, crop_margin: int = 0,
         count_limit: Optional[int] = None):
    """One keyframe pair: K, sub-frames (splat, gather, blend) and events, streaming
    over j.  Returns (events[N,5], L_ref', t_last', K).

    crop_margin m > 0 (R25): the frames carry an over-rendered margin of m
    pixels on every side; the warp uses all of it, the event model (and the
    noise) only the inner (H - 2m) x (W - 2m) pixels, whose events are in
    the cropped frame's coordinates; the margin's L_ref and t_last are left
    as they are.  count_limit: see crossing_count."""
    K = choose_k(pair, sensor)
    H, W = pair.shape
    m = int(crop_margin)
    inner = (slice(m, H - m), slice(m, W - m))
    on, off = sensor.thresholds(H, W)
    on, off = on[inner], off[inner]
    R = np.array(L_ref, F32, copy=True)
    track = t_last is not None
    tl = np.array(t_last, np.int64, copy=True) if track else np.full((H, W), T_LAST_INIT, np.int64)
    Rc, tlc = R[inner], tl[inner]                 # views: updated in place
    Dt = substep_dt(pair.t0_us, pair.t1_us, K)
    span = pair.t1_us - pair.t0_us
    log = EventLog()
    prev = pair.L_A.astype(F32)[inner]
    nz = sensor.noise
    hot = hot_pixels(H - 2 * m, W - 2 * m, nz) if nz is not None else None
    for j, L, _ in substep_frames(pair, K, range(1, K + 1), sensor.blend_mode):
        Lc = L[inner]
        emit_substep(j, prev, Lc, Rc, tlc, on, off, sensor.refractory_us, pair.t0_us, Dt,
                     span, env_id, log, track, count_limit)
        if nz is not None:
            noise_events(j, Lc, Dt, pair.t0_us, span, nz, env_id, log, hot)
        prev = Lc
    return log.array(), R, (tl.astype(np.int32) if track else None), K


# ---------------------------------------------------------------------------
# event record
# ---------------------------------------------------------------------------

def pack_events(ev: np.ndarray) -> np.ndarray:
    """[N,5] (x, y, t, p, env) -> [N,2] int64 of (x | y<<11 | p<<22 | env<<23, t)."""
    ev = np.asarray(ev, np.int64).reshape(-1, 5)
    word = ev[:, 0] | (ev[:, 1] << 11) | (ev[:, 3] << 22) | (ev[:, 4] << 23)
    return np.stack([word, ev[:, 2]], axis=1)


def unpack_events(rec: np.ndarray) -> np.ndarray:
    """Inverse of pack_events; accepts uint32/int32 words."""
    rec = np.asarray(rec).reshape(-1, 2)
    word = rec[:, 0].astype(np.int64) & 0xFFFF_FFFF
    t = rec[:, 1].astype(np.int64)
    x = word & 0x7FF
    y = (word >> 11) & 0x7FF
    p = (word >> 22) & 1
    env = (word >> 23) & 0x1FF
    return np.stack([x, y, t, p, env], axis=1)


def canonical(ev: np.ndarray) -> np.ndarray:
    """Events sorted by (env, t, y, x, p): the multiset in a fixed order."""
    ev = np.asarray(ev, np.int64).reshape(-1, 5)
    order = np.lexsort((ev[:, 3], ev[:, 0], ev[:, 1], ev[:, 2], ev[:, 4]))
    return ev[order]


# ---------------------------------------------------------------------------
# event voxel grid (R26)
# ---------------------------------------------------------------------------

def voxel_weights(t, t0_us: int, t1_us: int, bins: int):
    """Per event time: its position tau = (t - t0)(B - 1)/(t1 - t0) on the
    axis of bin centres (float64), the bin b = floor(tau) below it, and the
    linear-interpolation weights 1 - (tau - b) of bin b and tau - b of bin
    b + 1 (R26)."""
    tau = (np.asarray(t, np.int64) - t0_us).astype(np.float64) * float(bins - 1) \
        / float(t1_us - t0_us)
    b = np.floor(tau).astype(np.int64)
    last = b >= bins - 1                  # only t = t1 would land here; kept for safety
    b = np.where(last, bins - 1, b)
    w1 = np.where(last, 0.0, tau - b)
    return b, 1.0 - w1, w1


def voxel_counts(ev, env_id: int, H: int, W: int, t0_us: int, t1_us: int, bins: int = 128):
    """Weight sums [2][bins][H][W] (float64, no bound on the events per voxel)
    of one env's events with t0 <= t < t1."""
    ev = np.asarray(ev, np.int64).reshape(-1, 5)
    sel = (ev[:, 4] == env_id) & (ev[:, 2] >= t0_us) & (ev[:, 2] < t1_us)
    ev = ev[sel]
    acc = np.zeros((2, bins, H, W), np.float64)
    b, w0, w1 = voxel_weights(ev[:, 2], t0_us, t1_us, bins)
    x, y, p = ev[:, 0], ev[:, 1], ev[:, 3]
    np.add.at(acc, (p, b, y, x), w0)
    nxt = w1 > 0
    np.add.at(acc, (p[nxt], b[nxt] + 1, y[nxt], x[nxt]), w1[nxt])
    return acc


def voxel_grid(ev, env_id: int, H: int, W: int, t0_us: int, t1_us: int, bins: int = 128):
    """Normalised per-polarity voxel grid, float64 [2][bins][H][W] (R26):
    every (polarity, bin) plane divided by its own maximum."""
    acc = voxel_counts(ev, env_id, H, W, t0_us, t1_us, bins)
    mx = acc.reshape(2, bins, -1).max(axis=2)
    out = np.zeros((2, bins, H, W), np.float64)
    for p in range(2):
        for b in range(bins):
            if mx[p, b] > 0:
                out[p, b] = acc[p, b] / mx[p, b]
    return out

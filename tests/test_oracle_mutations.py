"""Plant one plausible mistake at a time into the CPU oracle and require the
pins to notice.  This shows the pins constrain every step of the oracle,
not only its overall shape.  CPU only; the mistakes live in patched copies
of oracle functions and never leave this process."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import evis_oracle as o
import oracle_pins as P

F32 = np.float32


def m_splat_sign(m_A, Z_A, Zend, f):
    H, W = Z_A.shape
    px, py = o.pixel_coords(H, W)
    qx = px + f * m_A[..., 0]                      # planted: wrong sign of Eq. 5
    qy = py + f * m_A[..., 1]
    zt = o.lerp(Z_A, Zend, f)
    src = np.arange(H * W, dtype=np.uint64).reshape(H, W)
    key = (zt.view(np.uint32).astype(np.uint64) << np.uint64(32)) | src
    return qx, qy, zt, key


def m_depth_swapped(m_A, Z_A, Zend, f):
    H, W = Z_A.shape
    px, py = o.pixel_coords(H, W)
    qx = px - f * m_A[..., 0]
    qy = py - f * m_A[..., 1]
    zt = o.lerp(Zend, Z_A, f)                      # planted: Eq. 7 weights swapped
    src = np.arange(H * W, dtype=np.uint64).reshape(H, W)
    key = (np.ascontiguousarray(zt).view(np.uint32).astype(np.uint64) << np.uint64(32)) | src
    return qx, qy, zt, key


def m_zbuffer_max(m_A, Z_A, Zend, f):
    H, W = Z_A.shape
    qx, qy, zt, key = o.splat_keys(m_A, Z_A, Zend, f)
    live = (zt > 0) & (np.abs(qx) < 2.0 ** 24) & (np.abs(qy) < 2.0 ** 24)
    zbuf = np.zeros(H * W, dtype=np.uint64)        # planted: farthest surface wins
    for cx, cy, sel in o.footprint(np.where(live, qx, F32(-8)), np.where(live, qy, F32(-8))):
        sel = sel & live & (cx >= 0) & (cx < W) & (cy >= 0) & (cy < H)
        np.maximum.at(zbuf, (cy * W + cx)[sel], key[sel])
    zbuf[zbuf == 0] = o.EMPTY_KEY
    return zbuf.reshape(H, W)


def m_zero_weight_corners(qx, qy):
    x0f, y0f = np.floor(qx), np.floor(qy)
    x0, y0 = x0f.astype(np.int64), y0f.astype(np.int64)
    allv = np.ones(qx.shape, bool)
    return [(x0, y0, allv), (x0 + 1, y0, allv), (x0, y0 + 1, allv), (x0 + 1, y0 + 1, allv)]


def m_gather_sign(zbuf, L_A, L_B, m_B, f, alpha):
    return o.__dict__["_orig_rgb"](zbuf, L_A, L_B, -m_B, f, alpha)   # planted: s = q + g m_B


def m_blend_swap(zbuf, L_A, L_B, m_B, f, alpha):
    H, W = L_A.shape
    out, vA, vB = o.__dict__["_orig_rgb"](zbuf, L_A, L_B, m_B, f, alpha)
    g = F32(1) - f
    ux, uy = o.pixel_coords(H, W)
    key = zbuf.reshape(-1)
    src = np.where(key != o.EMPTY_KEY, key & np.uint64(0xFFFF_FFFF), 0).astype(np.int64)
    Ah = L_A.reshape(-1)[src].reshape(H, W)
    sx, sy = ux - g * m_B[..., 0], uy - g * m_B[..., 1]
    Bh = np.zeros((H, W), F32)
    Bh[vB] = o.bilinear(L_B, sx[vB], sy[vB])
    swapped = o.lerp(Bh, Ah, alpha)                # planted: blend weights swapped
    return np.where(vA & vB, swapped, out).astype(F32), vA, vB


def m_bilinear_transposed(img, sx, sy):
    H, W = img.shape
    x0 = np.floor(sx).astype(np.int64)
    y0 = np.floor(sy).astype(np.int64)
    wx, wy = sx - np.floor(sx), sy - np.floor(sy)
    x1, y1 = np.minimum(x0 + 1, W - 1), np.minimum(y0 + 1, H - 1)
    t = img.T                                      # planted: rows and columns swapped
    top = o.lerp(t[np.minimum(y0, W - 1), np.minimum(x0, H - 1)],
                 t[np.minimum(y0, W - 1), np.minimum(x1, H - 1)], wx)
    bot = o.lerp(t[np.minimum(y1, W - 1), np.minimum(x0, H - 1)],
                 t[np.minimum(y1, W - 1), np.minimum(x1, H - 1)], wx)
    return o.lerp(top, bot, wy)


def m_adaptive_floor(m_A, m_B, K_max):
    best = 0.0
    for m in (m_A, m_B):
        msq = m[..., 0].astype(np.float64) ** 2 + m[..., 1].astype(np.float64) ** 2
        msq = msq[np.isfinite(msq)]
        best = max(best, float(msq.max()) if msq.size else 0.0)
    return int(min(max(int(math.floor(math.sqrt(best))), 1), K_max))   # planted: floor


def m_rounded_quotient(a, c, count_limit=None):
    return int(math.floor(F32(a) / F32(c)))               # planted: floor of fl32(a/c)


def m_time_shift(j, k, R, c, positive, prev, cur, Dt, span):
    return o.__dict__["_orig_cto"](j + 1, k, R, c, positive, prev, cur, Dt, span)  # planted: j, not j-1


def _emit_variant(drop_residual=False, flip=False, refr_keeps_ref=False):
    def emit(j, prev, cur, R, tl, on, off, refractory_us, t0_us, Dt, span, env_id, log,
             track_t_last=True, count_limit=None):
        H, W = cur.shape
        d = cur - R
        positive = d > 0
        c = np.where(positive, on, off)
        a = np.abs(d)
        hit = (a >= c) & (c > 0)
        for flat in np.flatnonzero(hit):
            y, x = divmod(int(flat), W)
            pos = bool(positive[y, x])
            cc = c[y, x]
            n = o.crossing_count(a[y, x], cc, count_limit)
            r0 = R[y, x]
            kept = 0
            for k in range(1, n + 1):
                t = t0_us + o.crossing_time_offset(j, k, r0, cc, pos, prev[y, x], cur[y, x], Dt, span)
                if refractory_us == 0 or t - int(tl[y, x]) >= refractory_us:
                    p = 1 if pos else 0
                    log.add(x, y, t, (1 - p) if flip else p, env_id)
                    kept += 1
                    if track_t_last:
                        tl[y, x] = t
            if drop_residual:
                R[y, x] = cur[y, x]
            else:
                nn = kept if refr_keeps_ref else n
                nc = F32(nn) * cc
                R[y, x] = r0 + nc if pos else r0 - nc
    return emit


def m_backward_sign(m_B, Z_B, Zstart, f):
    H, W = Z_B.shape
    px, py = o.pixel_coords(H, W)
    g = F32(1) - f
    qx = px - g * m_B[..., 0]                      # planted: q_B = p - (1 - f) m_B
    qy = py - g * m_B[..., 1]
    zt = o.lerp(Zstart, Z_B, f)
    src = np.arange(H * W, dtype=np.uint64).reshape(H, W)
    key = (np.ascontiguousarray(zt).view(np.uint32).astype(np.uint64) << np.uint64(32)) | src
    return qx, qy, zt, key


def m_backward_fraction(m_B, Z_B, Zstart, f):
    H, W = Z_B.shape
    px, py = o.pixel_coords(H, W)
    qx = px + f * m_B[..., 0]                      # planted: f where 1 - f belongs
    qy = py + f * m_B[..., 1]
    zt = o.lerp(Zstart, Z_B, f)
    src = np.arange(H * W, dtype=np.uint64).reshape(H, W)
    key = (np.ascontiguousarray(zt).view(np.uint32).astype(np.uint64) << np.uint64(32)) | src
    return qx, qy, zt, key


def m_backward_depth_swapped(m_B, Z_B, Zstart, f):
    qx, qy, _, _ = o.__dict__["_orig_skb"](m_B, Z_B, Zstart, f)
    H, W = Z_B.shape
    zt = o.lerp(Z_B, Zstart, f)                    # planted: Eq. 7 endpoints swapped
    src = np.arange(H * W, dtype=np.uint64).reshape(H, W)
    key = (np.ascontiguousarray(zt).view(np.uint32).astype(np.uint64) << np.uint64(32)) | src
    return qx, qy, zt, key


def m_start_depth_sign(Z_A, m_B):
    return o.endpoint_depth(Z_A, m_B)              # planted: Z_A at p - m_B(p)


def m_joint_a_first(m_A, Z_A, Zend, m_B, Z_B, Zstart, f):
    H, W = Z_A.shape
    zbuf = np.full(H * W, o.EMPTY_KEY, dtype=np.uint64)
    qx, qy, zt, key = o.splat_keys_backward(m_B, Z_B, Zstart, f)
    o.scatter_min(zbuf, qx, qy, zt, key | o.A_TAG)   # planted: A wins ties
    qx, qy, zt, key = o.splat_keys(m_A, Z_A, Zend, f)
    o.scatter_min(zbuf, qx, qy, zt, key)
    z = zbuf.reshape(H, W)
    low = z & np.uint64(0xFFFF_FFFF)
    hit = z != o.EMPTY_KEY
    return np.where(hit, (z & ~np.uint64(0xFFFF_FFFF)) | (low ^ o.A_TAG), z)


def m_two_splat_b_everywhere(zA, zB, L_A, L_B, alpha):
    if zB is not None:                             # planted: B valid wherever A's splat is
        zB = np.where(zB == o.EMPTY_KEY, np.arange(zB.size, dtype=np.uint64).reshape(zB.shape), zB)
    return o.__dict__["_orig_rts"](zA, zB, L_A, L_B, alpha)


def m_philox_multipliers_swapped(ctr, key, rounds=10):
    saved = o.PHILOX_M
    o.PHILOX_M = (saved[1], saved[0])              # planted: multipliers swapped
    try:
        return o.__dict__["_orig_philox"](ctr, key, rounds)
    finally:
        o.PHILOX_M = saved


def _noise_variant(dt_us=False, bright=False, leak_pol=False):
    def noise(j, cur, Dt, t0_us, span, nz, env_id, log, hot=None):
        H, W = cur.shape
        ux, uy = o.pixel_coords(H, W)
        xy = ux.astype(np.uint64) | (uy.astype(np.uint64) << np.uint64(11))
        key = (nz.seed & 0xFFFF_FFFF, (nz.seed >> 32) & 0xFFFF_FFFF)
        w0, w1, w2, _ = o.philox4x32((xy, j, nz.pair_index, 0), key)
        dts = F32(Dt) if dt_us else F32(Dt) * F32(1e-6)       # planted: microseconds
        ibar = (cur - F32(nz.shot_L0)) * F32(nz.shot_inv_range)
        ibar = np.where(ibar > 0, ibar, F32(0))
        ibar = np.where(ibar < 1, ibar, F32(1)).astype(F32)
        shade = ibar if bright else (F32(1) - ibar)              # planted: brighter fires more
        p_shot = (F32(nz.shot_rate_hz) * dts) * shade
        if hot is None:
            hot = o.hot_pixels(H, W, nz)
        fires = ((1, o.uniform24(w0) < F32(nz.leak_rate_hz) * dts),
                 (2, o.uniform24(w1) < p_shot),
                 (3, hot & (o.uniform24(w2) < F32(nz.hot_rate_hz) * dts)))
        for kind, fire in fires:
            for flat in np.flatnonzero(fire):
                y, x = divmod(int(flat), W)
                e0, e1, _, _ = o.philox4x32((np.uint64(x | (y << 11)), j, nz.pair_index, kind), key)
                v = (F32(j - 1) + o.uniform24(e0)) * F32(Dt)
                t = t0_us + min(int(np.floor(v)), span)
                pol = 1 if (kind == 1 and not leak_pol) else int(e1) & 1   # planted: random leak
                log.add(x, y, t, pol, env_id)
    return noise


def m_defocus_zero_padding(x, sigma):
    x = np.asarray(x, np.float64)
    w = o.defocus_weights(sigma)
    r = len(w) // 2
    planes = x[..., None] if x.ndim == 2 else x
    out = np.empty_like(planes)
    H, W = planes.shape[:2]
    for c in range(planes.shape[2]):
        p = np.pad(planes[..., c], ((0, 0), (r, r)))          # planted: zeros past the edge
        h = sum(w[i] * p[:, i:i + W] for i in range(2 * r + 1))
        p = np.pad(h, ((r, r), (0, 0)))
        out[..., c] = sum(w[i] * p[i:i + H, :] for i in range(2 * r + 1))
    return out[..., 0] if x.ndim == 2 else out


def m_defocus_radius(sigma):
    return int(math.ceil(2.0 * sigma))                      # planted: 2 sigma


def m_crop_after_the_fact(pair, sensor, L_ref, t_last=None, env_id=0, crop_margin=0):
    ev, R, tl, K = o.__dict__["_orig_step"](pair, sensor, L_ref, t_last, env_id)
    m = crop_margin
    H, W = pair.shape
    if m and len(ev):                               # planted: full-frame events and state,
        keep = (ev[:, 0] >= m) & (ev[:, 0] < W - m) & (ev[:, 1] >= m) & (ev[:, 1] < H - m)
        ev = ev[keep]                               # coordinates not shifted
    return ev, R, tl, K


def m_voxel_weights_swapped(t, t0_us, t1_us, bins):
    b, w0, w1 = o.__dict__["_orig_vw"](t, t0_us, t1_us, bins)
    return b, np.where(w1 == 0, w0, w1), np.where(w1 == 0, 0.0, w0)   # planted: wrong bins


def m_voxel_global_max(ev, env_id, H, W, t0_us, t1_us, bins=128):
    acc = o.voxel_counts(ev, env_id, H, W, t0_us, t1_us, bins)
    mx = acc.max()                                          # planted: one maximum for all bins
    return (acc / mx) if mx > 0 else np.zeros(acc.shape)


def m_voxel_nearest_bin(t, t0_us, t1_us, bins):
    b, w0, w1 = o.__dict__["_orig_vw"](t, t0_us, t1_us, bins)
    up = w1 >= 0.5                                          # planted: nearest bin, no interpolation
    return np.where(up, b + 1, b), np.ones_like(w0), np.zeros_like(w1)


def m_pack_shift(ev):
    ev = np.asarray(ev, np.int64).reshape(-1, 5)
    word = ev[:, 0] | (ev[:, 1] << 12) | (ev[:, 3] << 22) | (ev[:, 4] << 23)   # planted
    return np.stack([word, ev[:, 2]], axis=1)


MUTANTS = [
    ("splat_sign", "splat_keys", m_splat_sign, P.pin_integer_translation),
    ("depth_weights_swapped", "splat_keys", m_depth_swapped, P.pin_depth_interp),
    ("zbuffer_keeps_farthest", "splat_forward", m_zbuffer_max, P.pin_occlusion),
    ("zero_weight_corners", "footprint", m_zero_weight_corners, P.pin_integer_translation),
    ("gather_sign", "resolve_gather_blend", m_gather_sign, P.pin_gather_affine),
    ("blend_swapped", "resolve_gather_blend", m_blend_swap, P.pin_blend_modes),
    ("bilinear_transposed", "bilinear", m_bilinear_transposed, P.pin_endpoint_depth_affine),
    ("adaptive_k_floor", "adaptive_k", m_adaptive_floor, P.pin_adaptive_k),
    ("rounded_quotient", "crossing_count", m_rounded_quotient, P.pin_goldens),
    ("time_offset_shift", "crossing_time_offset", m_time_shift, P.pin_goldens),
    ("residual_dropped", "emit_substep", _emit_variant(drop_residual=True), P.pin_goldens),
    ("polarity_flipped", "emit_substep", _emit_variant(flip=True), P.pin_goldens),
    ("suppressed_keep_reference", "emit_substep", _emit_variant(refr_keeps_ref=True), P.pin_goldens),
    ("pack_bit_position", "pack_events", m_pack_shift, P.pin_event_record),
    ("backward_splat_sign", "splat_keys_backward", m_backward_sign, P.pin_backward_splat_reversal),
    ("backward_splat_fraction", "splat_keys_backward", m_backward_fraction,
     P.pin_backward_splat_reversal),
    ("backward_depth_swapped", "splat_keys_backward", m_backward_depth_swapped,
     P.pin_backward_splat_reversal),
    ("start_depth_sign", "start_depth", m_start_depth_sign, P.pin_start_depth_affine),
    ("joint_a_wins_ties", "splat_joint", m_joint_a_first, P.pin_joint_priority),
    ("two_splat_b_everywhere", "resolve_two_splat", m_two_splat_b_everywhere,
     P.pin_two_splat_layers),
    ("philox_multipliers_swapped", "philox4x32", m_philox_multipliers_swapped, P.pin_philox_kat),
    ("noise_rate_in_microseconds", "noise_events", _noise_variant(dt_us=True), P.pin_leak_rate),
    ("shot_noise_brighter_fires", "noise_events", _noise_variant(bright=True), P.pin_shot_darkness),
    ("leak_random_polarity", "noise_events", _noise_variant(leak_pol=True), P.pin_leak_rate),
    ("defocus_zero_padding", "defocus", m_defocus_zero_padding, P.pin_defocus_library),
    ("defocus_radius_two_sigma", "defocus_radius", m_defocus_radius, P.pin_defocus_closed_forms),
    ("crop_after_the_fact", "step", m_crop_after_the_fact, P.pin_crop_margin),
    ("voxel_weights_swapped", "voxel_weights", m_voxel_weights_swapped, P.pin_voxel_invariants),
    ("voxel_global_max", "voxel_grid", m_voxel_global_max, P.pin_voxel_closed_forms),
    ("voxel_nearest_bin", "voxel_weights", m_voxel_nearest_bin, P.pin_voxel_brute_force),
]


def test_unmutated_variant_passes(monkeypatch):
    """The harness's own copy of emit_substep, without a mistake, passes."""
    monkeypatch.setattr(o, "emit_substep", _emit_variant())
    P.pin_goldens(o)
    P.pin_residual_and_sum(o)


@pytest.mark.parametrize("name,attr,mutant,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_mutant(monkeypatch, name, attr, mutant, pin):
    monkeypatch.setitem(o.__dict__, "_orig_rgb", o.resolve_gather_blend)
    monkeypatch.setitem(o.__dict__, "_orig_cto", o.crossing_time_offset)
    monkeypatch.setitem(o.__dict__, "_orig_skb", o.splat_keys_backward)
    monkeypatch.setitem(o.__dict__, "_orig_rts", o.resolve_two_splat)
    monkeypatch.setitem(o.__dict__, "_orig_philox", o.philox4x32)
    monkeypatch.setitem(o.__dict__, "_orig_step", o.step)
    monkeypatch.setitem(o.__dict__, "_orig_vw", o.voxel_weights)
    monkeypatch.setattr(o, attr, mutant)
    with pytest.raises((AssertionError, IndexError, ValueError)):
        pin(o)

"""Pins of the CPU oracle to facts that do not come from the oracle itself.

Each ``pin_*`` takes the oracle module and raises AssertionError when the
oracle disagrees with a closed form, an invariant, a brute-force enumeration
or a hand-worked golden case.  ``test_oracle_pins.py`` runs them on the real
oracle; ``test_oracle_mutations.py`` runs them on copies of the oracle with
one plausible mistake planted, and requires some pin to fail.
"""
from __future__ import annotations

import math
import os
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np

F32 = np.float32
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ---------------------------------------------------------------------------
# helpers (inputs only; no oracle arithmetic)
# ---------------------------------------------------------------------------

def zero_motion_pair(o, L_A, L_B, Z=1.0, t0=0, t1=1000):
    L_A = np.asarray(L_A, F32)
    L_B = np.asarray(L_B, F32)
    H, W = L_A.shape
    m = np.zeros((H, W, 2), F32)
    z = np.full((H, W), F32(Z))
    return o.Pair(L_A, L_B, m, m.copy(), z, z.copy(), t0, t1)


def read_golden(name):
    kv, events = {}, []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = [s.strip() for s in line.split("=", 1)]
            if k == "event":
                events.append([int(t) for t in v.split()])
            else:
                kv[k] = v
    return kv, events


# ---------------------------------------------------------------------------
# log intensity
# ---------------------------------------------------------------------------

def pin_log_luminance(o):
    for v in (0.0, 1.0, 100.0, 1e3):
        got = float(o.log_luminance(np.array([v, v, v])))
        assert abs(got - math.log(v + 1e-3)) < 1e-12, (v, got)
    v = math.exp(2.0) - 1e-3
    assert abs(float(o.log_luminance(np.array([v, v, v]))) - 2.0) < 1e-12
    w = (0.2126, 0.7152, 0.0722)
    for ch in range(3):
        x = np.zeros(3)
        x[ch] = 1.0
        assert abs(float(o.log_luminance(x)) - math.log(w[ch] + 1e-3)) < 1e-12
    y = np.array([[0.5, 7.0]])
    assert np.allclose(o.log_luminance(y), np.log(y + 1e-3), rtol=0, atol=1e-14)


# ---------------------------------------------------------------------------
# substep count
# ---------------------------------------------------------------------------

def pin_defocus_library(o):
    """The blur equals scipy's Gaussian filter (same radius, edge mode
    'nearest') along both axes, for grey and RGB input."""
    from scipy import ndimage
    rng = np.random.default_rng(47)
    for sigma, shape in ((0.3, (9, 14)), (1.7, (23, 19)), (4.0, (31, 40, 3))):
        x = rng.uniform(0, 5, size=shape)
        r = o.defocus_radius(sigma)
        want = x
        for ax in (1, 0):
            want = ndimage.gaussian_filter1d(want, sigma, axis=ax, mode="nearest", radius=r)
        assert np.allclose(o.defocus(x, sigma), want, rtol=0, atol=1e-12), sigma


def pin_defocus_closed_forms(o):
    """A constant image is unchanged; a linear ramp is unchanged away from
    the edges (the kernel is symmetric); a point spreads into the outer
    product of the 1-D Gaussian weights, whose variance is about sigma^2."""
    sigma = 2.0
    r = o.defocus_radius(sigma)
    assert r == 6
    c = np.full((20, 25), 3.25)
    assert np.allclose(o.defocus(c, sigma), c, rtol=0, atol=1e-12)
    yy, xx = np.mgrid[0:30, 0:40].astype(np.float64)
    ramp = 0.5 + 0.25 * xx - 0.125 * yy
    got = o.defocus(ramp, sigma)
    assert np.allclose(got[r:-r, r:-r], ramp[r:-r, r:-r], rtol=0, atol=1e-12)
    d = np.zeros((31, 31))
    d[15, 15] = 1.0
    k = np.arange(-r, r + 1)
    g = np.exp(-k * k / (2 * sigma * sigma))
    g /= g.sum()
    assert np.allclose(o.defocus(d, sigma)[15 - r:16 + r, 15 - r:16 + r], np.outer(g, g), rtol=0, atol=1e-15)
    var = float((k * k * g).sum())
    assert abs(var - sigma * sigma) < 0.02 * sigma * sigma


def pin_log_channels(o):
    """Colour events: each channel's own log, channel-major."""
    x = np.array([[[1.0, 0.0, 100.0], [0.5, 2.0, 1e3]]])
    got = o.log_channels(x)
    assert got.shape == (3, 1, 2)
    for c in range(3):
        for i in range(2):
            assert abs(float(got[c, 0, i]) - math.log(x[0, i, c] + 1e-3)) < 1e-12
    # a grey pixel (R = G = B) has the luminance's log in every channel
    g = np.full((2, 2, 3), 7.5)
    assert np.allclose(o.log_channels(g), o.log_luminance(g)[None], rtol=0, atol=1e-12)


def _field(H, W, vec=None):
    m = np.zeros((H, W, 2), F32)
    if vec is not None:
        m[1, 2] = vec
    return m


def pin_adaptive_k(o):
    cases = [((0, 0), 1), ((0.5, 0), 1), ((1, 0), 1), ((1.0001, 0), 2), ((3, 4), 5),
             ((3, 4.0001), 6), ((2.5, 0), 3), ((-7, 0), 7), ((0, -7.5), 8), ((100, 0), 64)]
    for vec, want in cases:
        got = o.adaptive_k(_field(4, 5, vec), _field(4, 5), 64)
        assert got == want, (vec, got, want)
    # the second field counts as much as the first
    assert o.adaptive_k(_field(4, 5, (0.25, 0)), _field(4, 5, (6, 8)), 64) == 10
    # non-finite vectors are left out
    m = _field(4, 5, (3, 4))
    m[0, 0] = (np.nan, 0)
    m[2, 2] = (np.inf, 1)
    assert o.adaptive_k(m, _field(4, 5), 64) == 5
    # brute force: the smallest k with k*k >= the largest squared length
    rng = np.random.default_rng(7)
    for _ in range(50):
        mA = rng.normal(0, rng.uniform(0.1, 20), size=(3, 4, 2)).astype(F32)
        mB = rng.normal(0, rng.uniform(0.1, 20), size=(3, 4, 2)).astype(F32)
        big = max(float(v[0]) ** 2 + float(v[1]) ** 2 for v in
                  list(mA.reshape(-1, 2)) + list(mB.reshape(-1, 2)))
        want = next(k for k in range(1, 10_000) if k * k >= big)
        assert o.adaptive_k(mA, mB, 128) == min(want, 128)


# ---------------------------------------------------------------------------
# endpoint depth
# ---------------------------------------------------------------------------

def pin_endpoint_depth_affine(o):
    H, W = 8, 9
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    Z_B = (1.0 + 0.5 * xx + 0.25 * yy).astype(F32)
    m_A = np.zeros((H, W, 2), F32)
    m_A[..., 0] = -1.5
    m_A[..., 1] = 0.75
    got = o.endpoint_depth(Z_B, m_A).astype(np.float64)
    sx = np.minimum(xx + 1.5, W - 1)
    sy = np.maximum(yy - 0.75, 0.0)
    want = 1.0 + 0.5 * sx + 0.25 * sy
    assert np.array_equal(got, want), np.abs(got - want).max()


# ---------------------------------------------------------------------------
# forward splat
# ---------------------------------------------------------------------------

def pin_splat_bruteforce(o):
    """Scatter z-buffer == per-target enumeration of every covering source."""
    rng = np.random.default_rng(11)
    for trial in range(6):
        H, W = 8, 8
        if trial % 2 == 0:
            m = (np.round(rng.uniform(-3, 3, size=(H, W, 2)) * 4) / 4).astype(F32)
        else:
            m = rng.uniform(-3, 3, size=(H, W, 2)).astype(F32)
        Z_A = rng.choice(np.array([1.0, 2.0, 3.0, -1.0], F32), size=(H, W))
        Z_B = rng.choice(np.array([1.0, 2.0, 3.0], F32), size=(H, W))
        Zend = o.endpoint_depth(Z_B, m)
        for K, j in ((8, 3), (4, 2), (7, 5)):
            f = F32(j) / F32(K)
            zbuf = o.splat_forward(m, Z_A, Zend, f)
            for ty in range(H):
                for tx in range(W):
                    best = None
                    for py in range(H):
                        for px in range(W):
                            qx = F32(px) - f * m[py, px, 0]
                            qy = F32(py) - f * m[py, px, 1]
                            zt = Z_A[py, px] + f * (Zend[py, px] - Z_A[py, px])
                            if not zt > 0:
                                continue
                            x0, y0 = math.floor(qx), math.floor(qy)
                            okx = tx == x0 or (qx - x0 > 0 and tx == x0 + 1)
                            oky = ty == y0 or (qy - y0 > 0 and ty == y0 + 1)
                            if okx and oky:
                                cand = (float(zt), py * W + px)
                                if best is None or cand < best:
                                    best = cand
                    key = int(zbuf[ty, tx])
                    if best is None:
                        assert key == 0xFFFF_FFFF_FFFF_FFFF, (trial, tx, ty)
                    else:
                        depth = float(np.uint32(key >> 32).view(F32))
                        assert (depth, key & 0xFFFF_FFFF) == best, (trial, tx, ty, best)


def pin_integer_translation(o):
    """Content moving by an integer u per substep (K a power of two):
    every sub-frame is an exact shift of L_A where both ends are in view."""
    rng = np.random.default_rng(3)
    H, W, K = 16, 20, 4
    for u in ((1, 2), (-2, 1), (0, -1)):
        L_A = rng.normal(0, 2, size=(H, W)).astype(F32)
        L_B = rng.normal(0, 2, size=(H, W)).astype(F32)
        ux, uy = u
        for y in range(H):
            for x in range(W):
                sx, sy = x - K * ux, y - K * uy
                if 0 <= sx < W and 0 <= sy < H:
                    L_B[y, x] = L_A[sy, sx]
        m = np.zeros((H, W, 2), F32)
        m[..., 0] = -K * ux
        m[..., 1] = -K * uy
        Z = np.full((H, W), F32(2.0))
        pair = o.Pair(L_A, L_B, m, m.copy(), Z, Z.copy())
        Ls, _ = o.interpolate(pair, K, 1, K)
        for j in range(1, K):
            Lj = Ls[j - 1]
            for y in range(H):
                for x in range(W):
                    ax, ay = x - j * ux, y - j * uy            # A source
                    bx, by = x + (K - j) * ux, y + (K - j) * uy  # B sample
                    a_in = 0 <= ax < W and 0 <= ay < H
                    b_in = 0 <= bx < W and 0 <= by < H
                    if a_in:
                        assert Lj[y, x] == L_A[ay, ax], (u, j, x, y)
                    elif b_in:
                        assert Lj[y, x] == L_B[by, bx], (u, j, x, y)


def pin_static_scene(o):
    rng = np.random.default_rng(5)
    H, W, K = 12, 10, 7
    L = rng.normal(0, 3, size=(H, W)).astype(F32)
    m = np.zeros((H, W, 2), F32)
    Z_A = rng.uniform(0.5, 5, size=(H, W)).astype(F32)
    Z_A[2:5, 3:6] = -1.0                      # some A sources invisible
    Z_B = rng.uniform(0.5, 5, size=(H, W)).astype(F32)
    pair = o.Pair(L, L.copy(), m, m.copy(), Z_A, Z_B)
    for mode in (o.BLEND_TIME, o.BLEND_B_PRIMARY):
        Ls, _ = o.interpolate(pair, K, 0, K + 1, mode)
        for j in range(K + 1):
            assert np.array_equal(Ls[j], L), (mode, j)


def _square_scene(u=(2, 1), K=4):
    H, W = 24, 24
    ux, uy = u
    Z_A = np.full((H, W), F32(5.0))
    Z_B = np.full((H, W), F32(5.0))
    m_A = np.zeros((H, W, 2), F32)
    sq = (slice(4, 10), slice(4, 10))
    Z_A[sq] = 1.0
    m_A[sq + (0,)] = -K * ux
    m_A[sq + (1,)] = -K * uy
    Z_B[4 + K * uy:10 + K * uy, 4 + K * ux:10 + K * ux] = 1.0
    return H, W, Z_A, Z_B, m_A


def pin_occlusion(o):
    """A near square moving over a static far background: it wins wherever
    it lands, and the background it uncovers is a hole of the A splat."""
    K, u = 4, (2, 1)
    H, W, Z_A, Z_B, m_A = _square_scene(u, K)
    Zend = o.endpoint_depth(Z_B, m_A)
    for j in (1, 2, 3):
        zbuf = o.splat_forward(m_A, Z_A, Zend, F32(j) / F32(K))
        idx = (zbuf & np.uint64(0xFFFF_FFFF)).astype(np.int64)
        for y in range(H):
            for x in range(W):
                sx, sy = x - j * u[0], y - j * u[1]
                if 4 <= sx < 10 and 4 <= sy < 10:
                    assert idx[y, x] == sy * W + sx, (j, x, y)
                elif 4 <= x < 10 and 4 <= y < 10:
                    assert zbuf[y, x] == o.EMPTY_KEY, (j, x, y)
                else:
                    assert idx[y, x] == y * W + x, (j, x, y)


def pin_depth_interp(o):
    """Eq. 7 on one static source: Z~ = (1-f) Z_A + f Z_B, exact here."""
    H, W = 3, 3
    m = np.zeros((H, W, 2), F32)
    Z_A = np.full((H, W), F32(2.0))
    Z_B = np.full((H, W), F32(4.0))
    Zend = o.endpoint_depth(Z_B, m)
    for K, j, want in ((4, 1, 2.5), (4, 3, 3.5), (8, 1, 2.25)):
        zbuf = o.splat_forward(m, Z_A, Zend, F32(j) / F32(K))
        depth = (zbuf >> np.uint64(32)).astype(np.uint32).view(F32)
        assert np.all(depth == F32(want)), (K, j, depth)


def pin_tie_break(o):
    """Equal depths: the smaller source index wins; a nearer one beats both."""
    H, W, K = 1, 4, 2
    m = np.zeros((H, W, 2), F32)
    m[0, 0, 0] = -2.0      # lands on x = 1 at f = 1/2
    m[0, 2, 0] = 2.0       # lands on x = 1 at f = 1/2
    Z = np.full((H, W), F32(3.0))
    Zend = o.endpoint_depth(Z, m)
    zbuf = o.splat_forward(m, Z, Zend, F32(1) / F32(K))
    assert int(zbuf[0, 1]) & 0xFFFF_FFFF == 0
    Z2 = Z.copy()
    Z2[0, 2] = 2.5                            # Z~ = 2.5 + (3 - 2.5) / 2 = 2.75 < 3
    zbuf = o.splat_forward(m, Z2, o.endpoint_depth(Z, m), F32(1) / F32(K))
    assert int(zbuf[0, 1]) & 0xFFFF_FFFF == 2
    assert zbuf[0, 0] == o.EMPTY_KEY and int(zbuf[0, 3]) & 0xFFFF_FFFF == 3


# ---------------------------------------------------------------------------
# resolve, gather, blend
# ---------------------------------------------------------------------------

def pin_gather_affine(o):
    """Bilinear sampling reproduces an affine L_B exactly at dyadic points."""
    H, W, K = 12, 12, 4
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    L_B = (0.5 + 0.25 * xx - 0.125 * yy).astype(F32)
    L_A = np.zeros((H, W), F32)
    m_A = np.zeros((H, W, 2), F32)
    m_B = np.zeros((H, W, 2), F32)
    m_B[..., 0] = 1.5
    m_B[..., 1] = -0.75
    Z = np.full((H, W), F32(-1.0))           # no A source is visible
    pair = o.Pair(L_A, L_B, m_A, m_B, Z, Z.copy())
    Ls, holes = o.interpolate(pair, K, 1, K)
    for j in range(1, K):
        g = 1.0 - j / K
        sx, sy = xx - g * 1.5, yy + g * 0.75
        inside = (sx >= 0) & (sx <= W - 1) & (sy >= 0) & (sy <= H - 1)
        want = np.where(inside, 0.5 + 0.25 * sx - 0.125 * sy, (j / K) * L_B)
        assert np.array_equal(Ls[j - 1].astype(np.float64), want), j
        assert np.array_equal(holes[j - 1], np.where(inside, 1, 3)), j


def pin_blend_modes(o):
    H, W, K = 2, 3, 4
    L_A = np.full((H, W), F32(0.5))
    L_B = np.full((H, W), F32(1.5))
    m = np.zeros((H, W, 2), F32)
    far = np.zeros((H, W, 2), F32)
    far[..., 0] = 100.0                      # B sample always outside the image
    Zok = np.full((H, W), F32(1.0))
    Zbad = np.full((H, W), F32(-1.0))
    cases = [  # (m_B, Z, TIME value at j=1, B_PRIMARY value at j=1)
        (m, Zok, 0.75, 1.5),                 # both valid
        (far, Zok, 0.5, 0.5),                # only A valid
        (m, Zbad, 1.5, 1.5),                 # only B valid
        (far, Zbad, 0.75, 1.5),              # neither: lerp(L_A(q), L_B(q), alpha)
    ]
    for m_B, Z, want_t, want_b in cases:
        pair = o.Pair(L_A, L_B, m, m_B, Z, Z.copy())
        lt, _ = o.interpolate(pair, K, 1, 2, o.BLEND_TIME)
        lb, _ = o.interpolate(pair, K, 1, 2, o.BLEND_B_PRIMARY)
        assert np.all(lt == F32(want_t)) and np.all(lb == F32(want_b)), (want_t, want_b)


# ---------------------------------------------------------------------------
# two-splat and joint warp
# ---------------------------------------------------------------------------

def pin_start_depth_affine(o):
    """Z_A sampled at p + m_B(p), clamped: exact on an affine depth map."""
    H, W = 7, 10
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    Z_A = (2.0 + 0.25 * xx - 0.5 * yy).astype(F32)
    m_B = np.zeros((H, W, 2), F32)
    m_B[..., 0] = 2.5
    m_B[..., 1] = -1.25
    got = o.start_depth(Z_A, m_B).astype(np.float64)
    sx = np.minimum(xx + 2.5, W - 1)
    sy = np.maximum(yy - 1.25, 0.0)
    assert np.array_equal(got, 2.0 + 0.25 * sx - 0.5 * sy)


def pin_backward_splat_reversal(o):
    """Time reversal: splatting B back to fraction f is splatting a keyframe
    with motion -m_B forward by 1 - f with the depth roles of A and B
    swapped (Eq. 5 and Eq. 7 are symmetric under t -> 1 - t).  On dyadic
    inputs every value is exact in both forms, so the z-buffers agree bit
    for bit; the forward splat is pinned by brute force above."""
    rng = np.random.default_rng(37)
    H, W = 9, 11
    for trial in range(4):
        m_B = (rng.integers(-12, 13, size=(H, W, 2)) / 4.0).astype(F32)
        Z_A = rng.choice(np.array([1.0, 2.0, 3.0, 4.0], F32), size=(H, W))
        Z_B = rng.choice(np.array([1.0, 2.0, 3.0, -1.0], F32), size=(H, W))
        Zs = o.start_depth(Z_A, m_B)
        for K, j in ((8, 3), (4, 1), (8, 6)):
            f = F32(j) / F32(K)
            got = o.splat_backward(m_B, Z_B, Zs, f)
            neg = (-m_B).astype(F32)
            want = o.splat_forward(neg, Z_B, o.endpoint_depth(Z_A, neg), F32(K - j) / F32(K))
            assert np.array_equal(got, want), (trial, K, j)


def _layer_scene(u=(2, 1), K=4, seed=41):
    """A textured near square (depth 1) moving by u per substep over a static
    textured far background (depth 5): keyframes, motion and the exact
    frame at every substep."""
    rng = np.random.default_rng(seed)
    H, W = 22, 26
    ux, uy = u
    bg = rng.normal(0, 2, size=(H, W)).astype(F32)
    tex = rng.normal(4, 1, size=(6, 6)).astype(F32)

    def frame(j):
        L = bg.copy()
        Z = np.full((H, W), F32(5.0))
        y0, x0 = 4 + j * uy, 4 + j * ux
        L[y0:y0 + 6, x0:x0 + 6] = tex
        Z[y0:y0 + 6, x0:x0 + 6] = 1.0
        return L, Z

    L_A, Z_A = frame(0)
    L_B, Z_B = frame(K)
    m_A = np.zeros((H, W, 2), F32)
    m_B = np.zeros((H, W, 2), F32)
    m_A[4:10, 4:10] = (-K * ux, -K * uy)
    m_B[4 + K * uy:10 + K * uy, 4 + K * ux:10 + K * ux] = (-K * ux, -K * uy)
    return (L_A, L_B, m_A, m_B, Z_A, Z_B), frame


def pin_two_splat_layers(o):
    """The near square over the static background: the two-splat warp (either
    blend) and the joint warp rebuild every intermediate frame exactly, and
    B's holes are exactly the background the square covers in B but not at
    the substep (A's holes: covered in A but not at the substep)."""
    K, u = 4, (2, 1)
    args, frame = _layer_scene(u, K)
    pair = o.Pair(*args)
    H, W = pair.shape
    yy, xx = np.mgrid[0:H, 0:W]

    def square(j):
        y0, x0 = 4 + j * u[1], 4 + j * u[0]
        return (yy >= y0) & (yy < y0 + 6) & (xx >= x0) & (xx < x0 + 6)

    for mode in (o.WARP_SPLAT | o.BLEND_B_PRIMARY, o.WARP_SPLAT | o.BLEND_TIME,
                 o.WARP_JOINT | o.BLEND_TIME):
        Ls, holes = o.interpolate(pair, K, 1, K, mode)
        for j in range(1, K):
            want, _ = frame(j)
            assert np.array_equal(Ls[j - 1], want), (mode, j)
            if mode & o.WARP_MASK == o.WARP_SPLAT:
                bhole = square(K) & ~square(j)
                ahole = square(0) & ~square(j)
                assert np.array_equal((holes[j - 1] & 2) != 0, bhole), (mode, j)
                assert np.array_equal((holes[j - 1] & 1) != 0, ahole), (mode, j)


def pin_joint_priority(o):
    """An A source and a B source land on the same pixel: the nearer wins,
    and at equal depth B (the primary keyframe) wins."""
    H, W, K = 1, 7, 2
    L_A = np.arange(1, W + 1, dtype=F32).reshape(H, W)
    L_B = (10 * L_A).astype(F32)
    m_A = np.zeros((H, W, 2), F32)
    m_B = np.zeros((H, W, 2), F32)
    m_A[0, 0, 0] = -4.0         # A's x = 0 lands on x = 2 at f = 1/2; endpoint B x = 4
    m_B[0, 5, 0] = -6.0         # B's x = 5 lands on x = 2 at f = 1/2; endpoint A x = 0 (clamped)
    for e4, e5, want in ((3.0, 3.0, L_B[0, 5]), (2.0, 3.0, L_A[0, 0]), (3.0, 2.0, L_B[0, 5])):
        Z_A = np.full((H, W), F32(100.0))
        Z_B = np.full((H, W), F32(100.0))
        Z_A[0, 0] = 1.0
        Z_B[0, 4] = e4          # A's depth at f = 1/2: (1 + e4) / 2
        Z_B[0, 5] = e5          # B's depth at f = 1/2: (1 + e5) / 2
        pair = o.Pair(L_A, L_B, m_A, m_B, Z_A, Z_B)
        Ls, holes = o.interpolate(pair, K, 1, 2, o.WARP_JOINT | o.BLEND_TIME)
        assert Ls[0][0, 2] == want, (e4, e5, Ls[0][0, 2])
        assert holes[0][0, 2] == (2 if want < 10 else 1), (e4, e5)


# ---------------------------------------------------------------------------
# event emission
# ---------------------------------------------------------------------------

def pin_goldens(o):
    for name in ("ramp_refractory.txt", "multi_crossing.txt", "exact_floor_off.txt"):
        kv, want = read_golden(name)
        H, W = int(kv["H"]), int(kv["W"])
        pair = zero_motion_pair(o, np.full((H, W), float(kv["L_A"])),
                                np.full((H, W), float(kv["L_B"])),
                                t0=int(kv["t0"]), t1=int(kv["t1"]))
        C = float(kv["C"])
        sensor = o.Sensor(C_on=C, C_off=C, refractory_us=int(kv["refractory"]),
                          K=int(kv["K"]))
        L_ref = np.zeros((H, W), F32)
        t_last = np.full((H, W), o.T_LAST_INIT, np.int32)
        ev, R, _, K = o.step(pair, sensor, L_ref, t_last)
        got = sorted((int(e[0]), int(e[1]), int(e[2]), int(e[3])) for e in ev)
        assert got == sorted(tuple(e) for e in want), (name, got)
        assert float(R[0, 0]) == float(Decimal(kv["L_ref_end"])), (name, float(R[0, 0]))


def pin_uniform_ramp(o):
    """A uniform log ramp dL with zero motion gives floor(dL / C) events per
    pixel, evenly spaced in time (interpolation is exact for a ramp)."""
    rng = np.random.default_rng(9)
    H, W, K, C = 6, 7, 8, 0.2
    t0, t1 = 1000, 1000 + 16667
    L_A = rng.uniform(-2, 2, size=(H, W)).astype(F32)
    L_B = (L_A + F32(1.1)).astype(F32)
    pair = zero_motion_pair(o, L_A, L_B, t0=t0, t1=t1)
    ev, R, _, _ = o.step(pair, o.Sensor(C_on=C, C_off=C, K=K), L_A.copy())
    for y in range(H):
        for x in range(W):
            sel = ev[(ev[:, 0] == x) & (ev[:, 1] == y)]
            dL = float(L_B[y, x]) - float(L_A[y, x])
            n = math.floor(dL / float(F32(C)))
            assert len(sel) == n == 5, (x, y, len(sel))
            assert np.all(sel[:, 3] == 1)
            ts = np.sort(sel[:, 2])
            want = [t0 + k * float(F32(C)) / dL * (t1 - t0) for k in range(1, n + 1)]
            assert np.all(np.abs(ts - np.array(want)) <= 2.0), (ts, want)


def pin_constant_frame_no_events(o):
    rng = np.random.default_rng(13)
    H, W = 10, 11
    for L0 in (0.0, 1.7):
        L = np.full((H, W), F32(L0))
        pair = zero_motion_pair(o, L, L.copy())
        ev, _, _, _ = o.step(pair, o.Sensor(K=8), L.copy())
        assert len(ev) == 0
        # any motion over a constant image still gives constant sub-frames
        m = rng.uniform(-4, 4, size=(H, W, 2)).astype(F32)
        Z = rng.uniform(0.5, 5, size=(H, W)).astype(F32)
        pair = o.Pair(L, L.copy(), m, m.copy(), Z, Z.copy())
        ev, _, _, _ = o.step(pair, o.Sensor(K=5), L.copy())
        assert len(ev) == 0


def _random_pair(o, seed, H=20, W=24, amp=3.0):
    rng = np.random.default_rng(seed)
    L_A = rng.normal(0, amp, size=(H, W)).astype(F32)
    m = rng.normal(0, 2.0, size=(H, W, 2)).astype(F32)
    L_B = (L_A + rng.normal(0, 0.5, size=(H, W))).astype(F32)
    Z_A = rng.uniform(0.5, 5, size=(H, W)).astype(F32)
    Z_B = rng.uniform(0.5, 5, size=(H, W)).astype(F32)
    return o.Pair(L_A, L_B, m, (m + F32(0.25)).astype(F32), Z_A, Z_B, 0, 16667)


def pin_polarity_symmetry(o):
    pair = _random_pair(o, 17)
    sensor = o.Sensor(C_on=0.2, C_off=0.2, K=6)
    ev, R, _, _ = o.step(pair, sensor, pair.L_A.copy())
    neg = o.Pair(-pair.L_A, -pair.L_B, pair.m_A, pair.m_B, pair.Z_A, pair.Z_B, 0, 16667)
    ev2, R2, _, _ = o.step(neg, sensor, -pair.L_A)
    assert len(ev) > 50
    flipped = ev2.copy()
    flipped[:, 3] = 1 - flipped[:, 3]
    assert np.array_equal(o.canonical(ev), o.canonical(flipped))
    assert np.array_equal(R, -R2)


def pin_residual_and_sum(o):
    """After a pair: |L_B - L_ref| < C, and the reference moved by exactly
    the signed sum of C over the emitted crossings (no refractory period)."""
    C = 0.2
    pair = _random_pair(o, 19)
    L0 = pair.L_A.copy()
    ev, R, _, _ = o.step(pair, o.Sensor(C_on=C, C_off=C, K=5), L0)
    c = float(F32(C))
    assert np.all(np.abs(pair.L_B.astype(np.float64) - R) < c * (1 + 1e-5))
    H, W = pair.shape
    moved = np.zeros((H, W))
    np.add.at(moved, (ev[:, 1], ev[:, 0]), np.where(ev[:, 3] == 1, c, -c))
    assert np.allclose(R.astype(np.float64) - L0, moved, rtol=0, atol=1e-4)


def pin_timestamps(o):
    pair = _random_pair(o, 23)
    t_last = np.full(pair.shape, o.T_LAST_INIT, np.int32)
    ev, _, _, _ = o.step(pair, o.Sensor(K=7, refractory_us=150), pair.L_A.copy(), t_last)
    assert len(ev) > 20
    assert ev[:, 2].min() >= pair.t0_us and ev[:, 2].max() <= pair.t1_us
    H, W = pair.shape
    for flat in range(H * W):
        y, x = divmod(flat, W)
        ts = ev[(ev[:, 0] == x) & (ev[:, 1] == y), 2]       # emission order
        assert np.all(np.diff(ts) >= 150), (x, y, ts)


def pin_mismatch(o):
    """Eq. 8: rising pixels use theta_on, falling pixels theta_off."""
    L_A = np.zeros((1, 2), F32)
    L_B = np.array([[1.1, -1.1]], F32)
    pair = zero_motion_pair(o, L_A, L_B)
    on = np.array([[0.25, 0.25]], F32)
    off = np.array([[0.5, 0.5]], F32)
    s = o.Sensor(theta_on=on, theta_off=off, K=4)
    ev, _, _, _ = o.step(pair, s, L_A.copy())
    p0 = ev[ev[:, 0] == 0]
    p1 = ev[ev[:, 0] == 1]
    assert len(p0) == 4 and np.all(p0[:, 3] == 1)
    assert len(p1) == 2 and np.all(p1[:, 3] == 0)


def pin_crossing_count_exact(o):
    getcontext().prec = 80
    rng = np.random.default_rng(29)
    cases = [(F32(1.0), F32(0.2)), (F32(0.6), F32(0.2)), (F32(1.1), F32(0.2)),
             (F32(0.75), F32(0.25)), (F32(3.0), F32(0.1))]
    for _ in range(300):
        c = F32(rng.uniform(0.01, 1.0))
        a = F32(c * rng.integers(1, 40) * (1 + rng.choice([-1, 0, 1]) * 1e-7))
        if a >= c:
            cases.append((a, c))
    for a, c in cases:
        want = int((Decimal(float(a)) / Decimal(float(c))).to_integral_value(rounding="ROUND_FLOOR"))
        assert o.crossing_count(a, c) == want, (float(a), float(c))
    # no cap: a count far above any implementation's per-substep bound is exact
    for a, c in ((F32(1e6), F32(0.01)), (F32(20000.0), F32(0.2)), (F32(13107.25), F32(0.2))):
        want = int((Decimal(float(a)) / Decimal(float(c))).to_integral_value(rounding="ROUND_FLOOR"))
        assert want > 65535 and o.crossing_count(a, c) == want, (float(a), float(c))
    # an infinite difference has no count; a stated limit bounds it
    try:
        o.crossing_count(F32(np.inf), F32(0.2))
    except ValueError:
        pass
    else:
        raise AssertionError("an infinite |dL| must have no crossing count")
    assert o.crossing_count(F32(np.inf), F32(0.2), count_limit=7) == 7
    assert o.crossing_count(F32(3.0), F32(0.1), count_limit=7) == 7
    assert o.crossing_count(F32(0.6), F32(0.2), count_limit=7) == 3   # 3 * 0.2f < 0.6f


def pin_crop_margin(o):
    """Content translating by an integer u per substep into view: with an
    over-rendered margin of K|u| pixels every inner sub-frame is the exact
    shifted texture, so the cropped events equal the event model run on the
    exact inner frames (in cropped coordinates) and the margin's state is
    untouched; without the margin the boundary pixels differ."""
    rng = np.random.default_rng(53)
    K, u, m = 4, (1, -1), 4
    Hi, Wi = 14, 18                                    # inner size
    big = rng.normal(0, 2, size=(Hi + 2 * m + 2 * K, Wi + 2 * m + 2 * K)).astype(F32)

    def frame(j, mm):                                  # texture moving by j*u, frame with margin mm
        oy, ox = K + m - mm - j * u[1], K + m - mm - j * u[0]
        return big[oy:oy + Hi + 2 * mm, ox:ox + Wi + 2 * mm].copy()

    def pair_for(mm):
        H, W = Hi + 2 * mm, Wi + 2 * mm
        mv = np.zeros((H, W, 2), F32)
        mv[..., 0] = -K * u[0]
        mv[..., 1] = -K * u[1]
        Z = np.full((H, W), F32(2.0))
        return o.Pair(frame(0, mm), frame(K, mm), mv, mv.copy(), Z, Z.copy(), 0, 16667)

    s = o.Sensor(C_on=0.2, C_off=0.2, K=K)
    p = pair_for(m)
    L0 = p.L_A.copy()
    t0 = np.full(p.shape, o.T_LAST_INIT, np.int32)
    ev, R, tl, _ = o.step(p, s, L0, t0, env_id=2, crop_margin=m)
    exact = [frame(j, 0) for j in range(K + 1)]
    want, Rw, _ = o.emit_events(exact, 0, 16667, s, exact[0].copy(), np.full((Hi, Wi), o.T_LAST_INIT, np.int32), env_id=2)
    assert len(ev) > 100 and np.array_equal(o.canonical(ev), o.canonical(want))
    assert np.array_equal(R[m:-m, m:-m], Rw)
    ring = np.ones(p.shape, bool)
    ring[m:-m, m:-m] = False
    assert np.array_equal(R[ring], L0[ring]) and np.all(tl[ring] == o.T_LAST_INIT)
    ev0, _, _, _ = o.step(pair_for(0), s, frame(0, 0), None, env_id=2)
    assert not np.array_equal(o.canonical(ev0), o.canonical(want))


# ---------------------------------------------------------------------------
# noise events
# ---------------------------------------------------------------------------

def pin_philox_kat(o):
    """The generator against its published known-answer vectors."""
    n = 0
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            ctr, key, want = [[int(w, 16) for w in part.split()] for part in line.split("|")]
            got = [int(v) for v in o.philox4x32(ctr, key)]
            assert got == want, (ctr, key, [hex(v) for v in got])
            n += 1
    assert n == 3


def _flat_pair(o, H, W, L, K, t1=16667):
    pair = zero_motion_pair(o, np.full((H, W), F32(L)), np.full((H, W), F32(L)), t1=t1)
    return pair


def _binomial_ok(count, n, p, z=5.0):
    mean = n * p
    sd = math.sqrt(n * p * (1 - p))
    return abs(count - mean) <= z * sd + 1, (count, mean, sd)


def pin_leak_rate(o):
    """Leak events alone on constant frames: ON only, inside the pair, and
    their number a Binomial(pixels x substeps, r_l Dt) draw."""
    H, W, K = 64, 64, 10
    pair = _flat_pair(o, H, W, 0.5, K)
    nz = o.Noise(leak_rate_hz=20.0, seed=0x1234_5678_9ABC_DEF0, pair_index=3)
    ev, R, _, _ = o.step(pair, o.Sensor(K=K, noise=nz), pair.L_A.copy())
    assert np.array_equal(R, pair.L_A)                     # R23: the reference stays
    p = 20.0 * (16667 / K) * 1e-6
    ok, info = _binomial_ok(len(ev), H * W * K, p)
    assert ok, info
    assert len(ev) > 50 and np.all(ev[:, 3] == 1)
    assert ev[:, 2].min() >= 0 and ev[:, 2].max() <= 16667
    # each substep holds its share: times fall in K equal bins about evenly
    bins = np.bincount(np.minimum(ev[:, 2] * K // 16667, K - 1), minlength=K)
    assert bins.min() > 0


def pin_shot_darkness(o):
    """Shot noise alone: none where the normalised intensity is 1, the full
    rate where it is 0, polarity about even."""
    H, W, K = 48, 64, 8
    L = np.zeros((H, W), F32)
    L[:, W // 2:] = 3.0                                       # normalised intensity 1 there
    pair = zero_motion_pair(o, L, L.copy())
    nz = o.Noise(shot_rate_hz=3000.0, shot_L0=0.0, shot_inv_range=1.0 / 3.0, seed=99)
    ev, _, _, _ = o.step(pair, o.Sensor(K=K, noise=nz), L.copy())
    assert np.all(ev[:, 0] < W // 2)
    p = 3000.0 * (1000 / K) * 1e-6
    ok, info = _binomial_ok(len(ev), H * (W // 2) * K, p)
    assert ok, info
    ok, info = _binomial_ok(int(ev[:, 3].sum()), len(ev), 0.5)
    assert ok, info


def pin_hot_pixels(o):
    """Hot pixels alone: a fixed set of about the asked share of pixels,
    every event on it, at the hot rate."""
    H, W, K = 64, 80, 6
    pair = _flat_pair(o, H, W, 1.0, K, t1=60000)
    nz = o.Noise(hot_rate_hz=20.0, hot_fraction=0.05, seed=7)
    hot = o.hot_pixels(H, W, nz)
    ok, info = _binomial_ok(int(hot.sum()), H * W, 0.05)
    assert ok, info
    ev, _, _, _ = o.step(pair, o.Sensor(K=K, noise=nz), pair.L_A.copy())
    assert len(ev) > 0 and np.all(hot[ev[:, 1], ev[:, 0]])
    p = 20.0 * (60000 / K) * 1e-6
    ok, info = _binomial_ok(len(ev), int(hot.sum()) * K, p)
    assert ok, info


def pin_noise_off_and_seeded(o):
    """Zero rates add nothing; the same seed and pair index give the same
    events, another pair index other events."""
    pair = _random_pair(o, 43)
    base, _, _, _ = o.step(pair, o.Sensor(K=5), pair.L_A.copy())
    off, _, _, _ = o.step(pair, o.Sensor(K=5, noise=o.Noise(seed=5)), pair.L_A.copy())
    assert np.array_equal(o.canonical(base), o.canonical(off))
    nz = o.Noise(leak_rate_hz=40.0, shot_rate_hz=40.0, seed=5, pair_index=1)
    a, _, _, _ = o.step(pair, o.Sensor(K=5, noise=nz), pair.L_A.copy())
    b, _, _, _ = o.step(pair, o.Sensor(K=5, noise=nz), pair.L_A.copy())
    nz2 = o.Noise(leak_rate_hz=40.0, shot_rate_hz=40.0, seed=5, pair_index=2)
    c, _, _, _ = o.step(pair, o.Sensor(K=5, noise=nz2), pair.L_A.copy())
    assert np.array_equal(o.canonical(a), o.canonical(b)) and len(a) > len(base)
    assert not np.array_equal(o.canonical(a), o.canonical(c))


# ---------------------------------------------------------------------------
# voxel grid
# ---------------------------------------------------------------------------

def pin_voxel_closed_forms(o):
    """Hand-worked cases on a dyadic time scale ((B - 1) / (t1 - t0) = 4 / 1024
    = 2^-8, exact): an event on a bin centre fills that bin alone, one halfway
    between two centres gives each 1/2, one at tau = 1023/256 gives bin 3 the
    weight 1/256 and bin 4 the rest; other envs and times outside [t0, t1)
    add nothing; every non-empty (polarity, bin) plane peaks at exactly 1."""
    ev = np.array([[1, 2, 256, 1, 0],      # tau = 1.0   -> bin 1
                   [3, 0, 384, 0, 0],      # tau = 1.5   -> bins 1, 2 halves
                   [3, 0, 1023, 0, 0],     # tau = 3.996 -> bin 3 (and 4)
                   [0, 0, 100, 1, 1],      # another env
                   [0, 1, 1024, 1, 0],     # t = t1: outside the window
                   [0, 1, -1, 1, 0]])      # before t0
    acc = o.voxel_counts(ev, 0, 3, 4, 0, 1024, 5)
    assert acc[1, 1, 2, 1] == 1.0 and acc[1].sum() == 1.0
    assert acc[0, 1, 0, 3] == 0.5 and acc[0, 2, 0, 3] == 0.5
    assert acc[0, 3, 0, 3] == 1.0 / 256.0 and acc[0, 4, 0, 3] == 255.0 / 256.0
    assert acc.sum() == 3.0
    v = o.voxel_grid(ev, 0, 3, 4, 0, 1024, 5)
    assert v[1, 1, 2, 1] == 1.0 and v[0, 1, 0, 3] == 1.0 and v[0, 2, 0, 3] == 1.0
    assert v[0, 3, 0, 3] == 1.0 and v[0, 4, 0, 3] == 1.0
    assert np.count_nonzero(v) == 5


def pin_voxel_brute_force(o):
    """Linear interpolation in time written as the hat function: bin b of a
    voxel gets max(0, 1 - |tau - b|) from each event at real position tau
    (exact rationals, one event at a time), then each plane is divided by its
    maximum.  Agrees with the grid to float64 rounding on random events,
    including many events in one voxel (no bound on the count)."""
    rng = np.random.default_rng(83)
    n, H, W, B, t0, t1 = 400, 3, 4, 7, 5000, 91000
    ev = np.stack([rng.integers(0, W, n), rng.integers(0, H, n), rng.integers(t0 - 900, t1 + 900, n),
                   rng.integers(0, 2, n), rng.integers(0, 2, n)], axis=1)
    ev[:150, 0:2] = (1, 2)                  # a crowded voxel
    ev[:150, 4] = 1
    want = np.zeros((2, B, H, W))
    for x, y, t, p, e in ev.tolist():
        if e != 1 or not (t0 <= t < t1):
            continue
        tau = Fraction(t - t0) * (B - 1) / (t1 - t0)
        for b in range(B):
            w = 1 - abs(tau - b)
            if w > 0:
                want[p, b, y, x] += float(w)
    acc = o.voxel_counts(ev, 1, H, W, t0, t1, B)
    assert np.allclose(acc, want, rtol=1e-12, atol=1e-12)
    mx = want.reshape(2, B, -1).max(axis=2)
    norm = np.where(mx[:, :, None, None] > 0, want / np.where(mx > 0, mx, 1)[:, :, None, None], 0.0)
    assert np.allclose(o.voxel_grid(ev, 1, H, W, t0, t1, B), norm, rtol=1e-12, atol=1e-12)


def pin_voxel_invariants(o):
    """Random events: each event in the window adds exactly one unit of
    weight, whose centroid is its exact time position; each non-empty plane
    of the normalised grid has maximum 1."""
    rng = np.random.default_rng(59)
    n, H, W, B, t0, t1 = 3000, 9, 11, 128, 1000, 501000
    ev = np.stack([rng.integers(0, W, n), rng.integers(0, H, n), rng.integers(t0 - 5000, t1 + 5000, n),
                   rng.integers(0, 2, n), rng.integers(0, 2, n)], axis=1)
    inside = (ev[:, 4] == 1) & (ev[:, 2] >= t0) & (ev[:, 2] < t1)
    acc = o.voxel_counts(ev, 1, H, W, t0, t1, B)
    assert abs(acc.sum() - inside.sum()) <= 1e-9 * inside.sum()
    bidx = np.arange(B).reshape(1, B, 1, 1)
    cent = float((acc * bidx).sum())
    want = float(sum(Fraction(int(t) - t0) * (B - 1) / (t1 - t0) for t in ev[inside, 2]))
    assert abs(cent - want) <= 1e-9 * want
    v = o.voxel_grid(ev, 1, H, W, t0, t1, B)
    mx = v.reshape(2, B, -1).max(axis=2)
    assert np.all((mx == 1.0) | (mx == 0.0)) and np.all(mx[acc.reshape(2, B, -1).max(axis=2) > 0] == 1.0)
    assert v.min() >= 0.0


# ---------------------------------------------------------------------------
# event record
# ---------------------------------------------------------------------------

def pin_event_record(o):
    rec = o.pack_events(np.array([[5, 3, 77, 1, 2]]))
    assert int(rec[0, 0]) == 5 + 3 * 2048 + 1 * 4194304 + 2 * 8388608 and int(rec[0, 1]) == 77
    rng = np.random.default_rng(31)
    ev = np.stack([rng.integers(0, 2048, 100), rng.integers(0, 2048, 100),
                   rng.integers(0, 2 ** 31 - 1, 100), rng.integers(0, 2, 100),
                   rng.integers(0, 512, 100)], axis=1)
    assert np.array_equal(o.unpack_events(o.pack_events(ev).astype(np.uint32)), ev)


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]

"""Float64 oracle of the smooth event-count surrogate and its gradient.

TEST INFRASTRUCTURE (see evis_oracle's header for who may import it).

The paper's event model is piecewise constant in its inputs (Eq. 4 counts
are integers); to fit a contrast threshold and flow corrections by gradient
descent, each crossing indicator 1[|L_j - R_{j-1}| >= C] is replaced by the
logistic sigma((|L_j - R_{j-1}| - C) / tau):

    S(q) = sum_{j=1..K} sigma((|L_j(q) - R_{j-1}(q)| - C) / tau)

where L_j are the sub-frames of the warp (Eq. 5-7 and the blend) and
R_{j-1} is the hard reference-level trajectory of Eq. 4 with threshold C
both ways: R_j = R_{j-1} + p_j n_j C with integer n_j.  Where the n_j do not
change, dR_j/dC = dR_{j-1}/dC + p_j n_j and R does not move with L (so the
derivative through R is exact almost everywhere).  The gradient with
respect to L_A, L_B, the motion fields and C follows by the chain rule
through the blend, the winner-take-all splat (whose value does not depend on
m_A, so d/dm_A = 0 wherever the winners do not change), the bilinear gather
of B and, for C, the reference trajectory.

Discrete decisions (splat winner, B validity, bilinear cell) are inputs
``D`` of the float64 evaluation: ``decisions32`` takes them from the float32
oracle (the decisions the GPU path takes), ``decisions64`` from an
independent float64 splat and gather; finite differences use the latter.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

from . import evis_oracle as o

F32 = np.float32


@dataclass
class Decisions:
    winner: List[np.ndarray]   # per interior j: [H, W] int64 source index, -1 = none
    vB: List[np.ndarray]       # per interior j: [H, W] bool
    cx: List[np.ndarray]       # per interior j: [H, W] int64 floor(s_x) (valid where vB)
    cy: List[np.ndarray]


def reference_levels(frames32, L_ref32, C):
    """Hard float32 reference trajectory of Eq. 4 (threshold C for both
    polarities) from the float32 sub-frames, by the emission step of the
    float32 oracle (events discarded): (R_0..R_K, dR_0/dC..dR_K/dC)."""
    H, W = frames32[0].shape
    R = np.array(L_ref32, F32, copy=True)
    tl = np.full((H, W), o.T_LAST_INIT, np.int64)
    on = np.full((H, W), F32(C))
    traj = [R.copy()]
    dRdC = [np.zeros((H, W))]
    log = o.EventLog()
    Dt = o.substep_dt(0, 16667, len(frames32) - 1)
    c = float(F32(C))
    for j in range(1, len(frames32)):
        before = R.astype(np.float64)
        o.emit_substep(j, frames32[j - 1], frames32[j], R, tl, on, on, 0, 0, Dt, 16667, 0, log, False)
        moved = R.astype(np.float64) - before          # = p_j fl(n_j C)
        pn = np.rint(moved / c)                         # p_j n_j (exact: |error| << 1/2)
        traj.append(R.copy())
        dRdC.append(dRdC[-1] + pn)
    return traj, dRdC


def reference_levels64(frames64, L_ref, C, dRdC=None):
    """The same trajectory in float64: (R, dR/dC).  Counts come from exact
    float64 comparisons, or, with dRdC given (the cumulative p n of another
    evaluation), are held at those: R_j = L_ref + C dRdC_j."""
    if dRdC is not None:
        L_ref = np.asarray(L_ref, np.float64)
        return [L_ref + C * np.asarray(t, np.float64) for t in dRdC], list(dRdC)
    R = np.array(L_ref, np.float64, copy=True)
    traj, dRdC = [R.copy()], [np.zeros_like(R)]
    for j in range(1, len(frames64)):
        d = frames64[j] - R
        a = np.abs(d)
        n = np.where(a >= C, np.floor(a / C), 0.0)
        R = R + np.sign(d) * n * C
        traj.append(R.copy())
        dRdC.append(dRdC[-1] + np.sign(d) * n)
    return traj, dRdC


def decisions32(pair: o.Pair, K: int) -> Decisions:
    """Winners, B validity and gather cells exactly as the float32 path takes them."""
    H, W = pair.shape
    Zend = o.endpoint_depth(pair.Z_B, pair.m_A)
    ux, uy = o.pixel_coords(H, W)
    D = Decisions([], [], [], [])
    for j in range(1, K):
        f = o.substep_fraction(j, K)
        zbuf = o.splat_forward(pair.m_A, pair.Z_A, Zend, f)
        win = np.where(zbuf == o.EMPTY_KEY, -1,
                       (zbuf & np.uint64(0xFFFF_FFFF)).astype(np.int64)).astype(np.int64)
        g = F32(1) - f
        sx = ux - g * pair.m_B[..., 0]
        sy = uy - g * pair.m_B[..., 1]
        vB = (sx >= 0) & (sx <= W - 1) & (sy >= 0) & (sy <= H - 1)
        D.winner.append(win)
        D.vB.append(vB)
        D.cx.append(np.where(vB, np.floor(np.where(vB, sx, 0)), 0).astype(np.int64))
        D.cy.append(np.where(vB, np.floor(np.where(vB, sy, 0)), 0).astype(np.int64))
    return D


def decisions64(L_A, L_B, m_A, m_B, Z_A, Z_B, K: int) -> Decisions:
    """The same decisions from a float64 evaluation of Eq. 5-7 (an
    independent splat: candidates sorted by (target, depth, source))."""
    H, W = L_A.shape
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    mA = np.asarray(m_A, np.float64)
    mB = np.asarray(m_B, np.float64)
    ZA = np.asarray(Z_A, np.float64)
    ZB = np.asarray(Z_B, np.float64)
    # endpoint depth, clamped bilinear in float64
    ex = np.clip(np.nan_to_num(xx - mA[..., 0], nan=0.0), 0, W - 1)
    ey = np.clip(np.nan_to_num(yy - mA[..., 1], nan=0.0), 0, H - 1)
    Zend = _bilinear64(ZB, ex, ey)
    D = Decisions([], [], [], [])
    src = np.arange(H * W)
    for j in range(1, K):
        f = j / K
        qx = (xx - f * mA[..., 0]).ravel()
        qy = (yy - f * mA[..., 1]).ravel()
        zt = (ZA + f * (Zend - ZA)).ravel()
        live = (zt > 0) & np.isfinite(qx) & np.isfinite(qy)
        x0 = np.floor(np.where(live, qx, -8)).astype(np.int64)
        y0 = np.floor(np.where(live, qy, -8)).astype(np.int64)
        fx = np.where(live, qx, 0) - x0
        fy = np.where(live, qy, 0) - y0
        tgt, dep, idx = [], [], []
        for dx, dy, sel in ((0, 0, live), (1, 0, live & (fx > 0)), (0, 1, live & (fy > 0)),
                            (1, 1, live & (fx > 0) & (fy > 0))):
            cx, cy = x0 + dx, y0 + dy
            sel = sel & (cx >= 0) & (cx < W) & (cy >= 0) & (cy < H)
            tgt.append((cy * W + cx)[sel])
            dep.append(zt[sel])
            idx.append(src[sel])
        tgt, dep, idx = np.concatenate(tgt), np.concatenate(dep), np.concatenate(idx)
        order = np.lexsort((idx, dep, tgt))
        tgt, idx = tgt[order], idx[order]
        first = np.ones(len(tgt), bool)
        first[1:] = tgt[1:] != tgt[:-1]
        win = np.full(H * W, -1, np.int64)
        win[tgt[first]] = idx[first]
        g = 1.0 - f
        sx = xx - g * mB[..., 0]
        sy = yy - g * mB[..., 1]
        vB = (sx >= 0) & (sx <= W - 1) & (sy >= 0) & (sy <= H - 1)
        D.winner.append(win.reshape(H, W))
        D.vB.append(vB)
        D.cx.append(np.where(vB, np.floor(np.where(vB, sx, 0)), 0).astype(np.int64))
        D.cy.append(np.where(vB, np.floor(np.where(vB, sy, 0)), 0).astype(np.int64))
    return D


def _bilinear64(img, sx, sy):
    H, W = img.shape
    x0 = np.floor(sx).astype(np.int64)
    y0 = np.floor(sy).astype(np.int64)
    wx, wy = sx - x0, sy - y0
    x1 = np.minimum(x0 + 1, W - 1)
    y1 = np.minimum(y0 + 1, H - 1)
    top = img[y0, x0] + wx * (img[y0, x1] - img[y0, x0])
    bot = img[y1, x0] + wx * (img[y1, x1] - img[y1, x0])
    return top + wy * (bot - top)


def _logistic(u):
    """sigma(u) and sigma'(u) = sigma (1 - sigma) from e = exp(-|u|): the
    derivative as e / (1 + e)^2, which keeps its digits where sigma is
    within rounding of 1 (1 - sigma would cancel to 0 beyond |u| ~ 37)."""
    e = np.exp(-np.abs(u))
    inv = 1.0 / (1.0 + e)
    return np.where(u >= 0, inv, e * inv), e * inv * inv


def _subframe(LA, LB, mB, j, K, blend_mode, D: Decisions):
    """Float64 sub-frame j along D, with the pieces its gradient needs.
    j = K is L_B; 0 < j < K blends A^ = L_A[winner] and
    B^ = bilinear(L_B, q - (1 - j/K) m_B(q)) with weight alpha = j/K (time
    blend) or 1; where neither exists, lerp(L_A(q), L_B(q), alpha)."""
    if j == K:
        return LB, None
    H, W = LA.shape
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    f = j / K
    alpha = f if blend_mode == o.BLEND_TIME else 1.0
    g = 1.0 - f
    win = D.winner[j - 1]
    vA = win >= 0
    vB = D.vB[j - 1]
    Ah = np.where(vA, LA.ravel()[np.where(vA, win, 0)].reshape(H, W), 0.0)
    sx = xx - g * mB[..., 0]
    sy = yy - g * mB[..., 1]
    x0, y0 = D.cx[j - 1], D.cy[j - 1]
    x1 = np.minimum(x0 + 1, W - 1)
    y1 = np.minimum(y0 + 1, H - 1)
    wx = np.where(vB, sx - x0, 0.0)
    wy = np.where(vB, sy - y0, 0.0)
    a, b = LB[y0, x0], LB[y0, x1]
    c, d = LB[y1, x0], LB[y1, x1]
    top = a + wx * (b - a)
    bot = c + wx * (d - c)
    Bh = top + wy * (bot - top)
    both = vA & vB
    L = np.where(both, Ah + alpha * (Bh - Ah),
                 np.where(vA, Ah, np.where(vB, Bh, LA + alpha * (LB - LA))))
    parts = dict(alpha=alpha, g=g, win=win, vA=vA, vB=vB, both=both, x0=x0, y0=y0, x1=x1, y1=y1,
                 wx=wx, wy=wy, a=a, b=b, c=c, d=d, top=top, bot=bot)
    return L, parts


def subframes64(L_A, L_B, m_B, K, blend_mode, D: Decisions):
    """Float64 sub-frames L_0 = L_A, L_1..L_K along the decisions D."""
    LA = np.asarray(L_A, np.float64)
    LB = np.asarray(L_B, np.float64)
    mB = np.asarray(m_B, np.float64)
    return [LA] + [_subframe(LA, LB, mB, j, K, blend_mode, D)[0] for j in range(1, K + 1)]


def soft_count(L_A, L_B, m_A, m_B, C, R_traj, K, tau, blend_mode, D: Decisions, want_grad=False,
               gS=None, magnitudes=False, frames32=None):
    """Float64 S (and, with want_grad, the gradient of sum(gS * S) with
    respect to L_A, L_B, m_A, m_B and C) along the decisions D.  R_traj is
    (R_0..R_K, dR_0/dC..dR_K/dC) of reference_levels / reference_levels64;
    the sub-frames are those of _subframe.

    frames32 (optional): the float32 oracle's sub-frames L_0..L_K; the
    logistic is then evaluated at those values (the ones a float32
    evaluation along the same decisions sees) instead of the float64
    sub-frames, everything else in float64.

    magnitudes (with want_grad): also return, per gradient element ("L_A",
    "L_B", "m_B", "C") and for S, a bound on the error of a float32
    evaluation of the same sums along the same decisions and sub-frame
    values.  Each term is held to 2^-24 (3 |u| + 64) of its absolute value:
    u = (|L - R| - C) / tau carries about 2^-24 (3 |u| + 10) of absolute
    error from its three roundings (|L - R| = tau |u| + C), which is the
    relative error of exp(-|u|) and so of the logistic and its derivative,
    and 54 more roundings cover the products and sums around it.  The terms
    that go through B's bilinear weights add the weights' error from the
    float32 sample position (s = q - g m_B rounded at |s|:
    2^-23 (|s_x| + |s_y| + 1) per weight), and every element 1e-30 (float32
    underflow of terms below the normal range).  "abs_C" is the plain sum
    of the absolute C terms (for an accumulation whose order is not a short
    tree).  The returned S and gradient are the same either way."""
    LA = np.asarray(L_A, np.float64)
    LB = np.asarray(L_B, np.float64)
    mB = np.asarray(m_B, np.float64)
    H, W = LA.shape
    S = np.zeros((H, W))
    if want_grad:
        gS = np.ones((H, W)) if gS is None else np.asarray(gS, np.float64)
        gLA = np.zeros(H * W)
        gLB = np.zeros(H * W)
        gmB = np.zeros((H, W, 2))
        gC = 0.0
        if magnitudes:
            aLA, aLB, amB = np.zeros(H * W), np.zeros(H * W), np.zeros((H, W, 2))
            pLB, pmB = np.zeros(H * W), np.zeros((H, W, 2))      # position terms
            aC, rC, aS = 0.0, 0.0, np.zeros((H, W))
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    R_list, dRdC_list = R_traj
    for j in range(1, K + 1):
        R = np.asarray(R_list[j - 1], np.float64)
        dRdC = np.asarray(dRdC_list[j - 1], np.float64)
        L, p = _subframe(LA, LB, mB, j, K, blend_mode, D)
        if frames32 is not None:
            L = np.asarray(frames32[j], np.float64)
        dlt = L - R
        u = (np.abs(dlt) - C) / tau
        sg, sg1 = _logistic(u)
        S += sg
        if not want_grad:
            continue
        dS = sg1 / tau
        gL = gS * dS * np.sign(dlt)
        gC += float(np.sum(gS * dS * (-np.sign(dlt) * dRdC - 1.0)))
        if magnitudes:
            rf = 2.0 ** -24 * (3.0 * np.abs(u) + 64.0)      # relative error of one term
            tC = np.abs(gS * dS) * (np.abs(dRdC) + 1.0)
            aC += float(np.sum(tC))
            rC += float(np.sum(tC * rf))
            aS += sg * rf
            aL = np.abs(gL) * rf                              # |gL| held to its error
        if j == K:
            gLB += gL.ravel()
            if magnitudes:
                aLB += aL.ravel()
            continue
        alpha, vA, vB, both, win = p["alpha"], p["vA"], p["vB"], p["both"], p["win"]
        wx, wy = p["wx"], p["wy"]
        cA = np.where(both, 1.0 - alpha, np.where(vA, 1.0, 0.0)) * gL
        cB = np.where(both, alpha, np.where(vA, 0.0, np.where(vB, 1.0, 0.0))) * gL
        hole = ~vA & ~vB
        np.add.at(gLA, win[vA], cA[vA])
        gLA += np.where(hole, (1.0 - alpha) * gL, 0.0).ravel()
        gLB += np.where(hole, alpha * gL, 0.0).ravel()
        corners = ((p["y0"], p["x0"], (1 - wx) * (1 - wy)), (p["y0"], p["x1"], wx * (1 - wy)),
                   (p["y1"], p["x0"], (1 - wx) * wy), (p["y1"], p["x1"], wx * wy))
        for (ty, tx, wgt) in corners:
            np.add.at(gLB, (ty * W + tx)[vB], (cB * wgt)[vB])
        dBdwx = (1 - wy) * (p["b"] - p["a"]) + wy * (p["d"] - p["c"])
        dBdwy = p["bot"] - p["top"]
        gmB[..., 0] += np.where(vB, cB * dBdwx * -p["g"], 0.0)
        gmB[..., 1] += np.where(vB, cB * dBdwy * -p["g"], 0.0)
        if magnitudes:
            kA = np.where(both, 1.0 - alpha, np.where(vA, 1.0, 0.0)) * aL
            kB = np.where(both, alpha, np.where(vA, 0.0, np.where(vB, 1.0, 0.0))) * aL
            np.add.at(aLA, win[vA], kA[vA])
            aLA += np.where(hole, (1.0 - alpha) * aL, 0.0).ravel()
            aLB += np.where(hole, alpha * aL, 0.0).ravel()
            for (ty, tx, wgt) in corners:
                np.add.at(aLB, (ty * W + tx)[vB], (kB * wgt)[vB])
            # the position derivative sums the taps' differences: bound it
            # by the taps themselves
            taps = np.abs(p["a"]) + np.abs(p["b"]) + np.abs(p["c"]) + np.abs(p["d"])
            tapx = (1 - wy) * (np.abs(p["b"]) + np.abs(p["a"])) + wy * (np.abs(p["d"]) + np.abs(p["c"]))
            tapy = np.abs(p["bot"]) + np.abs(p["top"])
            amB[..., 0] += np.where(vB, kB * tapx * p["g"], 0.0)
            amB[..., 1] += np.where(vB, kB * tapy * p["g"], 0.0)
            # weights from the float32 sample position
            dw = 2.0 ** -23 * (np.abs(xx - p["g"] * mB[..., 0]) + np.abs(yy - p["g"] * mB[..., 1]) + 1.0)
            for (ty, tx, _) in corners:
                np.add.at(pLB, (ty * W + tx)[vB], (2.0 * np.abs(cB) * dw)[vB])
            pmB[..., 0] += np.where(vB, np.abs(cB) * dw * taps * p["g"], 0.0)
            pmB[..., 1] += np.where(vB, np.abs(cB) * dw * taps * p["g"], 0.0)
    if not want_grad:
        return S
    grads = dict(L_A=gLA.reshape(H, W), L_B=gLB.reshape(H, W), m_A=np.zeros((H, W, 2)), m_B=gmB, C=gC)
    if magnitudes:
        fl = 1e-30
        return S, grads, dict(L_A=aLA.reshape(H, W) + fl, L_B=aLB.reshape(H, W) + pLB.reshape(H, W) + fl,
                              m_B=amB + pmB + fl, C=rC + fl, S=aS + 2.0 ** -24 * K, abs_C=aC)
    return S, grads


def same_decisions(a: Decisions, b: Decisions) -> np.ndarray:
    """Pixels whose every decision agrees between a and b."""
    H, W = a.winner[0].shape if a.winner else (0, 0)
    ok = np.ones((H, W), bool)
    for j in range(len(a.winner)):
        ok &= (a.winner[j] == b.winner[j]) & (a.vB[j] == b.vB[j])
        ok &= ~a.vB[j] | ((a.cx[j] == b.cx[j]) & (a.cy[j] == b.cy[j]))
    return ok

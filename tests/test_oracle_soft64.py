"""The float64 surrogate oracle: analytic gradient against central finite
differences of the same surrogate, its reference trajectory recomputed at
each evaluation, or held as constants for the stop-gradient reading (CPU
only).  Elements whose +-h step changes a splat winner, a B validity, a
bilinear cell or a crossing count are skipped."""
import numpy as np
import pytest

from oracle import evis_oracle as o
from oracle import soft64 as s64

F32 = np.float32


def make_case(seed, H=12, W=14, K=4):
    rng = np.random.default_rng(seed)
    L_A = rng.normal(0, 1.0, size=(H, W))
    L_B = L_A + rng.normal(0, 0.3, size=(H, W))
    m = rng.normal(0, 1.2, size=(H, W, 2))
    m_B = m + rng.normal(0, 0.2, size=(H, W, 2))
    Z_A = rng.uniform(0.5, 5, size=(H, W))
    Z_B = rng.uniform(0.5, 5, size=(H, W))
    L_ref = L_A + rng.normal(0, 0.15, size=(H, W))
    return dict(L_A=L_A, L_B=L_B, m_A=m, m_B=m_B, Z_A=Z_A, Z_B=Z_B, L_ref=L_ref, K=K)


def evaluate(c, C, tau, mode, held=None):
    """float64 surrogate with its own decisions and its own float64
    reference trajectory (recomputed, so d/dC includes the trajectory), or
    with the reference levels `held` as constants."""
    D = s64.decisions64(c["L_A"], c["L_B"], c["m_A"], c["m_B"], c["Z_A"], c["Z_B"], c["K"])
    fr = s64.subframes64(c["L_A"], c["L_B"], c["m_B"], c["K"], mode, D)
    traj = s64.reference_levels64(fr, c["L_ref"], C)
    if held is not None:
        traj = (held, [np.zeros_like(r) for r in held])
    S = s64.soft_count(c["L_A"], c["L_B"], c["m_A"], c["m_B"], C, traj, c["K"], tau, mode, D)
    return S, D, traj


@pytest.mark.parametrize("hold", [False, True])
@pytest.mark.parametrize("mode", [o.BLEND_TIME, o.BLEND_B_PRIMARY])
@pytest.mark.parametrize("seed", [1, 2])
def test_gradient_matches_finite_differences(seed, mode, hold):
    c = make_case(seed)
    C, tau, h = 0.2, 0.05, 1e-6
    H, W = c["L_A"].shape
    gS = np.random.default_rng(100 + seed).normal(size=(H, W))
    _, D, traj = evaluate(c, C, tau, mode)
    held = traj[0] if hold else None
    if hold:
        traj = (traj[0], [np.zeros_like(r) for r in traj[0]])
    _, g = s64.soft_count(c["L_A"], c["L_B"], c["m_A"], c["m_B"], C, traj, c["K"], tau, mode, D,
                          want_grad=True, gS=gS)
    counts = lambda tr: np.stack(tr[1])
    rng = np.random.default_rng(200 + seed)
    checked = 0
    scale = max(np.abs(g["L_A"]).max(), np.abs(g["L_B"]).max(), np.abs(g["m_B"]).max())
    for name, shape in (("L_A", (H, W)), ("L_B", (H, W)), ("m_A", (H, W, 2)), ("m_B", (H, W, 2))):
        for _ in range(40):
            idx = tuple(rng.integers(0, n) for n in shape)
            cp, cm = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in c.items()}, \
                     {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in c.items()}
            cp[name][idx] += h
            cm[name][idx] -= h
            Sp, Dp, tp = evaluate(cp, C, tau, mode, held)
            Sm, Dm, tm = evaluate(cm, C, tau, mode, held)
            if not (s64.same_decisions(Dp, D).all() and s64.same_decisions(Dm, D).all()):
                continue
            if not (np.array_equal(counts(tp), counts(traj)) and np.array_equal(counts(tm), counts(traj))):
                continue
            fd = (np.sum(gS * Sp) - np.sum(gS * Sm)) / (2 * h)
            an = g[name][idx]
            assert abs(fd - an) <= 1e-5 * scale + 1e-4 * abs(an), (name, idx, fd, an)
            checked += 1
    # C (the reference trajectory moves with C; its counts must not change)
    Sp, _, tp = evaluate(c, C + h, tau, mode, held)
    Sm, _, tm = evaluate(c, C - h, tau, mode, held)
    assert np.array_equal(counts(tp), counts(traj)) and np.array_equal(counts(tm), counts(traj))
    fd = (np.sum(gS * Sp) - np.sum(gS * Sm)) / (2 * h)
    assert abs(fd - g["C"]) <= 1e-5 * max(1.0, abs(g["C"])), (fd, g["C"])
    assert checked > 100
    assert np.all(g["m_A"] == 0)


def test_forward_is_a_smooth_count():
    """With tau -> 0 each term tends to the crossing indicator |dL| > C."""
    c = make_case(3)
    C = 0.2
    pr = o.Pair(c["L_A"].astype(F32), c["L_B"].astype(F32), c["m_A"].astype(F32),
                c["m_B"].astype(F32), c["Z_A"].astype(F32), c["Z_B"].astype(F32))
    fr32, _ = o.interpolate(pr, c["K"], 0, c["K"] + 1)
    R = s64.reference_levels(list(fr32), c["L_ref"].astype(F32), C)
    D = s64.decisions32(o.Pair(c["L_A"].astype(F32), c["L_B"].astype(F32), c["m_A"].astype(F32),
                               c["m_B"].astype(F32), c["Z_A"].astype(F32), c["Z_B"].astype(F32)),
                        c["K"])
    S = s64.soft_count(c["L_A"].astype(F32), c["L_B"].astype(F32), c["m_A"].astype(F32),
                       c["m_B"].astype(F32), C, R, c["K"], 1e-6, o.BLEND_TIME, D)
    pair = o.Pair(c["L_A"].astype(F32), c["L_B"].astype(F32), c["m_A"].astype(F32),
                  c["m_B"].astype(F32), c["Z_A"].astype(F32), c["Z_B"].astype(F32))
    frames, _ = o.interpolate(pair, c["K"], 0, c["K"] + 1)
    hard = np.zeros_like(S)
    for j in range(1, c["K"] + 1):
        hard += np.abs(frames[j].astype(np.float64) - R[0][j - 1]) > C
    assert np.array_equal(np.round(S), hard)

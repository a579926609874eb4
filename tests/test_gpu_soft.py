"""Smooth event-count surrogate on the GPU: forward and backward against
the float64 oracle evaluated along the float32 path's discrete decisions
(splat winners, B validity, gather cells, crossing counts of the reference
trajectory); the backward also against float64 central finite differences
of the surrogate (crossing counts held, like the other decisions); and the fit of
the contrast threshold and a flow correction with Adam.

Bars, per element: 1e-4 relative of the float64 value plus the oracle's
bound on a float32 evaluation of the same sums (a multiple of the sum of
the absolute terms, the float32 sample positions' effect on B's bilinear
weights, and for C the order of its atomic sum); against finite
differences also the difference quotient's own error."""
import numpy as np
import pytest

from oracle import evis_oracle as o
from oracle import soft64 as s64
import gpu_util as U

pytestmark = pytest.mark.gpu
F32 = np.float32


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


@pytest.fixture(scope="module")
def ectx(torch):
    from paper_2607_08098_amd import evis
    c = evis.Context(0)
    yield c
    c.close()


def say(*a):
    print("[case]", *a, flush=True)


def batch(seeds, H, W, flow="translate"):
    pairs = [U.oracle_pair(U.blob_scene(H, W, s, flow=flow, **({"omega": 9.0} if flow == "rotate" else {})))
             for s in seeds]
    rng = np.random.default_rng(seeds[0])
    L_refs = [(p.L_A + rng.normal(0, 0.1, size=p.L_A.shape)).astype(F32) for p in pairs]
    return pairs, L_refs


def to_dev(torch, pairs, L_refs):
    st = lambda xs: torch.from_numpy(np.ascontiguousarray(np.stack(xs))).cuda()
    return dict(L_A=st([p.L_A for p in pairs]), L_B=st([p.L_B for p in pairs]),
                m_A=st([p.m_A for p in pairs]), m_B=st([p.m_B for p in pairs]),
                Z_A=st([p.Z_A for p in pairs]), Z_B=st([p.Z_B for p in pairs]), L_ref=st(L_refs))


def oracle_soft(pair, L_ref, C, K, tau, mode, gS=None, hold_ref=False):
    """Float64 surrogate along the float32 path's decisions and sub-frame
    values: (S, gradients, per-element error bounds of a float32
    evaluation)."""
    frames, _ = o.interpolate(pair, K, 0, K + 1, mode)
    R = s64.reference_levels(list(frames), L_ref, C)
    if hold_ref:   # the trajectory as a constant: no dR/dC term
        R = (R[0], [np.zeros_like(t) for t in R[1]])
    D = s64.decisions32(pair, K)
    return s64.soft_count(pair.L_A, pair.L_B, pair.m_A, pair.m_B, C, R, K, tau, mode, D,
                          want_grad=True, gS=gS, magnitudes=True, frames32=list(frames))


def run_backward(torch, ectx, pairs, L_refs, Cs, K, tau, mode, gS_np, hold_ref):
    from paper_2607_08098_amd import evis
    d = to_dev(torch, pairs, L_refs)
    C = torch.from_numpy(np.asarray(Cs, F32)).cuda()
    S = torch.empty_like(d["L_A"])
    envs = evis.soft_env_array(d["L_A"], d["L_B"], d["m_A"], d["m_B"], d["Z_A"], d["Z_B"], d["L_ref"], S=S)
    evis.evis_soft_count_forward(ectx, envs, K, tau, mode, C)
    gS = torch.from_numpy(gS_np).cuda()
    outs = {k: torch.empty_like(d[k]) for k in ("L_A", "L_B", "m_A", "m_B")}
    gC = torch.empty_like(C)
    envs = evis.soft_env_array(d["L_A"], d["L_B"], d["m_A"], d["m_B"], d["Z_A"], d["Z_B"], d["L_ref"],
                               gS=gS, gL_A=outs["L_A"], gL_B=outs["L_B"], gm_A=outs["m_A"],
                               gm_B=outs["m_B"])
    evis.evis_soft_count_backward(ectx, envs, K, tau, mode, C, gC,
                                  evis.EVIS_SOFT_HOLD_REF if hold_ref else 0)
    torch.cuda.synchronize()
    return (S.cpu().numpy().astype(np.float64), {k: v.cpu().numpy().astype(np.float64) for k, v in outs.items()},
            gC.cpu().numpy().astype(np.float64))


def check_vs_float64(S_gpu, g_gpu, gC_gpu, pairs, L_refs, Cs, K, tau, mode, gS_np, hold_ref, H, W):
    """Every element: |GPU - float64| <= 1e-4 |float64| + the oracle's bound
    on a float32 evaluation (the C sum goes through one atomic per
    workgroup, so its bound is the plain term sum times 2^-24 per add)."""
    items = ((W + 31) // 32) * ((H + 15) // 16)
    for e, (pair, L_ref) in enumerate(zip(pairs, L_refs)):
        S64, g64, bnd = oracle_soft(pair, L_ref, float(Cs[e]), K, tau, mode,
                                    gS=gS_np[e].astype(np.float64), hold_ref=hold_ref)
        err = np.abs(S_gpu[e] - S64)
        assert np.all(err <= 1e-4 * np.abs(S64) + bnd["S"]), ("S", e, float(err.max()))
        for k in ("L_A", "L_B", "m_B"):
            got, want = g_gpu[k][e], g64[k]
            tol = 1e-4 * np.abs(want) + bnd[k]
            bad = np.abs(got - want) > tol
            worst = np.unravel_index(np.argmax(np.abs(got - want) - tol), want.shape)
            assert not bad.any(), (k, e, int(bad.sum()), worst, float(got[worst]), float(want[worst]),
                                   float(tol[worst]))
        assert np.all(g_gpu["m_A"][e] == 0)
        tol_C = 1e-4 * abs(g64["C"]) + bnd["C"] + (items + 256) * 2.0 ** -24 * bnd["abs_C"]
        assert abs(gC_gpu[e] - g64["C"]) <= tol_C, (float(gC_gpu[e]), g64["C"], tol_C)


@pytest.mark.parametrize("hold_ref", [False, True])
@pytest.mark.parametrize("mode", [o.BLEND_TIME, o.BLEND_B_PRIMARY])
def test_soft_forward_backward_vs_float64(torch, ectx, mode, hold_ref):
    K, tau, H, W = 8, 0.02, 48, 64
    pairs, L_refs = batch([501, 502], H, W, flow="rotate")
    Cs = np.array([0.2, 0.25], F32)
    gS_np = np.random.default_rng(7).normal(size=(2, H, W)).astype(F32)
    say("soft forward/backward", mode, "hold_ref" if hold_ref else "")
    S, g, gC = run_backward(torch, ectx, pairs, L_refs, Cs, K, tau, mode, gS_np, hold_ref)
    check_vs_float64(S, g, gC, pairs, L_refs, Cs, K, tau, mode, gS_np, hold_ref, H, W)


def test_soft_forward_backward_vs_float64_full_size(torch, ectx):
    """The differentiation workload's shape: 640x480 frames of the
    translating blob scene, K = 16, tau = 0.02, every element."""
    K, tau, H, W = 16, 0.02, 480, 640
    pairs, L_refs = batch([5000, 5001], H, W)
    Cs = np.array([0.25, 0.18], F32)
    gS_np = np.random.default_rng(8).normal(size=(2, H, W)).astype(F32)
    say("soft forward/backward 2 x 640x480, K 16")
    S, g, gC = run_backward(torch, ectx, pairs, L_refs, Cs, K, tau, o.BLEND_TIME, gS_np, False)
    check_vs_float64(S, g, gC, pairs, L_refs, Cs, K, tau, o.BLEND_TIME, gS_np, False, H, W)


def fd_check(torch, ectx, seed, H, W, K, tau, hold_ref, crop, n_samples, flow="rotate"):
    """GPU gradient against float64 central differences at sampled
    elements.  The function differentiated is the surrogate along the
    float32 path's sub-frame values, moved by the float64 change of the
    sub-frames under the perturbation (and the reference levels by C times
    the held counts): S(L32_j + L64_j(v) - L64_j(v0), R32 + (C - C0) dR/dC),
    the function the backward kernel differentiates.  Elements whose splat
    or gather decisions change under +-h are skipped.  With crop, each
    element's differences are taken on the window of +-crop px around it
    (the perturbation moves only sub-frame pixels within the motion, a few
    px for the translating scene, of it).  Bar: 1e-4 |fd|
    plus the oracle's float32 bound plus the difference quotient's own
    error: float64 rounding of the loss over 2h, and h^2 / 6 times the
    third derivative (that of the logistic is at most 1 / (8 tau^3) per
    substep)."""
    C0, h = 0.2, 1e-6
    pairs, L_refs = batch([seed], H, W, flow=flow)
    pair, L_ref = pairs[0], L_refs[0]
    gS_np = np.random.default_rng(seed).normal(size=(1, H, W)).astype(F32)
    say("soft backward for finite differences", H, W, "K", K, "hold_ref" if hold_ref else "")
    _, got, gC = run_backward(torch, ectx, pairs, L_refs, [C0], K, tau, o.BLEND_TIME, gS_np, hold_ref)
    frames, _ = o.interpolate(pair, K, 0, K + 1)
    R32, counts32 = s64.reference_levels(list(frames), L_ref, C0)
    traj = (R32, [np.zeros_like(c) for c in counts32]) if hold_ref else (R32, counts32)
    _, _, bnd = s64.soft_count(pair.L_A, pair.L_B, pair.m_A, pair.m_B, C0, traj, K, tau,
                               o.BLEND_TIME, s64.decisions32(pair, K), want_grad=True,
                               gS=gS_np[0].astype(np.float64), magnitudes=True, frames32=list(frames))
    F64 = [np.asarray(f, np.float64) for f in frames]
    R64 = [np.asarray(r, np.float64) for r in R32]
    dR = [np.asarray(c, np.float64) for c in traj[1]]
    g = gS_np[0].astype(np.float64)
    base = {k: getattr(pair, k).astype(np.float64) for k in ("L_A", "L_B", "m_A", "m_B", "Z_A", "Z_B")}

    def loss_of(L_list, Cv, sl):
        tot = 0.0
        for j in range(1, K + 1):
            Rj = R64[j - 1][sl] + (Cv - C0) * dR[j - 1][sl]
            u = (np.abs(L_list[j] - Rj) - Cv) / tau
            tot += float(np.sum(g[sl] / (1.0 + np.exp(-u))))
        return tot

    def window(idx):
        if crop is None:
            return (slice(0, H), slice(0, W))
        y, x = idx[0], idx[1]
        return (slice(max(0, y - crop), min(H, y + crop + 1)), slice(max(0, x - crop), min(W, x + crop + 1)))

    def moved(v, sl):
        """Sub-frames on the window, L32 + (L64(v) - L64(v0)), and the decisions."""
        c = {k: v[k][sl] for k in v}
        c0 = {k: base[k][sl] for k in base}
        D = s64.decisions64(c["L_A"], c["L_B"], c["m_A"], c["m_B"], c["Z_A"], c["Z_B"], K)
        D0 = s64.decisions64(c0["L_A"], c0["L_B"], c0["m_A"], c0["m_B"], c0["Z_A"], c0["Z_B"], K)
        L1 = s64.subframes64(c["L_A"], c["L_B"], c["m_B"], K, o.BLEND_TIME, D0)
        L0 = s64.subframes64(c0["L_A"], c0["L_B"], c0["m_B"], K, o.BLEND_TIME, D0)
        return [F64[j][sl] + (L1[j] - L0[j]) for j in range(K + 1)], D, D0

    rng = np.random.default_rng(seed + 1)
    checked = 0
    for name in ("L_A", "L_B", "m_B"):
        got_all = got[name][0]
        for _ in range(n_samples):
            idx = tuple(int(rng.integers(0, n)) for n in base[name].shape)
            sl = window(idx)
            vp = {k: v.copy() for k, v in base.items()}
            vm = {k: v.copy() for k, v in base.items()}
            vp[name][idx] += h
            vm[name][idx] -= h
            Lp, Dp, D0 = moved(vp, sl)
            Lm, Dm, _ = moved(vm, sl)
            if not (s64.same_decisions(Dp, D0).all() and s64.same_decisions(Dm, D0).all()):
                continue
            fd = (loss_of(Lp, C0, sl) - loss_of(Lm, C0, sl)) / (2 * h)
            scale = float(np.sum(np.abs(g[sl]))) * K
            fd_err = 4 * 2.0 ** -53 * scale / (2 * h) + h * h / 6 * K * np.abs(g).max() / (8 * tau ** 3)
            tol = 1e-4 * abs(fd) + float(np.asarray(bnd[name])[idx]) + fd_err
            assert abs(got_all[idx] - fd) <= tol, (name, idx, got_all[idx], fd, tol)
            checked += 1
    full = (slice(0, H), slice(0, W))
    fd = (loss_of(F64, C0 + h, full) - loss_of(F64, C0 - h, full)) / (2 * h)
    fd_err = 4 * 2.0 ** -53 * float(np.sum(np.abs(g))) * K / (2 * h)
    items = ((W + 31) // 32) * ((H + 15) // 16)
    tol_C = 1e-4 * abs(fd) + bnd["C"] + (items + 256) * 2.0 ** -24 * bnd["abs_C"] + fd_err
    assert abs(float(gC[0]) - fd) <= tol_C, (float(gC[0]), fd, tol_C)
    return checked


@pytest.mark.parametrize("hold_ref", [False, True])
def test_soft_backward_vs_finite_differences(torch, ectx, hold_ref):
    checked = fd_check(torch, ectx, 601, 24, 32, 8, 0.02, hold_ref, None, 40)
    assert checked > 60


def test_soft_backward_vs_finite_differences_full_size(torch, ectx):
    """The differentiation workload's shape (640x480 translating blob scene,
    K = 16, tau = 0.02): differences on +-24 px windows."""
    checked = fd_check(torch, ectx, 602, 480, 640, 16, 0.02, False, 24, 20, flow="translate")
    assert checked > 30


def multiscale_loss(torch, S, T):
    """Squared error of S against T at 1x1, 4x4 and 16x16 pixel pooling.
    The per-pixel term alone plateaus a few hundredths away from the true
    threshold (the reference trajectories then share few crossings); the
    pooled counts fall monotonically in C and keep a wide basin."""
    F = torch.nn.functional
    loss = ((S - T) ** 2).mean()
    for k in (4, 16):
        loss = loss + ((F.avg_pool2d(S[:, None], k) - F.avg_pool2d(T[:, None], k)) ** 2).mean()
    return loss


def fit(torch, ectx, n_env, H, W, steps, K=16, tau=0.02, lr_c=1e-2, lr_delta=3e-2, lr_end=0.05):
    from paper_2607_08098_amd.autograd import soft_count
    pairs, L_refs = batch(list(range(5000, 5000 + n_env)), H, W)
    d = to_dev(torch, pairs, L_refs)
    delta_true = torch.tensor([-0.3, 0.0], device="cuda")
    C_true = torch.full((n_env,), 0.18, device="cuda")
    with torch.no_grad():
        target = soft_count(d["L_A"], d["L_B"], d["m_A"] + delta_true, d["m_B"] + delta_true, C_true,
                            d["Z_A"], d["Z_B"], d["L_ref"], K, tau, o.BLEND_TIME, ectx)
    C = torch.full((n_env,), 0.25, device="cuda", requires_grad=True)
    delta = torch.zeros(2, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([{"params": [C], "lr": lr_c}, {"params": [delta], "lr": lr_delta}])
    # learning rates fall linearly to lr_end of their start: without it Adam
    # keeps stepping at full size once the small case's loss is near zero
    sched = torch.optim.lr_scheduler.LambdaLR(opt, lambda i: 1.0 - (1.0 - lr_end) * i / steps)
    first = None
    for it in range(steps):
        opt.zero_grad()
        S = soft_count(d["L_A"], d["L_B"], d["m_A"] + delta, d["m_B"] + delta, C, d["Z_A"], d["Z_B"],
                       d["L_ref"], K, tau, o.BLEND_TIME, ectx)
        loss = multiscale_loss(torch, S, target)
        if first is None:
            first = loss.item()
        loss.backward()
        opt.step()
        sched.step()
        with torch.no_grad():
            C.clamp_(min=0.02)
    return C.detach().cpu().numpy(), delta.detach().cpu().numpy(), loss.item(), first


def check_fit(C, delta, loss, first):
    # plausibility, not parity: C recovered, the flow correction moves
    # towards the injected bias, the loss falls
    assert np.all(np.abs(C - 0.18) < 0.01), C
    assert -0.45 < delta[0] < -0.1 and abs(delta[1]) < 0.1, delta
    assert loss < 0.25 * first, (loss, first)


def test_fit_threshold_and_flow_small(torch, ectx):
    say("Adam fit, 2 envs 96x128, 600 steps")
    C, delta, loss, first = fit(torch, ectx, 2, 96, 128, 600)
    print("fit:", C, delta, loss, first, flush=True)
    check_fit(C, delta, loss, first)


def test_fit_threshold_and_flow_full_size(torch, ectx):
    """8 envs at 640x480, K = 16, tau = 0.02, 600 Adam steps."""
    say("Adam fit, 8 envs 640x480, 600 steps")
    C, delta, loss, first = fit(torch, ectx, 8, 480, 640, 600)
    print("fit:", C, delta, loss, first, flush=True)
    check_fit(C, delta, loss, first)

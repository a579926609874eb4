"""Over-render crop margin and colour events through the C ABI against the
CPU oracle: events bit-exact as multisets, inner states bit-exact, margin
states untouched; per-channel log intensity within 4e-6 absolute (the
same bar as the luminance's log)."""
import dataclasses

import numpy as np
import pytest

from oracle import evis_oracle as o
import gpu_util as U

pytestmark = pytest.mark.gpu
F32 = np.float32


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_2607_08098_amd import evis
    c = evis.Context(0)
    yield c
    c.close()


def say(*a):
    print("[case]", *a, flush=True)


def run_step(torch, ctx, pairs, sensors, L_refs, t_lasts, env_ids, margins, capacity=8 << 20):
    from paper_2607_08098_amd import evis
    envs = []
    for pair, s, L_ref, tl, eid, m in zip(pairs, sensors, L_refs, t_lasts, env_ids, margins):
        d = U.device_pair(pair, torch)
        d.update(C_on=s.C_on, C_off=s.C_off, refractory_us=s.refractory_us, K=s.K,
                 K_max=s.K_max, blend_mode=s.blend_mode, env_id=eid, crop_margin=m)
        if s.theta_on is not None:
            d["theta_on"] = torch.from_numpy(s.theta_on).cuda()
            d["theta_off"] = torch.from_numpy(s.theta_off).cuda()
        if s.noise is not None:
            d["noise"] = dataclasses.asdict(s.noise)
        d["L_ref"] = torch.from_numpy(L_ref.copy()).cuda()
        d["t_last"] = None if tl is None else torch.from_numpy(tl.copy()).cuda()
        envs.append(d)
    out, n = evis.event_buffer(capacity)
    evis.evis_step_batch(ctx, envs, out, n, None)
    torch.cuda.synchronize()
    return (evis.decode_events(out, n), int(n.item()), [d["L_ref"].cpu().numpy() for d in envs],
            [None if d["t_last"] is None else d["t_last"].cpu().numpy() for d in envs])


def check(got, pairs, sensors, L_refs, t_lasts, env_ids, margins):
    ev, n, Rs, tls = got
    wevs = []
    for pair, s, L_ref, tl, eid, m, R, gtl in zip(pairs, sensors, L_refs, t_lasts, env_ids, margins,
                                                  Rs, tls):
        wev, wR, wtl, _ = o.step(pair, s, L_ref, tl, eid, crop_margin=m)
        wevs.append(wev)
        assert np.array_equal(R.view(np.uint32), wR.view(np.uint32)), eid
        if wtl is not None:
            assert np.array_equal(gtl, wtl), eid
    want = np.concatenate(wevs)
    assert n == len(want), (n, len(want))
    assert U.same_multiset(ev, want), U.multiset_diff(ev, want)
    return n


@pytest.mark.parametrize("margin", [1, 3, 17])
def test_step_crop_margin(torch, ctx, margin):
    pair = U.oracle_pair(U.blob_scene(90, 120, 31, flow="rotate", omega=12.0))
    s = o.Sensor(C_on=0.2, C_off=0.2, K=0, K_max=64)
    tl = np.full(pair.shape, o.T_LAST_INIT, np.int32)
    s2 = dataclasses.replace(s, refractory_us=50)
    args = ([pair, pair], [s, s2], [pair.L_A.copy(), pair.L_A.copy()], [None, tl], [3, 4],
            [margin, margin])
    say("step_batch crop margin", margin)
    n = check(run_step(torch, ctx, *args), *args)
    assert n > 1000


def test_step_crop_margin_with_noise_and_splat(torch, ctx):
    """Margins of different widths in one launch, with sensor noise (drawn
    at the cropped coordinates) and the two-splat warp."""
    pairs, sensors, Ls, tls, ids, ms = [], [], [], [], [], []
    for i, (H, W, m) in enumerate(((64, 80, 0), (70, 55, 5), (40, 96, 12))):
        pair = U.oracle_pair(U.blob_scene(H, W, 500 + i, flow="rotate", omega=8.0 + 3 * i))
        nz = o.Noise(leak_rate_hz=50.0, shot_rate_hz=80.0, hot_rate_hz=500.0, hot_fraction=0.03,
                     shot_L0=-4.0, shot_inv_range=0.1, seed=31 + i, pair_index=i)
        pairs.append(pair)
        sensors.append(o.Sensor(C_on=0.2, C_off=0.2, K=0, K_max=64, blend_mode=o.WARP_SPLAT,
                                noise=nz))
        Ls.append(pair.L_A.copy())
        tls.append(None)
        ids.append(10 + i)
        ms.append(m)
    args = (pairs, sensors, Ls, tls, ids, ms)
    say("step_batch crop margins with noise, splat warp")
    check(run_step(torch, ctx, *args), *args)


def test_colour_events(torch, ctx):
    """Colour events: per-channel log on the device, then one env per
    channel (shared motion and depth) in one fused launch."""
    from paper_2607_08098_amd import evis, scenes
    H, W = 72, 96
    sc = scenes.blob_pair(H, W, 77, flow="rotate", omega=10.0)
    rng = np.random.default_rng(78)
    tint = rng.uniform(0.3, 1.5, size=3)
    rgb_A = (sc["I_A"][..., None] * tint).astype(F32)
    rgb_B = (sc["I_B"][..., None] * tint[::-1]).astype(F32)
    say("log_channels", rgb_A.shape)
    got = evis.evis_log_channels(ctx, torch.from_numpy(rgb_A).cuda()).cpu().numpy()
    want = o.log_channels(rgb_A.astype(np.float64))
    assert got.shape == (3, H, W) and np.abs(got - want).max() <= 4e-6
    LA = o.log_channels(rgb_A).astype(F32)
    LB = o.log_channels(rgb_B).astype(F32)
    pairs = [o.Pair(LA[c], LB[c], sc["m_A"], sc["m_B"], sc["Z_A"], sc["Z_B"], 0, 16667)
             for c in range(3)]
    s = o.Sensor(C_on=0.25, C_off=0.25, K=0, K_max=64)
    args = (pairs, [s] * 3, [p.L_A.copy() for p in pairs], [None] * 3, [0, 1, 2], [0, 0, 0])
    say("step_batch colour events")
    ev, n, _, _ = got_step = run_step(torch, ctx, *args)
    check(got_step, *args)
    per = np.bincount(ev[:, 4], minlength=3)
    assert np.all(per[:3] > 100)


def test_crop_margin_errors(torch, ctx):
    from paper_2607_08098_amd import evis
    pair = U.oracle_pair(U.blob_scene(20, 30, 3))
    out, n = evis.event_buffer(1024)
    for m in (-1, 10, 15):
        d = U.device_pair(pair, torch)
        d.update(C_on=0.2, C_off=0.2, refractory_us=0, K=4, K_max=64, blend_mode=0, env_id=0,
                 crop_margin=m)
        d["L_ref"] = torch.from_numpy(pair.L_A.copy()).cuda()
        d["t_last"] = None
        with pytest.raises(evis.EvisError) as ei:
            evis.evis_step_batch(ctx, [d], out, n, None)
        assert ei.value.code == evis.EVIS_ERR_INVALID and "crop_margin" in str(ei.value), m

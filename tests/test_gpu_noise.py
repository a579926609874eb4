"""Sensor-noise events (leak, shot noise, hot pixels from Philox4x32-10) of
the fused step through the C ABI against the CPU oracle on the same seeded
inputs: events bit-exact as multisets (crossings and noise together),
states bit-exact."""
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


def run_step(torch, ctx, pairs, sensors, L_refs, t_lasts, env_ids, capacity=8 * 1024 * 1024):
    from paper_2607_08098_amd import evis
    envs = []
    for pair, s, L_ref, tl, eid in zip(pairs, sensors, L_refs, t_lasts, env_ids):
        d = U.device_pair(pair, torch)
        d.update(C_on=s.C_on, C_off=s.C_off, refractory_us=s.refractory_us, K=s.K,
                 K_max=s.K_max, blend_mode=s.blend_mode, env_id=eid)
        if s.theta_on is not None:
            d["theta_on"] = torch.from_numpy(s.theta_on).cuda()
            d["theta_off"] = torch.from_numpy(s.theta_off).cuda()
        if s.noise is not None:
            d["noise"] = dataclasses.asdict(s.noise)
        d["L_ref"] = torch.from_numpy(L_ref.copy()).cuda()
        d["t_last"] = None if tl is None else torch.from_numpy(tl.copy()).cuda()
        envs.append(d)
    out, n = evis.event_buffer(capacity)
    K_used = torch.zeros(len(envs), dtype=torch.int32, device="cuda")
    evis.evis_step_batch(ctx, envs, out, n, K_used)
    torch.cuda.synchronize()
    ev = evis.decode_events(out, n)
    return (ev, int(n.item()), [d["L_ref"].cpu().numpy() for d in envs],
            [None if d["t_last"] is None else d["t_last"].cpu().numpy() for d in envs],
            K_used.cpu().numpy())


def oracle_steps(pairs, sensors, L_refs, t_lasts, env_ids):
    evs, Rs, tls, Ks = [], [], [], []
    for pair, s, L_ref, tl, eid in zip(pairs, sensors, L_refs, t_lasts, env_ids):
        ev, R, tl2, K = o.step(pair, s, L_ref, tl, eid)
        evs.append(ev)
        Rs.append(R)
        tls.append(tl2)
        Ks.append(K)
    return np.concatenate(evs) if evs else np.zeros((0, 5), np.int64), Rs, tls, Ks


def check_step(got, want):
    ev, n, Rs, tls, Ks = got
    wev, wRs, wtls, wKs = want
    assert list(Ks) == list(wKs), (list(Ks), wKs)
    assert n == len(wev), (n, len(wev))
    assert U.same_multiset(ev, wev), U.multiset_diff(ev, wev)
    for a, b in zip(Rs, wRs):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    for a, b in zip(tls, wtls):
        if b is not None:
            assert np.array_equal(a, b)


def noise(seed, pair_index=0, scale=1.0):
    return o.Noise(leak_rate_hz=30.0 * scale, shot_rate_hz=60.0 * scale, hot_rate_hz=400.0 * scale,
                   hot_fraction=0.02, shot_L0=-4.0, shot_inv_range=1.0 / 10.0, seed=seed,
                   pair_index=pair_index)


@pytest.mark.parametrize("warp", [o.WARP_GATHER, o.WARP_SPLAT, o.WARP_JOINT])
def test_step_noise(torch, ctx, warp):
    pair = U.oracle_pair(U.blob_scene(128, 128, 1000, flow="rotate", omega=9.0))
    s = o.Sensor(C_on=0.2, C_off=0.2, K=8, blend_mode=warp, noise=noise(0xDEADBEEF12345678, 4))
    args = ([pair], [s], [pair.L_A.copy()], [None], [0])
    want = oracle_steps(*args)
    plain = o.step(pair, dataclasses.replace(s, noise=None), pair.L_A.copy())[0]
    assert len(want[0]) > len(plain) + 100          # the noise is there
    say("step_batch with noise 128x128 K=8 warp", hex(warp))
    check_step(run_step(torch, ctx, *args), want)


def test_step_noise_mixed_batch(torch, ctx):
    """Envs with and without noise, different seeds and pair indices,
    mismatch and refractory, adaptive K, ragged sizes, in one launch."""
    from paper_2607_08098_amd import scenes
    specs = [(40, 56, "rotate", 5.0), (64, 48, "translate", None), (33, 71, "rotate", 19.0),
             (17, 9, "rotate", 2.0), (90, 64, "rotate", 11.0)]
    pairs, sensors, L_refs, tls, ids = [], [], [], [], []
    for i, (H, W, flow, om) in enumerate(specs):
        kw = dict(flow=flow, omega=om) if flow == "rotate" else dict(flow=flow)
        pair = U.oracle_pair(U.blob_scene(H, W, 400 + i, **kw), t0=5000 * i, t1=5000 * i + 16667)
        nz = None if i == 2 else noise(1000 + 17 * i, pair_index=i)
        if i % 2 == 0:
            s = o.Sensor(C_on=0.2, C_off=0.2, K=0, K_max=64, noise=nz)
            tl = None
        else:
            on, off = scenes.mismatch_thresholds(H, W, 0.25, 0.03, 0.01, scenes.rng_for(60 + i))
            s = o.Sensor(theta_on=on, theta_off=off, refractory_us=100, K=0, K_max=64, noise=nz)
            tl = np.full((H, W), o.T_LAST_INIT, np.int32)
        pairs.append(pair)
        sensors.append(s)
        L_refs.append(pair.L_A.copy())
        tls.append(tl)
        ids.append(5 * i + 2)
    args = (pairs, sensors, L_refs, tls, ids)
    want = oracle_steps(*args)
    say("step_batch noise mixed 5 envs")
    check_step(run_step(torch, ctx, *args), want)


def test_step_heavy_noise_overflows_the_stage(torch, ctx):
    """Rates near one event per pixel-substep: the workgroup's event buffer
    overflows every substep, so waves write straight to the stream."""
    pair = U.oracle_pair(U.blob_scene(96, 112, 2024, flow="translate"))
    nz = o.Noise(leak_rate_hz=4000.0, shot_rate_hz=6000.0, hot_rate_hz=8000.0, hot_fraction=0.5,
                 shot_L0=-4.0, shot_inv_range=0.1, seed=77, pair_index=9)
    s = o.Sensor(C_on=0.2, C_off=0.2, K=6, noise=nz)
    args = ([pair], [s], [pair.L_A.copy()], [None], [1])
    want = oracle_steps(*args)
    assert len(want[0]) > 96 * 112 * 6 // 2
    say("step_batch heavy noise")
    check_step(run_step(torch, ctx, *args), want)


def test_noise_argument_errors(torch, ctx):
    from paper_2607_08098_amd import evis
    pair = U.oracle_pair(U.blob_scene(20, 24, 3))
    out, n = evis.event_buffer(1024)
    for bad in (dict(leak_rate_hz=-1.0), dict(hot_fraction=1.5), dict(shot_rate_hz=float("inf")),
                dict(shot_inv_range=float("nan"))):
        d = U.device_pair(pair, torch)
        d.update(C_on=0.2, C_off=0.2, refractory_us=0, K=4, K_max=64, blend_mode=0, env_id=0,
                 noise=bad)
        d["L_ref"] = torch.from_numpy(pair.L_A.copy()).cuda()
        d["t_last"] = None
        with pytest.raises(evis.EvisError) as ei:
            evis.evis_step_batch(ctx, [d], out, n, None)
        assert ei.value.code == evis.EVIS_ERR_INVALID and "noise" in str(ei.value), bad
    torch.cuda.synchronize()
    assert int(n.item()) == 0


@pytest.mark.parametrize("shape,K,scale", [((64, 80), 5, 1.0), ((600, 500), 3, 0.1),
                                           ((1100, 1000), 2, 0.01)])
def test_generate_events_noise(torch, ctx, shape, K, scale):
    """The event model over caller-supplied frames with sensor noise (every
    pixels-per-thread variant of the kernel), mismatch and refractory."""
    from paper_2607_08098_amd import evis, scenes
    H, W = shape
    pair = U.oracle_pair(U.blob_scene(H, W, 700 + H, flow="rotate", omega=6.0))
    frames, _ = o.interpolate(pair, K, 0, K + 1)
    on, off = scenes.mismatch_thresholds(H, W, 0.25, 0.03, 0.01, scenes.rng_for(77))
    nz = noise(4242 + H, pair_index=7, scale=scale)
    s = o.Sensor(theta_on=on, theta_off=off, refractory_us=80, K=K, noise=nz)
    tl = np.full((H, W), o.T_LAST_INIT, np.int32)
    want, R, wtl = o.emit_events(list(frames), 1000, 17667, s, pair.L_A.copy(), tl.copy(), env_id=9)
    Ls = torch.from_numpy(np.ascontiguousarray(frames)).cuda()
    sensor = dict(C_on=0.2, C_off=0.2, theta_on=torch.from_numpy(on).cuda(),
                  theta_off=torch.from_numpy(off).cuda(), refractory_us=80)
    state = dict(L_ref=torch.from_numpy(pair.L_A.copy()).cuda(), t_last=torch.from_numpy(tl).cuda())
    out, n = evis.event_buffer(1 << 23)
    say("generate_events with noise", shape, "K", K)
    evis.evis_generate_events(ctx, Ls, 1000, 17667, sensor, state, 9, out, n,
                              noise=dataclasses.asdict(nz))
    torch.cuda.synchronize()
    ev = evis.decode_events(out, n)
    assert int(n.item()) == len(want)
    assert U.same_multiset(ev, want), U.multiset_diff(ev, want)
    assert np.array_equal(state["L_ref"].cpu().numpy().view(np.uint32), R.view(np.uint32))
    assert np.array_equal(state["t_last"].cpu().numpy(), wtl)

"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (autotuned tile, one persistent graph-replayed launch):

* the 64-env mixed batch (24 x 346x260, 24 x 640x480, 16 x 1280x720,
  rotating blob scenes, adaptive K <= 64): every event and the reference
  levels of sampled envs against the oracle fed the same (device-computed)
  log frames;
* 512 rotating-disc envs at 346x260 (adaptive K <= 128, static background
  on the static-tile path), sustained for 200 steps with the state carried
  on the device: sampled envs at sampled steps against the oracle started
  from the device state of that step; stream size and capacity checks on
  every step;
* the benchmark's variants on the same batch (two-splat warps, sensor
  noise): sampled envs against the oracle;
* a textured-plane scene at 640x480 seen by a random-walk camera (exact
  flow and depth, true occlusion), per-pixel threshold mismatch and a 100 us
  refractory period, three keyframe pairs chained through the state: every
  event, reference level and last-event time against the oracle chained
  the same way.
"""
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


def host(t):
    return t.detach().cpu().numpy().copy()


def env_events(ev, e, t0=None, t1=None):
    sel = ev[:, 4] == e
    if t0 is not None:
        sel &= (ev[:, 2] >= t0) & (ev[:, 2] <= t1)
    return ev[sel]


def test_mixed64_full_size_sampled_parity(torch, ctx):
    from paper_2607_08098_amd import evis, scenes, workloads
    say("mixed64 full size: build workload")
    batch = workloads.mixed_batch(ctx, specs=scenes.mixed_batch_specs(3000))
    sensor = dict(C_on=0.2, C_off=0.2, K=0, K_max=64, refractory_us=0)
    envs = batch.env_dicts(sensor)
    arr = evis.env_array(envs)
    out, n = evis.event_buffer(1 << 28)
    say("mixed64 full size: autotune")
    best, _ = evis.evis_autotune(ctx, arr, out, n, reps=2)
    evis.evis_set_tuning(ctx, **best.as_dict())
    samples = [0, 24, 48]
    snap = {e: {k: host(v) for k, v in envs[e].items() if hasattr(v, "cpu")} for e in samples}
    K_used = torch.zeros(len(envs), dtype=torch.int32, device="cuda")
    say("mixed64 full size: step, tile", best.tile_w, best.tile_h)
    n.zero_()
    evis.evis_step_batch(ctx, arr, out, n, K_used, 0)
    torch.cuda.synchronize()
    total = int(n.item())
    assert 0 < total <= out.shape[0]
    ev = evis.decode_events(out, n)
    assert np.all(np.bincount(ev[:, 4], minlength=64) > 0)   # every env fired
    Ks = host(K_used)
    for e in samples:
        s = snap[e]
        say("mixed64 oracle env", e, s["L_A"].shape, "K", int(Ks[e]))
        pair = o.Pair(s["L_A"], s["L_B"], s["m_A"], s["m_B"], s["Z_A"], s["Z_B"], 0, 16667)
        want, R, _, K = o.step(pair, o.Sensor(C_on=0.2, C_off=0.2, K=0, K_max=64), s["L_ref"], None, e)
        assert K == Ks[e]
        got = env_events(ev, e)
        assert U.same_multiset(got, want), (e, len(got), len(want), U.multiset_diff(got, want))
        assert np.array_equal(host(envs[e]["L_ref"]).view(np.uint32), R.view(np.uint32))


@pytest.mark.parametrize("variant", ["splat_b_primary", "joint", "gather_with_noise"])
def test_mixed64_variants_sampled_parity(torch, ctx, variant):
    """The benchmark's variants at full size in its launch configuration
    (same batch, the tile shape it autotunes for the gather warp): every
    event and reference level of sampled envs against the oracle."""
    from paper_2607_08098_amd import evis, scenes, workloads
    say("mixed64 variant", variant, ": build workload")
    batch = workloads.mixed_batch(ctx, specs=scenes.mixed_batch_specs(3000))
    mode = {"splat_b_primary": o.WARP_SPLAT | o.BLEND_B_PRIMARY, "joint": o.WARP_JOINT,
            "gather_with_noise": o.WARP_GATHER}[variant]
    sensor = dict(C_on=0.2, C_off=0.2, K=0, K_max=64, refractory_us=0, blend_mode=mode)
    envs = batch.env_dicts(sensor)
    noise = None
    if variant == "gather_with_noise":
        noise = dict(leak_rate_hz=0.1, shot_rate_hz=1.0, hot_rate_hz=100.0, hot_fraction=1e-3,
                     shot_L0=-7.0, shot_inv_range=0.1)
        for e, d in enumerate(envs):
            d["noise"] = dict(noise, seed=9000 + e)
    arr = evis.env_array(envs)
    out, n = evis.event_buffer(1 << 28)
    evis.evis_set_tuning(ctx, tile_w=32, tile_h=16)
    samples = [0, 24] if variant == "splat_b_primary" else [0]
    snap = {e: {k: host(v) for k, v in envs[e].items() if hasattr(v, "cpu")} for e in samples}
    K_used = torch.zeros(len(envs), dtype=torch.int32, device="cuda")
    say("mixed64 variant", variant, ": step")
    n.zero_()
    evis.evis_step_batch(ctx, arr, out, n, K_used, 0)
    torch.cuda.synchronize()
    assert 0 < int(n.item()) <= out.shape[0]
    ev = evis.decode_events(out, n)
    Ks = host(K_used)
    for e in samples:
        s = snap[e]
        say("mixed64 variant", variant, "oracle env", e, s["L_A"].shape, "K", int(Ks[e]))
        pair = o.Pair(s["L_A"], s["L_B"], s["m_A"], s["m_B"], s["Z_A"], s["Z_B"], 0, 16667)
        nz = o.Noise(seed=9000 + e, **noise) if noise else None
        sen = o.Sensor(C_on=0.2, C_off=0.2, K=0, K_max=64, blend_mode=mode, noise=nz)
        want, R, _, K = o.step(pair, sen, s["L_ref"], None, e)
        assert K == Ks[e]
        got = env_events(ev, e)
        assert U.same_multiset(got, want), (e, len(got), len(want), U.multiset_diff(got, want))
        assert np.array_equal(host(envs[e]["L_ref"]).view(np.uint32), R.view(np.uint32))


def test_disc512_sustained_sampled_parity(torch, ctx):
    from paper_2607_08098_amd import evis, workloads
    say("disc512: build workload")
    batch = workloads.DiscBatch(ctx, n_envs=512, H=260, W=346, seed_base=4000)
    batch.start(0)
    sensor = dict(C_on=0.2, C_off=0.2, K=0, K_max=128, refractory_us=0)
    out, n = evis.event_buffer(1 << 26)
    K_used = torch.zeros(512, dtype=torch.int32, device="cuda")
    evis.evis_set_tuning(ctx, tile_w=32, tile_h=16)
    check_at = {0: [0, 257], 100: [13, 400], 199: [511, 77]}
    counts = []
    for step in range(200):
        if step > 0:
            batch.advance()
        t0, t1 = batch.times()
        envs = batch.env_dicts(sensor, t0, t1)
        arr = evis.env_array(envs)
        snap = None
        if step in check_at:
            torch.cuda.synchronize()
            snap = {e: {k: host(v) for k, v in envs[e].items() if hasattr(v, "cpu")} for e in check_at[step]}
        evis.evis_step_batch(ctx, arr, out, n, K_used, evis.EVIS_FLAG_RESET_CURSOR)
        if snap is None:
            if step % 50 == 0:
                torch.cuda.synchronize()
                say("disc512 step", step, "events", int(n.item()))
            continue
        torch.cuda.synchronize()
        total = int(n.item())
        counts.append(total)
        assert 0 < total <= out.shape[0], total
        ev = evis.decode_events(out, n)
        Ks = host(K_used)
        assert Ks.max() <= 128
        for e, s in snap.items():
            say("disc512 oracle step", step, "env", e, "K", int(Ks[e]))
            pair = o.Pair(s["L_A"], s["L_B"], s["m_A"], s["m_B"], s["Z_A"], s["Z_B"], t0, t1)
            want, R, _, K = o.step(pair, o.Sensor(C_on=0.2, C_off=0.2, K=0, K_max=128), s["L_ref"],
                                   None, e)
            assert K == Ks[e]
            got = env_events(ev, e)
            assert U.same_multiset(got, want), (step, e, len(got), len(want), U.multiset_diff(got, want))
            assert np.array_equal(host(envs[e]["L_ref"]).view(np.uint32), R.view(np.uint32))
    assert max(counts) < out.shape[0]


def test_planes_chained_mismatch_refractory(torch, ctx):
    from paper_2607_08098_amd import evis, scenes
    H, W, n_pairs = 480, 640, 3
    say("planes 640x480: render", n_pairs + 1, "frames")
    sc = scenes.PlaneScene(H, W, 2000, n_pairs)
    on, off = scenes.mismatch_thresholds(H, W, 0.25, 0.03, 0.01, scenes.rng_for(2001))
    sensor = o.Sensor(theta_on=on, theta_off=off, refractory_us=100, K=0, K_max=64)
    pairs = []
    for k in range(n_pairs):
        pr = sc.pair(k)
        pairs.append(U.oracle_pair(pr, t0=scenes.frame_time_us(k), t1=scenes.frame_time_us(k + 1)))
    # the oracle, chained through its own state
    R_o = pairs[0].L_A.copy()
    tl_o = np.full((H, W), o.T_LAST_INIT, np.int32)
    # the GPU, chained through device state
    L_ref = torch.from_numpy(R_o.copy()).cuda()
    t_last = torch.from_numpy(tl_o.copy()).cuda()
    th_on, th_off = torch.from_numpy(on).cuda(), torch.from_numpy(off).cuda()
    out, n = evis.event_buffer(1 << 24)
    K_used = torch.zeros(1, dtype=torch.int32, device="cuda")
    for k, pair in enumerate(pairs):
        d = U.device_pair(pair, torch)
        d.update(C_on=0.25, C_off=0.25, theta_on=th_on, theta_off=th_off, refractory_us=100, K=0,
                 K_max=64, L_ref=L_ref, t_last=t_last, env_id=9)
        say("planes pair", k, "GPU")
        n.zero_()
        evis.evis_step_batch(ctx, [d], out, n, K_used)
        torch.cuda.synchronize()
        got = evis.decode_events(out, n)
        say("planes pair", k, "oracle, K", int(K_used[0]))
        want, R_o, tl_o, K = o.step(pair, sensor, R_o, tl_o, 9)
        assert K == int(K_used[0])
        assert len(want) > 1000
        assert U.same_multiset(got, want), (k, len(got), len(want), U.multiset_diff(got, want))
        assert np.array_equal(host(L_ref).view(np.uint32), R_o.view(np.uint32))
        assert np.array_equal(host(t_last), tl_o)

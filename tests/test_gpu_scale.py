"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (autotuned tile, one persistent graph-replayed launch),
against digests the CPU oracle computed from the same seeded scenes
(``tests/golden/fullsize.py``; both sides are fed the oracle's float64 log
intensity rounded to float32, so no input of the oracle comes from the
library):

* the 64-env mixed batch as a keyframe sequence (24 x 346x260,
  24 x 640x480, 16 x 1280x720 rotating blob sequences, adaptive K <= 64),
  three pairs chained through the state: every env's event multiset,
  K and reference level at every step;
* 512 rotating-disc envs at 346x260 (adaptive K <= 128, static background
  on the static-tile path), 200 pairs with the state carried on the device:
  32 envs spread over the batch at every step (event counts each step,
  chained event and state digests every tenth step); at one step, every
  one of the 512 envs in the batched launch against the same env launched
  alone (same events, same reference level);
* the textured-plane scene at 640x480 (exact flow and depth, true
  occlusion), per-pixel threshold mismatch and a 100 us refractory period,
  100 pairs chained through the state: every pair's events, reference
  level and last-event times;
* the benchmark's variants on the mixed batch (two-splat warps, sensor
  noise): sampled envs against the oracle run directly.
"""
import importlib.util
import json
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import evis_oracle as o
import gpu_util as U

pytestmark = pytest.mark.gpu
F32 = np.float32

_spec = importlib.util.spec_from_file_location(
    "fullsize", os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize.py"))
F = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(F)


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


@pytest.fixture(scope="module")
def golden():
    if not os.path.exists(F.DIGEST_FILE):
        return {}
    with open(F.DIGEST_FILE) as fh:
        return json.load(fh)


def case_digests(golden, case):
    if case not in golden:
        pytest.skip(f"the oracle's digests of {case} are not in {os.path.basename(F.DIGEST_FILE)}")
    return golden[case]


def say(*a):
    print("[case]", *a, flush=True)


def host(t):
    return t.detach().cpu().numpy().copy()


def sorted_env_keys(torch, out, n, n_envs=512):
    """The stream's events as sorted int64 keys env << 54 | t << 23 | y << 12
    | x << 1 | p (on the device), and each env's [begin, end) in it."""
    cnt = min(int(n.item()), out.shape[0])
    rec = out[:cnt].long()
    word = rec[:, 0] & 0xFFFFFFFF
    x, y, p = word & 0x7FF, (word >> 11) & 0x7FF, (word >> 22) & 1
    env = (word >> 23) & 0x1FF
    key = (env << 54) | (rec[:, 1] << 23) | (y << 12) | (x << 1) | p
    key, _ = torch.sort(key)
    starts = torch.arange(n_envs, device=key.device, dtype=torch.int64) << 54
    pos = np.append(host(torch.searchsorted(key, starts)), key.numel())
    return key, pos


def env_digest(keys_host_all, pos, e):
    k = keys_host_all[pos[e]:pos[e + 1]] & ((1 << 54) - 1)
    return int(len(k)), F.keys_digest(k)


# ---------------------------------------------------------------------------
# the benchmark's mixed batch as a sequence
# ---------------------------------------------------------------------------

def test_mixed64_sequence_every_env(torch, ctx, golden):
    from paper_2607_08098_amd import evis, workloads
    g = case_digests(golden, "mixed64")
    assert g["steps"] == F.MIXED_STEPS and len(g["envs"]) == 64
    say("mixed64 sequence: generate", F.MIXED_STEPS + 1, "keyframes")
    seq = workloads.MixedSequence(ctx, F.MIXED_STEPS + 1, specs=F.mixed_specs(),
                                  log_fn=F.log_intensity, threads=16)
    sensor = dict(F.MIXED_SENSOR)
    out, n = evis.event_buffer(1 << 28)
    seq.reset_state(0)
    say("mixed64 sequence: autotune")
    best, _ = evis.evis_autotune(ctx, evis.env_array(seq.env_dicts(0, sensor)), out, n, reps=2)
    evis.evis_set_tuning(ctx, **best.as_dict())
    K_used = torch.zeros(64, dtype=torch.int32, device="cuda")
    for s in range(F.MIXED_STEPS):
        say("mixed64 sequence: step", s, "tile", best.tile_w, best.tile_h)
        arr = evis.env_array(seq.env_dicts(s, sensor))
        n.zero_()
        evis.evis_step_batch(ctx, arr, out, n, K_used, 0)
        torch.cuda.synchronize()
        assert 0 < int(n.item()) <= out.shape[0]
        key, pos = sorted_env_keys(torch, out, n)
        keys = host(key)
        Ks = host(K_used)
        L_ref = host(seq.L_ref)
        bad = []
        for e in range(64):
            want = g["envs"][e]["steps"][s]
            cnt, dig = env_digest(keys, pos, e)
            a, b = seq.offsets[e], seq.offsets[e + 1]
            got = dict(K=int(Ks[e]), n=cnt, events=dig, L_ref=F.plane_digest(L_ref[a:b]))
            if got != want:
                bad.append((e, got, want))
        assert not bad, (s, len(bad), bad[:4])


@pytest.mark.parametrize("variant", ["splat_b_primary", "joint", "gather_with_noise"])
def test_mixed64_variants_sampled_parity(torch, ctx, variant):
    """The benchmark's variants at full size in its launch configuration
    (same batch, the tile shape it autotunes for the gather warp): every
    event and reference level of sampled envs against the oracle."""
    from paper_2607_08098_amd import evis, scenes, workloads
    say("mixed64 variant", variant, ": build workload")
    batch = workloads.mixed_batch(ctx, specs=scenes.mixed_batch_specs(3000), log_fn=F.log_intensity)
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
    samples = {"splat_b_primary": [3, 29], "joint": [11], "gather_with_noise": [37]}[variant]
    snap = {e: {k: host(v) for k, v in envs[e].items() if hasattr(v, "cpu")} for e in samples}
    K_used = torch.zeros(len(envs), dtype=torch.int32, device="cuda")
    say("mixed64 variant", variant, ": step")
    n.zero_()
    evis.evis_step_batch(ctx, arr, out, n, K_used, 0)
    torch.cuda.synchronize()
    assert 0 < int(n.item()) <= out.shape[0]
    cnt = int(n.item())
    env_of = (out[:cnt, 0].long() & 0xFFFFFFFF) >> 23
    assert bool((torch.bincount(env_of, minlength=64) > 0).all())   # every env fired
    lut = torch.zeros(512, dtype=torch.bool, device="cuda")
    lut[samples] = True
    sub = out[:cnt][lut[env_of]].contiguous()
    ev = evis.decode_events(sub, torch.tensor([sub.shape[0]], dtype=torch.int64))
    Ks = host(K_used)
    for e in samples:
        s = snap[e]
        say("mixed64 variant", variant, "oracle env", e, s["L_A"].shape, "K", int(Ks[e]))
        pair = o.Pair(s["L_A"], s["L_B"], s["m_A"], s["m_B"], s["Z_A"], s["Z_B"], 0, 16667)
        nz = o.Noise(seed=9000 + e, **noise) if noise else None
        sen = o.Sensor(C_on=0.2, C_off=0.2, K=0, K_max=64, blend_mode=mode, noise=nz)
        want, R, _, K = o.step(pair, sen, s["L_ref"], None, e)
        assert K == Ks[e]
        got = ev[ev[:, 4] == e]
        assert U.same_multiset(got, want), (e, len(got), len(want), U.multiset_diff(got, want))
        assert np.array_equal(host(envs[e]["L_ref"]).view(np.uint32), R.view(np.uint32))


# ---------------------------------------------------------------------------
# 512 discs sustained for 200 steps
# ---------------------------------------------------------------------------

def test_disc512_sustained(torch, ctx, golden):
    from paper_2607_08098_amd import evis, scenes, workloads
    g = case_digests(golden, "disc512")
    checked = F.DISC_ENVS
    assert [r["env"] for r in g["envs"]] == checked and g["steps"] == F.DISC_STEPS
    gold = {r["env"]: r for r in g["envs"]}
    say("disc512: build workload")
    batch = workloads.DiscBatch(ctx, n_envs=F.DISC_N, H=F.DISC_H, W=F.DISC_W,
                                seed_base=F.DISC_SEED_BASE)
    batch.start(0)
    # the checked envs get the host log intensity of the scene generator's
    # frames (the oracle's input); the other 480 keep the device front end
    discs = {e: scenes.DiscScene(F.DISC_H, F.DISC_W,
                                 scenes.disc_scene_params(F.DISC_H, F.DISC_W, F.DISC_SEED_BASE + e))
             for e in checked}
    for e in checked:
        assert np.array_equal(host(batch.view(batch.m_A, e)), discs[e].m)
        assert np.array_equal(host(batch.view(batch.Z_A, e)), discs[e].Z)
    pool = ThreadPoolExecutor(16)

    def host_logs(i):
        return list(pool.map(lambda e: F.log_intensity(discs[e].frame(i / 60.0)), checked))

    def put(buf, i_logs):
        for e, L in zip(checked, i_logs):
            batch.view(buf, e).copy_(torch.from_numpy(L))

    put(batch.L_A, host_logs(0))
    put(batch.L_B, host_logs(1))
    put(batch.L_ref, host_logs(0))
    nxt = pool.submit(host_logs, 2)
    sensor = dict(F.DISC_SENSOR)
    out, n = evis.event_buffer(1 << 26)
    K_used = torch.zeros(F.DISC_N, dtype=torch.int32, device="cuda")
    evis.evis_set_tuning(ctx, tile_w=32, tile_h=16)
    chained = {e: "" for e in checked}
    lut = torch.zeros(512, dtype=torch.bool, device="cuda")
    lut[checked] = True
    for step in range(F.DISC_STEPS):
        if step > 0:
            batch.advance()
            put(batch.L_B, nxt.result())
            if step + 2 <= F.DISC_STEPS:
                nxt = pool.submit(host_logs, step + 2)
        t0, t1 = batch.times()
        arr = evis.env_array(batch.env_dicts(sensor, t0, t1))
        if step == 100:
            _batched_vs_alone(torch, ctx, batch, sensor, t0, t1, out, n)
        evis.evis_step_batch(ctx, arr, out, n, K_used, evis.EVIS_FLAG_RESET_CURSOR)
        torch.cuda.synchronize()
        total = int(n.item())
        assert 0 < total <= out.shape[0], (step, total)
        # only the checked envs' events leave the device
        cnt = min(total, out.shape[0])
        word = out[:cnt, 0].long() & 0xFFFFFFFF
        sel = lut[(word >> 23) & 0x1FF]
        sub = out[:cnt][sel].contiguous()
        nsub = torch.tensor([sub.shape[0]], dtype=torch.int64, device="cuda")
        key, pos = sorted_env_keys(torch, sub, nsub)
        keys = host(key)
        Ks = host(K_used)
        L_ref = host(batch.L_ref)
        bad = []
        for e in checked:
            r = gold[e]
            cnt_e, dig = env_digest(keys, pos, e)
            a, b = batch.offsets[e], batch.offsets[e + 1]
            chained[e] = F.chain(chained[e], dig, F.plane_digest(L_ref[a:b]))
            if cnt_e != r["n"][step] or int(Ks[e]) not in r["K"]:
                bad.append((e, cnt_e, r["n"][step], int(Ks[e]), r["K"]))
            elif str(step) in r["chained"] and chained[e] != r["chained"][str(step)]:
                bad.append((e, "chained digest", step))
        assert not bad, (step, bad[:4])
        if step % 50 == 0:
            say("disc512 step", step, "events", total)
    pool.shutdown()


def _batched_vs_alone(torch, ctx, batch, sensor, t0, t1, out, n):
    """Every env of the batch: the batched launch against the same env
    launched alone, from the same state (events and reference level)."""
    from paper_2607_08098_amd import evis
    say("disc512: every env batched against alone")
    envs = batch.env_dicts(sensor, t0, t1)
    R0 = batch.L_ref.clone()
    n.zero_()
    evis.evis_step_batch(ctx, evis.env_array(envs), out, n, None, 0)
    torch.cuda.synchronize()
    k_batched, _ = sorted_env_keys(torch, out, n)
    R_batched = batch.L_ref.clone()
    batch.L_ref.copy_(R0)
    n.zero_()
    for d in envs:
        evis.evis_step_batch(ctx, evis.env_array([d]), out, n, None, 0)
    torch.cuda.synchronize()
    k_alone, _ = sorted_env_keys(torch, out, n)
    assert k_batched.shape == k_alone.shape and bool(torch.equal(k_batched, k_alone))
    assert bool(torch.equal(R_batched.view(torch.int32), batch.L_ref.view(torch.int32)))
    batch.L_ref.copy_(R0)


# ---------------------------------------------------------------------------
# the textured-plane scene: mismatch, refractory period, 100 pairs
# ---------------------------------------------------------------------------

def test_planes_chained_mismatch_refractory(torch, ctx, golden):
    from paper_2607_08098_amd import evis, scenes
    g = case_digests(golden, "planes640")
    H, W, n_pairs = F.PLANES_H, F.PLANES_W, F.PLANES_PAIRS
    assert len(g["pairs"]) == n_pairs
    say("planes 640x480: render", n_pairs + 1, "keyframes; tuning",
        evis.evis_get_tuning(ctx).as_dict())
    sc = scenes.PlaneScene(H, W, F.PLANES_SEED, n_pairs)
    kf = scenes.render_keyframes(sc, range(n_pairs + 1), threads=16)
    with ThreadPoolExecutor(16) as pool:
        L = list(pool.map(lambda k: F.log_intensity(k[0]), kf))
    on, off = F.planes_thresholds()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    L_ref = dev(L[0])
    t_last = torch.full((H, W), o.T_LAST_INIT, dtype=torch.int32, device="cuda")
    th_on, th_off = dev(on), dev(off)
    out, n = evis.event_buffer(1 << 24)
    K_used = torch.zeros(1, dtype=torch.int32, device="cuda")
    for k in range(n_pairs):
        d = dict(L_A=dev(L[k]), L_B=dev(L[k + 1]), m_A=dev(kf[k][1]), m_B=dev(kf[k + 1][2]),
                 Z_A=dev(kf[k][3]), Z_B=dev(kf[k + 1][3]), t0=scenes.frame_time_us(k),
                 t1=scenes.frame_time_us(k + 1), C_on=0.25, C_off=0.25, theta_on=th_on,
                 theta_off=th_off, L_ref=L_ref, t_last=t_last, env_id=F.PLANES_ENV,
                 **F.PLANES_SENSOR)
        n.zero_()
        evis.evis_step_batch(ctx, [d], out, n, K_used)
        torch.cuda.synchronize()
        key, pos = sorted_env_keys(torch, out, n)
        cnt, dig = env_digest(host(key), pos, F.PLANES_ENV)
        got = dict(K=int(K_used[0]), n=cnt, events=dig, L_ref=F.plane_digest(host(L_ref)),
                   t_last=F.plane_digest(host(t_last)))
        assert got == g["pairs"][k], (k, got, g["pairs"][k])
        if k % 20 == 0:
            say("planes pair", k, "K", got["K"], "events", cnt)

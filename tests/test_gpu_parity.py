"""HIP path (through the C ABI) against the CPU oracle on the same seeded
inputs.  Bars: events and integer outputs bit-exact (as multisets);
interpolated log frames within 1e-5 absolute in float32 (the kernels follow
the oracle's operation order, so they are expected bit-exact and the test
also reports the exact match); log luminance within 4e-6 absolute."""
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


def run_interp(torch, ctx, pair, K, j0, j1, mode):
    from paper_2607_08098_amd import evis
    dp = U.device_pair(pair, torch)
    L, hole = evis.evis_interpolate(ctx, dp, K, j0, j1, mode)
    torch.cuda.synchronize()
    return L.cpu().numpy(), hole.cpu().numpy()


def check_interp(got_L, got_h, want_L, want_h, tag):
    diff = np.abs(got_L.astype(np.float64) - want_L.astype(np.float64))
    assert np.all(np.isfinite(got_L) == np.isfinite(want_L)), tag
    fin = np.isfinite(want_L)
    assert diff[fin].max(initial=0.0) <= 1e-5, (tag, diff[fin].max())
    assert np.array_equal(got_h, want_h), tag
    # the operation order is the oracle's: expect every bit to agree
    assert np.array_equal(got_L.view(np.uint32), want_L.view(np.uint32)), (tag, "not bit-exact")


# ---------------------------------------------------------------------------
# interpolation (splat, gather, blend)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mode", [o.BLEND_TIME, o.BLEND_B_PRIMARY])
def test_interpolate_config1(torch, ctx, mode):
    say("interpolate 128x128 K=8 mode", mode)
    pair = U.oracle_pair(U.blob_scene(128, 128, 1000))
    K = 8
    want_L, want_h = o.interpolate(pair, K, 0, K + 1, mode)
    got_L, got_h = run_interp(torch, ctx, pair, K, 0, K + 1, mode)
    check_interp(got_L, got_h, want_L, want_h, "cfg1")


@pytest.mark.parametrize("shape,seed,K,flow", [
    ((37, 53), 5, 7, "translate"), ((70, 45), 6, 5, "rotate"), ((1, 1), 7, 3, "translate"),
    ((1, 40), 8, 4, "rotate"), ((33, 1), 9, 4, "rotate"), ((96, 130), 10, 16, "rotate")])
def test_interpolate_ragged(torch, ctx, shape, seed, K, flow):
    H, W = shape
    say("interpolate ragged", shape, K, flow)
    kw = dict(flow=flow, omega=12.0) if flow == "rotate" else dict(flow=flow)
    pair = U.oracle_pair(U.blob_scene(H, W, seed, **kw))
    want_L, want_h = o.interpolate(pair, K, 0, K + 1)
    got_L, got_h = run_interp(torch, ctx, pair, K, 0, K + 1, o.BLEND_TIME)
    check_interp(got_L, got_h, want_L, want_h, (shape, K))


def test_interpolate_subrange_and_list_fallback(torch, ctx):
    from paper_2607_08098_amd import evis
    pair = U.oracle_pair(U.blob_scene(80, 90, 11, flow="rotate", omega=18.0))
    K = 12
    want_L, want_h = o.interpolate(pair, K, 3, 9)
    say("interpolate sub-range j=3..8")
    got_L, got_h = run_interp(torch, ctx, pair, K, 3, 9, o.BLEND_TIME)
    check_interp(got_L, got_h, want_L, want_h, "subrange")
    old = evis.evis_get_tuning(ctx).as_dict()
    try:
        evis.evis_set_tuning(ctx, list_cap=3)     # forces the window-scan path
        say("interpolate with the candidate list forced to overflow")
        got_L, got_h = run_interp(torch, ctx, pair, K, 3, 9, o.BLEND_TIME)
        check_interp(got_L, got_h, want_L, want_h, "fallback")
        evis.evis_set_tuning(ctx, list_cap=40)    # some tiles overflow, some do not
        say("interpolate with a partly overflowing candidate list")
        got_L, got_h = run_interp(torch, ctx, pair, K, 3, 9, o.BLEND_TIME)
        check_interp(got_L, got_h, want_L, want_h, "partly overflowing")
    finally:
        evis.evis_set_tuning(ctx, **old)


def test_interpolate_occlusion_and_invalid_depth(torch, ctx):
    rng = np.random.default_rng(12)
    H, W, K = 48, 64, 8
    sc = U.blob_scene(H, W, 12, flow="translate", mean=(6.0, -3.0), noise=0.7)
    pair = U.oracle_pair(sc)
    Z_A = pair.Z_A.copy()
    Z_A[rng.random((H, W)) < 0.05] = -1.0
    Z_A[rng.random((H, W)) < 0.02] = np.nan
    Z_A[rng.random((H, W)) < 0.02] = np.inf
    pair = o.Pair(pair.L_A, pair.L_B, pair.m_A, pair.m_B, Z_A, pair.Z_B)
    want_L, want_h = o.interpolate(pair, K, 0, K + 1)
    say("interpolate with invalid depths")
    got_L, got_h = run_interp(torch, ctx, pair, K, 0, K + 1, o.BLEND_TIME)
    check_interp(got_L, got_h, want_L, want_h, "invalid depth")


# ---------------------------------------------------------------------------
# emission on caller-supplied frames
# ---------------------------------------------------------------------------

def gen_events(torch, ctx, L_seq, t0, t1, sensor, L_ref, t_last, env_id=0, capacity=None):
    from paper_2607_08098_amd import evis
    dev = "cuda"
    Ls = torch.from_numpy(np.ascontiguousarray(L_seq)).to(dev)
    st = dict(L_ref=torch.from_numpy(L_ref.copy()).to(dev),
              t_last=None if t_last is None else torch.from_numpy(t_last.copy()).to(dev))
    sd = dict(C_on=sensor.C_on, C_off=sensor.C_off, refractory_us=sensor.refractory_us)
    if sensor.theta_on is not None:
        sd["theta_on"] = torch.from_numpy(sensor.theta_on).to(dev)
        sd["theta_off"] = torch.from_numpy(sensor.theta_off).to(dev)
    cap = capacity if capacity is not None else 4 * 1024 * 1024
    out, n = evis.event_buffer(cap)
    evis.evis_generate_events(ctx, Ls, t0, t1, sd, st, env_id, out, n)
    torch.cuda.synchronize()
    ev = evis.decode_events(out, n)
    return ev, int(n.item()), st["L_ref"].cpu().numpy(), (None if t_last is None else st["t_last"].cpu().numpy())


@pytest.mark.parametrize("variant", ["plain", "mismatch", "mismatch_nonpositive",
                                     "mismatch_refractory", "hdr_many"])
def test_generate_events_bit_exact(torch, ctx, variant):
    pair = U.oracle_pair(U.blob_scene(96, 120, 21))
    K = 8
    frames, _ = o.interpolate(pair, K, 0, K + 1)
    H, W = pair.shape
    sensor = o.Sensor(C_on=0.2, C_off=0.2, K=K)
    t_last = None
    L_ref = pair.L_A.copy()
    if variant in ("mismatch", "mismatch_nonpositive", "mismatch_refractory"):
        from paper_2607_08098_amd import scenes
        on, off = scenes.mismatch_thresholds(H, W, 0.25, 0.03, 0.01, scenes.rng_for(5))
        if variant == "mismatch_nonpositive":
            # thresholds that are not > 0 (zero, negative, NaN) never cross
            rng = np.random.default_rng(6)
            for th in (on, off):
                th[rng.random((H, W)) < 0.05] = F32(0.0)
                th[rng.random((H, W)) < 0.05] = F32(-0.1)
                th[rng.random((H, W)) < 0.05] = F32(np.nan)
        refr = 100 if variant == "mismatch_refractory" else 0
        sensor = o.Sensor(theta_on=on, theta_off=off, refractory_us=refr, K=K)
        t_last = np.full((H, W), o.T_LAST_INIT, np.int32)
    if variant == "hdr_many":
        # large per-substep contrast: dozens of crossings per pixel-substep
        frames = frames.copy()
        frames[4:] += F32(9.0)
        sensor = o.Sensor(C_on=0.05, C_off=0.07, K=K)
    say("generate_events", variant)
    want, R, tl = o.emit_events(list(frames), 1000, 1000 + 16667, sensor, L_ref, t_last, env_id=3)
    got, n, gR, gtl = gen_events(torch, ctx, frames, 1000, 1000 + 16667, sensor, L_ref, t_last, 3)
    assert n == len(want)
    assert U.same_multiset(got, want), U.multiset_diff(got, want)
    assert np.array_equal(gR.view(np.uint32), R.view(np.uint32))
    if t_last is not None:
        assert np.array_equal(gtl, tl)


def test_generate_events_goldens(torch, ctx):
    import oracle_pins as P
    for name in ("ramp_refractory.txt", "multi_crossing.txt", "exact_floor_off.txt"):
        kv, want = P.read_golden(name)
        K = int(kv["K"])
        L_A, L_B = float(kv["L_A"]), float(kv["L_B"])
        frames = np.stack([np.full((1, 1), F32(L_A + (L_B - L_A) * j / K)) for j in range(K + 1)]).astype(F32)
        C = float(kv["C"])
        sensor = o.Sensor(C_on=C, C_off=C, refractory_us=int(kv["refractory"]), K=K)
        say("generate_events golden", name)
        got, n, R, _ = gen_events(torch, ctx, frames, int(kv["t0"]), int(kv["t1"]), sensor,
                                  np.zeros((1, 1), F32), np.full((1, 1), o.T_LAST_INIT, np.int32))
        assert sorted(map(tuple, got[:, :4].tolist())) == sorted(map(tuple, want)), name


def test_generate_events_capacity_overflow(torch, ctx):
    pair = U.oracle_pair(U.blob_scene(64, 64, 23))
    K = 6
    frames, _ = o.interpolate(pair, K, 0, K + 1)
    sensor = o.Sensor(C_on=0.1, C_off=0.1, K=K)
    want, R, _ = o.emit_events(list(frames), 0, 16667, sensor, pair.L_A.copy())
    assert len(want) > 300
    say("generate_events capacity", 100)
    got, n, gR, _ = gen_events(torch, ctx, frames, 0, 16667, sensor, pair.L_A.copy(), None, capacity=100)
    assert n == len(want) and len(got) == 100
    wanted = set(map(tuple, want.tolist()))
    assert all(tuple(e) in wanted for e in got.tolist())
    assert np.array_equal(gR.view(np.uint32), R.view(np.uint32))   # state still advances


def test_generate_events_appends_and_fills_exact_capacity(torch, ctx):
    """Calls append at the cursor: a first call with reset, a second one
    without (a refractory-free env: the sharded stream whose base is the
    cursor), a third in the workgroup form (refractory period); the union is
    the three oracle multisets.  Then one call into a buffer of exactly its
    event count (every slot of the prefix filled) and one into a buffer one
    event short (the prefix still full, the count still whole)."""
    from paper_2607_08098_amd import evis
    dev = "cuda"
    cases = []
    for e, (seed, refr) in enumerate(((31, 0), (32, 0), (33, 100))):
        pair = U.oracle_pair(U.blob_scene(70, 90, seed))
        frames, _ = o.interpolate(pair, 7, 0, 8)
        sensor = o.Sensor(C_on=0.15, C_off=0.15, K=7, refractory_us=refr)
        t_last = np.full(pair.shape, o.T_LAST_INIT, np.int32) if refr else None
        want, _, _ = o.emit_events(list(frames), 500, 500 + 16667, sensor, pair.L_A.copy(), t_last,
                                   env_id=e)
        cases.append((frames, sensor, pair.L_A.copy(), t_last, want))
    out, n = evis.event_buffer(1 << 20)
    n.fill_(12345)
    for e, (frames, sensor, L_ref, t_last, _) in enumerate(cases):
        st = dict(L_ref=torch.from_numpy(L_ref.copy()).to(dev),
                  t_last=None if t_last is None else torch.from_numpy(t_last.copy()).to(dev))
        sd = dict(C_on=sensor.C_on, C_off=sensor.C_off, refractory_us=sensor.refractory_us)
        say("generate_events append", e)
        evis.evis_generate_events(ctx, torch.from_numpy(np.ascontiguousarray(frames)).to(dev), 500,
                                  500 + 16667, sd, st, e, out, n,
                                  flags=evis.EVIS_FLAG_RESET_CURSOR if e == 0 else 0)
    torch.cuda.synchronize()
    want_all = np.concatenate([c[4] for c in cases])
    assert int(n.item()) == len(want_all)
    assert U.same_multiset(evis.decode_events(out, n), want_all)
    frames, sensor, L_ref, _, want = cases[0]
    for cap in (len(want), len(want) - 1):
        say("generate_events capacity", cap, "of", len(want))
        got, cnt, _, _ = gen_events(torch, ctx, frames, 500, 500 + 16667, sensor, L_ref, None, 0,
                                    capacity=cap)
        assert cnt == len(want) and len(got) == cap
        if cap == len(want):
            assert U.same_multiset(got, want)
        wanted = set(map(tuple, want.tolist()))
        assert all(tuple(e) in wanted for e in got.tolist())


# ---------------------------------------------------------------------------
# fused step
# ---------------------------------------------------------------------------

def run_step(torch, ctx, pairs, sensors, L_refs, t_lasts, env_ids, capacity=8 * 1024 * 1024):
    from paper_2607_08098_amd import evis
    envs, keep = [], []
    for pair, s, L_ref, tl, eid in zip(pairs, sensors, L_refs, t_lasts, env_ids):
        d = U.device_pair(pair, torch)
        d.update(C_on=s.C_on, C_off=s.C_off, refractory_us=s.refractory_us, K=s.K,
                 K_max=s.K_max, blend_mode=s.blend_mode, env_id=eid)
        if s.theta_on is not None:
            d["theta_on"] = torch.from_numpy(s.theta_on).cuda()
            d["theta_off"] = torch.from_numpy(s.theta_off).cuda()
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


def test_step_config1(torch, ctx):
    pair = U.oracle_pair(U.blob_scene(128, 128, 1000))
    s = o.Sensor(C_on=0.2, C_off=0.2, K=8)
    args = ([pair], [s], [pair.L_A.copy()], [None], [0])
    say("step_batch 128x128 blob scene K=8")
    got = run_step(torch, ctx, *args)
    check_step(got, oracle_steps(*args))
    assert got[1] > 1000


@pytest.mark.parametrize("shape,seed,flow,omega", [((96, 130), 31, "rotate", 12.0),
                                                   ((37, 53), 32, "translate", None),
                                                   ((200, 260), 33, "rotate", 40.0)])
def test_one_warped_substep(torch, ctx, shape, seed, flow, omega):
    """K = 2 (one warped substep, the small-motion case): the sub-frames and
    the fused step's events and reference level against the oracle, bit
    for bit, on ragged multi-tile frames, one with motion of tens of
    pixels."""
    H, W = shape
    kw = dict(flow=flow, omega=omega) if flow == "rotate" else dict(flow=flow)
    pair = U.oracle_pair(U.blob_scene(H, W, seed, **kw))
    say("one warped substep", shape, flow, omega)
    want_L, want_h = o.interpolate(pair, 2, 0, 3)
    got_L, got_h = run_interp(torch, ctx, pair, 2, 0, 3, o.BLEND_TIME)
    check_interp(got_L, got_h, want_L, want_h, (shape, "K=2"))
    s = o.Sensor(C_on=0.1, C_off=0.1, K=2)
    args = ([pair], [s], [pair.L_A.copy()], [None], [3])
    got = run_step(torch, ctx, *args)
    check_step(got, oracle_steps(*args))
    assert got[1] > 100


def test_step_mixed_small_batch(torch, ctx):
    """Envs of uneven size, K, blend mode, mismatch and refractory in one launch."""
    from paper_2607_08098_amd import scenes
    specs = [(40, 56, "rotate", 5.0), (64, 48, "translate", None), (33, 71, "rotate", 19.0),
             (17, 9, "rotate", 2.0), (90, 64, "rotate", 11.0)]
    pairs, sensors, L_refs, tls, ids = [], [], [], [], []
    for i, (H, W, flow, om) in enumerate(specs):
        kw = dict(flow=flow, omega=om) if flow == "rotate" else dict(flow=flow)
        pair = U.oracle_pair(U.blob_scene(H, W, 300 + i, **kw), t0=5000 * i, t1=5000 * i + 16667)
        if i % 2 == 0:
            s = o.Sensor(C_on=0.2, C_off=0.2, K=0, K_max=64)
            tl = None
        else:
            on, off = scenes.mismatch_thresholds(H, W, 0.25, 0.03, 0.01, scenes.rng_for(50 + i))
            s = o.Sensor(theta_on=on, theta_off=off, refractory_us=100, K=0, K_max=64,
                         blend_mode=o.BLEND_B_PRIMARY if i == 3 else o.BLEND_TIME)
            tl = np.full((H, W), o.T_LAST_INIT, np.int32)
        pairs.append(pair)
        sensors.append(s)
        L_refs.append(pair.L_A.copy())
        tls.append(tl)
        ids.append(7 * i + 1)
    args = (pairs, sensors, L_refs, tls, ids)
    want = oracle_steps(*args)
    say("step_batch mixed 5 envs")
    check_step(run_step(torch, ctx, *args), want)


@pytest.mark.parametrize("list_cap", [12, 48, 160])
def test_step_capped_candidate_lists(torch, ctx, list_cap):
    """A fast rotation with the candidate list capped: tiles whose list
    overflows take the window scan; the events must not change."""
    from paper_2607_08098_amd import evis
    pair = U.oracle_pair(U.blob_scene(96, 112, 41, flow="rotate", omega=19.0))
    s = o.Sensor(C_on=0.2, C_off=0.2, K=0, K_max=64)
    args = ([pair], [s], [pair.L_A.copy()], [None], [5])
    want = oracle_steps(*args)
    old = evis.evis_get_tuning(ctx).as_dict()
    try:
        evis.evis_set_tuning(ctx, list_cap=list_cap)
        say("step_batch with list_cap", list_cap)
        check_step(run_step(torch, ctx, *args), want)
    finally:
        evis.evis_set_tuning(ctx, **old)


def test_step_static_scene_fast_path(torch, ctx):
    """Zero motion everywhere and L_A == L_B: the static-tile path must give
    the oracle's events (from the reference catching up with L_A)."""
    sc = U.blob_scene(70, 90, 31)
    L_A, _ = U.log_frames(sc)
    m = np.zeros_like(sc["m_A"])
    pair = o.Pair(L_A, L_A.copy(), m, m.copy(), sc["Z_A"], sc["Z_A"].copy(), 0, 16667)
    rng = np.random.default_rng(31)
    L_ref = (L_A + rng.normal(0, 0.5, size=L_A.shape)).astype(F32)
    s = o.Sensor(C_on=0.2, C_off=0.2, K=6)
    args = ([pair], [s], [L_ref], [None], [2])
    want = oracle_steps(*args)
    assert len(want[0]) > 100
    say("step_batch static scene")
    check_step(run_step(torch, ctx, *args), want)


def test_substep_count(torch, ctx):
    from paper_2607_08098_amd import evis
    for seed, om in ((1, 0.5), (2, 7.3), (3, 19.9)):
        pair = U.oracle_pair(U.blob_scene(60, 80, seed, flow="rotate", omega=om))
        for K_max in (64, 5):
            say("substep_count", seed, K_max)
            K = evis.evis_substep_count(ctx, U.device_pair(pair, torch), K_max)
            torch.cuda.synchronize()
            assert int(K.item()) == o.adaptive_k(pair.m_A, pair.m_B, K_max)


def test_log_luminance(torch, ctx):
    from paper_2607_08098_amd import evis
    rng = np.random.default_rng(41)
    mono = (10.0 ** rng.uniform(-2, 3, size=(50, 70))).astype(F32)
    rgb = (10.0 ** rng.uniform(-2, 3, size=(30, 20, 3))).astype(F32)
    for x in (mono, rgb):
        say("log_luminance", x.shape)
        got = evis.evis_log_luminance(ctx, torch.from_numpy(x).cuda()).cpu().numpy()
        want = o.log_luminance(x.astype(np.float64))
        assert np.abs(got - want).max() <= 4e-6

"""evis_generate_events_batch: the event model over caller frames of many
envs in one call, against the oracle env by env (bit-exact event
multisets, reference levels and last-event times), with uneven sizes and
substep counts (below, at and above a block of eight), per-pixel
thresholds with and without a refractory period (the two envs with one
go to the workgroup form, the others to the wave form), dozens of
crossings per pixel-substep in another; and its host-detected errors
enqueue nothing."""
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


def make_case(H, W, K, seed, kind):
    from paper_2607_08098_amd import scenes
    pair = U.oracle_pair(U.blob_scene(H, W, seed, flow="rotate", omega=5.0 + seed % 7))
    frames, _ = o.interpolate(pair, K, 0, K + 1)
    sensor = o.Sensor(C_on=0.2, C_off=0.2, K=K)
    t_last = None
    if kind in ("refractory", "mismatch"):
        on, off = scenes.mismatch_thresholds(H, W, 0.25, 0.03, 0.01, scenes.rng_for(seed))
        refr = 100 if kind == "refractory" else 0
        sensor = o.Sensor(theta_on=on, theta_off=off, refractory_us=refr, K=K)
        t_last = np.full((H, W), o.T_LAST_INIT, np.int32)
    if kind == "hdr":
        frames = frames.copy()
        frames[K // 2:] += F32(6.0)
        sensor = o.Sensor(C_on=0.05, C_off=0.07, K=K)
    return frames, sensor, pair.L_A.copy(), t_last


def test_generate_events_batch_matches_oracle(torch, ctx):
    from paper_2607_08098_amd import evis
    specs = [(37, 53, 3, 801, None), (96, 120, 8, 802, "refractory"), (260, 346, 11, 803, None),
             (64, 64, 5, 804, "hdr"), (1, 1, 1, 805, None), (200, 17, 16, 806, None),
             (90, 70, 9, 807, "mismatch"), (50, 61, 4, 808, "refractory")]
    dev = "cuda"
    items, want = [], []
    for e, (H, W, K, seed, kind) in enumerate(specs):
        frames, sensor, L_ref, t_last = make_case(H, W, K, seed, kind)
        t0 = 1000 * (e + 1)
        t1 = t0 + 16667
        w, R, tl = o.emit_events(list(frames), t0, t1, sensor, L_ref, t_last, env_id=10 + e)
        want.append((w, R, tl))
        d = dict(L_seq=torch.from_numpy(np.ascontiguousarray(frames)).to(dev), t0=t0, t1=t1,
                 env_id=10 + e, C_on=sensor.C_on, C_off=sensor.C_off,
                 refractory_us=sensor.refractory_us, L_ref=torch.from_numpy(L_ref).to(dev))
        if t_last is not None:
            d["t_last"] = torch.from_numpy(t_last.copy()).to(dev)
        if sensor.theta_on is not None:
            d["theta_on"] = torch.from_numpy(sensor.theta_on).to(dev)
            d["theta_off"] = torch.from_numpy(sensor.theta_off).to(dev)
        items.append(d)
    out, n = evis.event_buffer(1 << 22)
    say("generate_events_batch", len(items), "envs")
    evis.evis_generate_events_batch(ctx, items, out, n)
    torch.cuda.synchronize()
    got = evis.decode_events(out, n)
    assert int(n.item()) == sum(len(w[0]) for w in want)
    for e, (d, (w, R, tl)) in enumerate(zip(items, want)):
        g = got[got[:, 4] == 10 + e]
        assert U.same_multiset(g, w), (e, len(g), len(w), U.multiset_diff(g, w))
        assert np.array_equal(d["L_ref"].cpu().numpy().view(np.uint32), R.view(np.uint32)), e
        if tl is not None:
            assert np.array_equal(d["t_last"].cpu().numpy(), tl), e


def test_generate_events_batch_errors_enqueue_nothing(torch, ctx):
    from paper_2607_08098_amd import evis
    L = torch.zeros((5, 8, 9), dtype=torch.float32, device="cuda")
    good = dict(L_seq=L, t0=0, t1=100, C_on=0.2, C_off=0.2, L_ref=torch.zeros(8, 9, device="cuda"))
    out, n = evis.event_buffer(64)
    n.fill_(5)
    for bad, code in ((dict(C_on=0.0), evis.EVIS_ERR_INVALID), (dict(t1=0), evis.EVIS_ERR_INVALID),
                      (dict(refractory_us=10), evis.EVIS_ERR_INVALID),
                      (dict(env_id=600), evis.EVIS_ERR_INVALID)):
        with pytest.raises(evis.EvisError) as ei:
            evis.evis_generate_events_batch(ctx, [good, dict(good, **bad)], out, n, flags=0)
        assert ei.value.code == code, bad
    torch.cuda.synchronize()
    assert int(n.item()) == 5


def _items(torch, specs, t0=1000):
    from paper_2607_08098_amd import evis
    dev = "cuda"
    items, want = [], []
    for e, (H, W, K, seed, kind) in enumerate(specs):
        frames, sensor, L_ref, t_last = make_case(H, W, K, seed, kind)
        w, R, tl = o.emit_events(list(frames), t0, t0 + 16667, sensor, L_ref, t_last, env_id=20 + e)
        want.append((w, R, tl))
        d = dict(L_seq=torch.from_numpy(np.ascontiguousarray(frames)).to(dev), t0=t0, t1=t0 + 16667,
                 env_id=20 + e, C_on=sensor.C_on, C_off=sensor.C_off,
                 refractory_us=sensor.refractory_us, L_ref=torch.from_numpy(L_ref).to(dev))
        if t_last is not None:
            d["t_last"] = torch.from_numpy(t_last.copy()).to(dev)
        if sensor.theta_on is not None:
            d["theta_on"] = torch.from_numpy(sensor.theta_on).to(dev)
            d["theta_off"] = torch.from_numpy(sensor.theta_off).to(dev)
        items.append(d)
    return items, want


def test_generate_events_batch_overflow_appends_and_reset(torch, ctx):
    """A batch appended after existing events (no reset): the union; the
    same batch into a buffer too small for it: the count is whole, every
    stored slot holds one of its events, the states still advance; a batch
    of refractory envs only (no wave form) with the reset flag starts at 0;
    K = 128, the largest substep count."""
    from paper_2607_08098_amd import evis
    specs = [(40, 70, 128, 811, None), (90, 70, 9, 812, "mismatch"), (33, 65, 7, 813, "refractory")]
    items, want = _items(torch, specs)
    total = sum(len(w[0]) for w in want)
    out, n = evis.event_buffer(1 << 22)
    say("batch appended after", 777, "events")
    n.fill_(777)
    evis.evis_generate_events_batch(ctx, items, out, n, flags=0)
    torch.cuda.synchronize()
    assert int(n.item()) == 777 + total
    got = evis.decode_events(out[777:], torch.tensor([total], dtype=torch.int64))
    assert U.same_multiset(got, np.concatenate([w[0] for w in want]))
    for d, (w, R, tl) in zip(items, want):
        assert np.array_equal(d["L_ref"].cpu().numpy().view(np.uint32), R.view(np.uint32))
    # too small a buffer (fresh states)
    items, want = _items(torch, specs)
    cap = total // 2
    out2, n2 = evis.event_buffer(cap)
    say("batch into a buffer of", cap, "for", total)
    evis.evis_generate_events_batch(ctx, items, out2, n2)
    torch.cuda.synchronize()
    assert int(n2.item()) == total
    got = evis.decode_events(out2, n2)
    assert len(got) == cap
    wanted = set(map(tuple, np.concatenate([w[0] for w in want]).tolist()))
    assert all(tuple(e) in wanted for e in got.tolist())
    for d, (w, R, tl) in zip(items, want):
        assert np.array_equal(d["L_ref"].cpu().numpy().view(np.uint32), R.view(np.uint32))
    # refractory envs only, with reset
    items, want = _items(torch, [(33, 65, 7, 814, "refractory"), (20, 20, 3, 815, "refractory")])
    n.fill_(999)
    say("batch of refractory envs with reset")
    evis.evis_generate_events_batch(ctx, items, out, n)
    torch.cuda.synchronize()
    w_all = np.concatenate([w[0] for w in want])
    assert int(n.item()) == len(w_all)
    assert U.same_multiset(evis.decode_events(out, n), w_all)

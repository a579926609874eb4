"""The library's documented bound on the crossings of one pixel-substep
(EVIS_MAX_CROSSINGS = 65535, include/evis.h), tested on its own.

Eq. 4 has no such bound and the oracle's default count is exact; the
library caps n at the bound (an infinite difference counting as the bound)
and moves the reference by fl(n * C) with the capped n.  For log
intensities from the library's own front end (ln(Y + 1e-3) of a finite
float32 Y lies in [ln 1e-3, ln FLT_MAX], a span below 96) the cap is out of
reach for any C above 96 / 65535 = 0.0015; caller-supplied frames can reach
it.  Here pixels of a zero-motion pair climb 15000 log units per substep at
C = 0.2 (75000 crossings, capped) and 13000 (exactly 65000, not capped)."""
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


def steep_pair():
    H, W = 16, 24
    rng = np.random.default_rng(5)
    L_A = rng.uniform(-1.0, 1.0, (H, W)).astype(F32)
    L_B = (L_A + rng.uniform(-0.5, 0.5, (H, W))).astype(F32)
    L_B[3, 5] = F32(L_A[3, 5] + F32(30000.0))       # 15000 per substep at K = 2: capped
    L_B[9, 17] = F32(L_A[9, 17] - F32(30000.0))      # falling, capped
    L_B[12, 2] = F32(L_A[12, 2] + F32(26000.0))      # 13000 per substep: 65000, exact
    m = np.zeros((H, W, 2), F32)
    Z = np.ones((H, W), F32)
    return o.Pair(L_A, L_B, m, m.copy(), Z, Z.copy(), 0, 16667)


def test_cap_is_active_in_the_case():
    """The exact count exceeds the bound at the two steep pixels and not at the third."""
    from paper_2607_08098_amd import evis
    p = steep_pair()
    c = F32(0.2)
    for (y, x), capped in (((3, 5), True), ((9, 17), True), ((12, 2), False)):
        half = o.lerp(p.L_A[y, x], p.L_B[y, x], F32(0.5))
        n = o.crossing_count(abs(half - p.L_A[y, x]), c)
        assert (n > evis.EVIS_MAX_CROSSINGS) == capped, (y, x, n)


def test_step_caps_crossings(torch, ctx):
    from paper_2607_08098_amd import evis
    pair = steep_pair()
    s = o.Sensor(C_on=0.2, C_off=0.2, K=2)
    want, R, _, _ = o.step(pair, s, pair.L_A.copy(), count_limit=evis.EVIS_MAX_CROSSINGS)
    d = U.device_pair(pair, torch)
    d.update(C_on=0.2, C_off=0.2, refractory_us=0, K=2, K_max=64, blend_mode=0, env_id=9)
    d["L_ref"] = torch.from_numpy(pair.L_A.copy()).cuda()
    d["t_last"] = None
    out, n = evis.event_buffer(1 << 20)
    say("step_batch at the crossing bound, oracle events", len(want))
    evis.evis_step_batch(ctx, [d], out, n, None)
    torch.cuda.synchronize()
    ev = evis.decode_events(out, n)
    want[:, 4] = 9
    assert int(n.item()) == len(want)
    assert U.same_multiset(ev, want), U.multiset_diff(ev, want)
    per_px = {(x, y): int(((ev[:, 0] == x) & (ev[:, 1] == y)).sum()) for (y, x) in ((3, 5), (9, 17), (12, 2))}
    assert per_px[(5, 3)] == per_px[(17, 9)] == 2 * evis.EVIS_MAX_CROSSINGS
    assert per_px[(2, 12)] == 2 * 65000
    got_R = d["L_ref"].cpu().numpy()
    assert np.array_equal(got_R.view(np.uint32), R.view(np.uint32))


def test_generate_events_caps_crossings(torch, ctx):
    """The event model over caller frames (k_events) applies the same bound."""
    from paper_2607_08098_amd import evis
    pair = steep_pair()
    frames = np.stack([pair.L_A, o.lerp(pair.L_A, pair.L_B, F32(0.5)), pair.L_B]).astype(F32)
    s = o.Sensor(C_on=0.2, C_off=0.2, K=2)
    want, R, _ = o.emit_events(list(frames), 0, 16667, s, pair.L_A.copy(), env_id=4,
                               count_limit=evis.EVIS_MAX_CROSSINGS)
    L_ref = torch.from_numpy(pair.L_A.copy()).cuda()
    out, n = evis.event_buffer(1 << 20)
    say("generate_events at the crossing bound, oracle events", len(want))
    evis.evis_generate_events(ctx, torch.from_numpy(frames).cuda(), 0, 16667,
                              dict(C_on=0.2, C_off=0.2, refractory_us=0, K=2, K_max=64,
                                   blend_mode=0),
                              dict(L_ref=L_ref), 4, out, n)
    torch.cuda.synchronize()
    ev = evis.decode_events(out, n)
    assert int(n.item()) == len(want)
    assert U.same_multiset(ev, want), U.multiset_diff(ev, want)
    assert np.array_equal(L_ref.cpu().numpy().view(np.uint32), R.view(np.uint32))

"""Frames that do not change: zero motion and L_B = L_A, so every tile of the
fused step's gather warp takes the static-tile path (K = 8 fixed; the path
is tried for K > 3); the two-splat warps, which run the full path, on the
same frames.  Every sample of such a tile is L_A, so once a substep leaves each
pixel within its thresholds of the reference no later substep can emit,
and the kernel stops the tile's substeps there.  Against the oracle's full
step: events as a multiset, reference level and last-event times bit for
bit, for a reference equal to L_A (no events), offset from it (events at
the first substep only), the same with a refractory period, and pixels
whose reference is so far off that the per-substep crossing bound leaves
them above threshold (the later substeps keep emitting)."""
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


def static_pair(H, W, seed):
    rng = np.random.default_rng(seed)
    L = rng.uniform(-2.0, 2.0, (H, W)).astype(F32)
    m = np.zeros((H, W, 2), F32)
    Z = np.ones((H, W), F32)
    return o.Pair(L, L.copy(), m, m.copy(), Z, Z.copy(), 1000, 17667)


@pytest.mark.parametrize("warp", [0, o.WARP_SPLAT, o.WARP_JOINT])
@pytest.mark.parametrize("case", ["quiet", "offset", "offset_refractory", "capped"])
def test_static_tiles(torch, ctx, case, warp):
    from paper_2607_08098_amd import evis
    H, W, K = 70, 100, 8
    pair = static_pair(H, W, 40)
    rng = np.random.default_rng(41)
    R0 = pair.L_A.copy()
    refr, tl0 = 0, None
    limit = None
    if case != "quiet":
        R0 = (pair.L_A + rng.uniform(-1.0, 1.0, (H, W))).astype(F32)
    if case == "offset_refractory":
        refr = 100
        tl0 = np.full((H, W), o.T_LAST_INIT, np.int32)
        tl0[::3, ::2] = 1000 + 2000   # a recent event: the first substep's are suppressed there
    if case == "capped":
        limit = evis.EVIS_MAX_CROSSINGS
        R0[5, 7] = F32(pair.L_A[5, 7] - F32(20000.0))    # 100000 crossings at C = 0.2
        R0[40, 90] = F32(pair.L_A[40, 90] + F32(14000.0))
    s = o.Sensor(C_on=0.2, C_off=0.2, K=K, refractory_us=refr, blend_mode=warp)
    want, R, tl, Kw = o.step(pair, s, R0.copy(), None if tl0 is None else tl0.copy(), 6,
                             count_limit=limit)
    d = U.device_pair(pair, torch)
    d.update(C_on=0.2, C_off=0.2, refractory_us=refr, K=K, K_max=64, blend_mode=warp, env_id=6)
    d["L_ref"] = torch.from_numpy(R0.copy()).cuda()
    d["t_last"] = None if tl0 is None else torch.from_numpy(tl0.copy()).cuda()
    out, n = evis.event_buffer(1 << 22)
    K_used = torch.zeros(1, dtype=torch.int32, device="cuda")
    say("static tiles", case, hex(warp), "oracle events", len(want))
    evis.evis_step_batch(ctx, [d], out, n, K_used)
    torch.cuda.synchronize()
    ev = evis.decode_events(out, n)
    assert int(K_used[0]) == Kw == K
    assert int(n.item()) == len(want)
    assert U.same_multiset(ev, want), U.multiset_diff(ev, want)
    got_R = d["L_ref"].cpu().numpy()
    assert np.array_equal(got_R.view(np.uint32), R.view(np.uint32))
    if tl0 is not None:
        assert np.array_equal(d["t_last"].cpu().numpy(), tl)
    if case == "quiet":
        assert len(want) == 0
    if case in ("offset", "offset_refractory"):   # all at the first substep
        assert len(want) > 1000 and len(np.unique(want[:, 2])) == 1
    if case == "capped":   # the capped pixel goes on emitting after the first substep
        px = want[(want[:, 0] == 7) & (want[:, 1] == 5)]
        assert len(px) > limit and len(np.unique(px[:, 2])) >= 2

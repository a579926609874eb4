"""Event voxel grid through the C ABI against the CPU oracle on the same
event stream.

The oracle is the paper's reading in float64 (real time positions, linear
interpolation weights, no bound on the events per voxel).  The library
keeps its sums in 16-bit fixed point (uint32 atomics, exact and
order-free) with a float32 time scale, so each voxel is compared within a
bound derived from that format:

* per event and bin the weight differs by at most
  eps_e = 2^-16 (the floor of the fraction to 16 bits) + (B - 1) 2^-22 (the
  float32 scale and product; the interpolation weight is 1-Lipschitz in
  the time position, so a bin decision taken on either side of a bin
  centre changes a weight by no more than the position does);
* a voxel touched by n_v events (those within one bin, plus the rounding
  margin, of its centre) has |sum_lib - sum| <= n_v eps_e, and its plane
  maximum M moves by at most D_M = max over the plane of n_v eps_e;
* after the division, |g_lib - g| <= (n_v eps_e + g D_M) / (M - D_M) plus
  four float32 roundings (two integer conversions, the quotient, slack).
Planes whose maximum is not above D_M are undetermined by the bound; the
test requires them to be rare.  The library's own limit (a voxel holds at
most 65535 full-weight events before its uint32 sum wraps) is tested at
its boundary."""
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


def stream_of_two_envs(torch, ctx, capacity=1 << 22):
    """Events of two envs from the fused step, left on the device."""
    from paper_2607_08098_amd import evis
    envs = []
    for i, (H, W) in enumerate(((60, 80), (45, 70))):
        pair = U.oracle_pair(U.blob_scene(H, W, 900 + i, flow="rotate", omega=14.0),
                             t0=100000, t1=116667)
        d = U.device_pair(pair, torch)
        d.update(C_on=0.15, C_off=0.15, refractory_us=0, K=0, K_max=64, blend_mode=0, env_id=3 + i)
        d["L_ref"] = torch.from_numpy(pair.L_A.copy()).cuda()
        d["t_last"] = None
        envs.append(d)
    out, n = evis.event_buffer(capacity)
    evis.evis_step_batch(ctx, envs, out, n, None)
    torch.cuda.synchronize()
    return out, n


def touch_counts(ev, env, H, W, t0, t1, bins):
    """n_v: events of the env in [t0, t1) within 1 + 1e-3 bins of each voxel's
    bin centre (the events that can give it weight on either side)."""
    ev = np.asarray(ev, np.int64).reshape(-1, 5)
    ev = ev[(ev[:, 4] == env) & (ev[:, 2] >= t0) & (ev[:, 2] < t1)]
    tau = (ev[:, 2] - t0).astype(np.float64) * (bins - 1) / (t1 - t0)
    cnt = np.zeros((2, bins, H, W), np.int64)
    base = np.floor(tau).astype(np.int64)
    for off in (-1, 0, 1, 2):
        bb = base + off
        sel = (bb >= 0) & (bb < bins) & (np.abs(tau - bb) <= 1.001)
        np.add.at(cnt, (ev[sel, 3], bb[sel], ev[sel, 1], ev[sel, 0]), 1)
    return cnt


def check_grid(got, ev, env, H, W, t0, t1, bins):
    """got (library, float32) against the float64 oracle within the derived
    bound; returns the number of undetermined planes."""
    want = o.voxel_grid(ev, env, H, W, t0, t1, bins)
    acc = o.voxel_counts(ev, env, H, W, t0, t1, bins)
    n_v = touch_counts(ev, env, H, W, t0, t1, bins).astype(np.float64)
    eps_e = 2.0 ** -16 + (bins - 1) * 2.0 ** -22
    M = acc.reshape(2, bins, -1).max(axis=2)[:, :, None, None]
    D_M = (n_v * eps_e).reshape(2, bins, -1).max(axis=2)[:, :, None, None]
    determined = M > D_M
    with np.errstate(divide="ignore", invalid="ignore"):
        tol = (n_v * eps_e + want * D_M) / (M - D_M) + 4.0 * 2.0 ** -24 * (want + 1.0)
    err = np.abs(got.astype(np.float64) - want)
    bad = determined & (err > tol)
    assert not bad.any(), (int(bad.sum()), float(err[bad].max()), float(tol[bad].min()))
    # planes with no event at all are zero on both sides
    empty = (n_v.reshape(2, bins, -1).max(axis=2) == 0)[:, :, None, None]
    assert np.all(got[np.broadcast_to(empty, got.shape)] == 0.0)
    return int((~determined).sum())


@pytest.mark.parametrize("bins,window", [(128, (100000, 116667)), (5, (103000, 111000)),
                                         (2, (100000, 200000))])
def test_voxel_grid_matches_oracle(torch, ctx, bins, window):
    from paper_2607_08098_amd import evis
    out, n = stream_of_two_envs(torch, ctx)
    ev = evis.decode_events(out, n)
    assert len(ev) > 5000
    t0, t1 = window
    undetermined = 0
    for env, (H, W) in ((3, (60, 80)), (4, (45, 70))):
        say("voxel grid", bins, window, env)
        got = evis.evis_voxel_grid(ctx, out, n, env, H, W, t0, t1, bins).cpu().numpy()
        undetermined += check_grid(got, ev, env, H, W, t0, t1, bins)
        assert got.max() == 1.0
    assert undetermined <= max(1, (2 * 2 * bins) // 100), undetermined


@pytest.mark.parametrize("shift", [1, 2, 3])
def test_voxel_grid_unaligned_output(torch, ctx, shift):
    """A grid that starts `shift` words past a 16-byte boundary (the zero
    fill's word head and tail, the per-plane passes' word paths) equals the
    grid written to an aligned buffer, bit for bit, and no word outside it
    is written."""
    from paper_2607_08098_amd import evis
    out, n = stream_of_two_envs(torch, ctx)
    for env, (H, W) in ((3, (60, 80)), (4, (45, 70))):
        for bins in (5, 128):
            say("voxel grid unaligned", shift, env, bins)
            ref = evis.evis_voxel_grid(ctx, out, n, env, H, W, 100000, 116667, bins)
            m = 2 * bins * H * W
            big = torch.full((m + 8,), -7.0, dtype=torch.float32, device="cuda")
            view = big[shift:shift + m].view(2, bins, H, W)
            evis.evis_voxel_grid(ctx, out, n, env, H, W, 100000, 116667, bins, out=view)
            torch.cuda.synchronize()
            assert torch.equal(view, ref)
            assert bool((big[:shift] == -7.0).all()) and bool((big[shift + m:] == -7.0).all())


def test_voxel_grid_full_voxel_limit(torch, ctx):
    """65535 events on one bin centre of one voxel (the most a voxel holds
    at full weight before its uint32 sum wraps), plus a few elsewhere: the
    crowded voxel is exactly the plane maximum and the rest match the
    oracle."""
    from paper_2607_08098_amd import evis
    H, W, bins, t0, t1 = 4, 5, 9, 0, 8000            # bin centres every 1000 us
    n_full = 65535
    rng = np.random.default_rng(17)
    ev = np.zeros((n_full + 300, 5), np.int64)
    ev[:n_full] = (2, 1, 3000, 1, 7)                  # tau = 3 exactly
    ev[n_full:] = np.stack([rng.integers(0, W, 300), rng.integers(0, H, 300),
                            rng.integers(t0, t1, 300), rng.integers(0, 2, 300),
                            np.full(300, 7)], axis=1)
    crowd = (ev[n_full:, 0] == 2) & (ev[n_full:, 1] == 1)
    ev[n_full:, 3][crowd] = 0                         # nothing else in the crowded voxel's polarity
    rec = o.pack_events(ev).astype(np.int64)
    dev = torch.from_numpy(rec.astype(np.uint32).view(np.int32)).cuda().contiguous()
    n = torch.tensor([len(ev)], dtype=torch.int64, device="cuda")
    say("voxel grid at the per-voxel limit")
    got = evis.evis_voxel_grid(ctx, dev, n, 7, H, W, t0, t1, bins).cpu().numpy()
    assert got[1, 3, 1, 2] == 1.0
    check_grid(got, ev, 7, H, W, t0, t1, bins)


def test_voxel_grid_reads_at_most_capacity(torch, ctx):
    """A cursor past the buffer: only the stored events count."""
    from paper_2607_08098_amd import evis
    out, n = stream_of_two_envs(torch, ctx, capacity=3000)
    assert int(n.item()) > 3000
    ev = evis.decode_events(out, n)
    assert len(ev) == 3000
    say("voxel grid of a truncated stream")
    got = evis.evis_voxel_grid(ctx, out, n, 3, 60, 80, 100000, 116667, 16).cpu().numpy()
    check_grid(got, ev, 3, 60, 80, 100000, 116667, 16)


def test_voxel_grid_errors(torch, ctx):
    from paper_2607_08098_amd import evis
    out, n = evis.event_buffer(16)
    for kw in (dict(bins=1), dict(bins=2000), dict(t1_us=0), dict(env_id=600), dict(H=3000)):
        args = dict(env_id=0, H=8, W=8, t0_us=0, t1_us=100, bins=4)
        args.update(kw)
        with pytest.raises(evis.EvisError) as ei:
            evis.evis_voxel_grid(ctx, out, n, args["env_id"], args["H"], args["W"], args["t0_us"],
                                 args["t1_us"], args["bins"],
                                 out=torch.empty(2 * args["bins"] * args["H"] * args["W"],
                                                 device="cuda"))
        assert ei.value.code in (evis.EVIS_ERR_INVALID, evis.EVIS_ERR_UNSUPPORTED), kw

"""Event voxel grid through the C ABI against the CPU oracle on the same
event stream: bit-exact (integer fixed-point sums, then one float32
division per voxel by its plane's maximum)."""
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


@pytest.mark.parametrize("bins,window", [(128, (100000, 116667)), (5, (103000, 111000)),
                                         (2, (100000, 200000))])
def test_voxel_grid_matches_oracle(torch, ctx, bins, window):
    from paper_2607_08098_amd import evis
    out, n = stream_of_two_envs(torch, ctx)
    ev = evis.decode_events(out, n)
    assert len(ev) > 5000
    t0, t1 = window
    for env, (H, W) in ((3, (60, 80)), (4, (45, 70))):
        say("voxel grid", bins, window, env)
        got = evis.evis_voxel_grid(ctx, out, n, env, H, W, t0, t1, bins).cpu().numpy()
        want = o.voxel_grid(ev, env, H, W, t0, t1, bins)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (bins, env)
        assert got.max() == 1.0


def test_voxel_grid_reads_at_most_capacity(torch, ctx):
    """A cursor past the buffer: only the stored events count."""
    from paper_2607_08098_amd import evis
    out, n = stream_of_two_envs(torch, ctx, capacity=3000)
    assert int(n.item()) > 3000
    ev = evis.decode_events(out, n)
    assert len(ev) == 3000
    say("voxel grid of a truncated stream")
    got = evis.evis_voxel_grid(ctx, out, n, 3, 60, 80, 100000, 116667, 16).cpu().numpy()
    want = o.voxel_grid(ev, 3, 60, 80, 100000, 116667, 16)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_voxel_grid_errors(torch, ctx):
    from paper_2607_08098_amd import evis
    out, n = evis.event_buffer(16)
    for kw in (dict(bins=1), dict(bins=2000), dict(t1_us=0), dict(env_id=600), dict(H=3000)):
        args = dict(env_id=0, H=8, W=8, t0_us=0, t1_us=100, bins=4)
        args.update(kw)
        with pytest.raises(evis.EvisError) as ei:
            evis.evis_voxel_grid(ctx, out, n, args["env_id"], args["H"], args["W"], args["t0_us"],
                                 args["t1_us"], args["bins"],
                                 out=torch.empty(2 * 4 * 8 * 8, device="cuda"))
        assert ei.value.code in (evis.EVIS_ERR_INVALID, evis.EVIS_ERR_UNSUPPORTED), kw

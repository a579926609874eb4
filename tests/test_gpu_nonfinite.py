"""Non-finite inputs (NaN and infinite log intensities and motion vectors)
through the fused step for every warp, with sensor noise: the kernels stay
inside their arrays and, since every decision is an IEEE float32
comparison on both sides, the events and states still match the oracle
bit for bit.

An infinite log-intensity difference has no crossing count in Eq. 4 (the
oracle raises on it); the library bounds the crossings of one
pixel-substep by its documented EVIS_MAX_CROSSINGS, so the oracle is run
with that bound as its count_limit here, and only here and in the test of
that bound."""
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


def poisoned_pair(seed):
    rng = np.random.default_rng(seed)
    H, W = 48, 64
    p = U.oracle_pair(U.blob_scene(H, W, seed, flow="rotate", omega=10.0))
    L_A, L_B = p.L_A.copy(), p.L_B.copy()
    m_A, m_B = p.m_A.copy(), p.m_B.copy()
    for arr in (L_A, L_B):
        arr[rng.random((H, W)) < 0.02] = np.nan
    L_B[5, 7] = np.inf                                   # 65535 crossings per substep there
    L_A[20, 30] = -np.inf
    for arr in (m_A, m_B):
        arr[rng.random((H, W)) < 0.02, 0] = np.nan
        arr[rng.random((H, W)) < 0.01, 1] = np.inf
        arr[rng.random((H, W)) < 0.01, 0] = -np.inf
    return o.Pair(L_A, L_B, m_A, m_B, p.Z_A, p.Z_B, 0, 16667)


@pytest.mark.parametrize("warp", [o.WARP_GATHER, o.WARP_SPLAT, o.WARP_JOINT])
def test_step_nonfinite_inputs(torch, ctx, warp):
    from paper_2607_08098_amd import evis
    pair = poisoned_pair(61)
    nz = o.Noise(leak_rate_hz=20.0, shot_rate_hz=40.0, hot_rate_hz=300.0, hot_fraction=0.02,
                 shot_L0=-4.0, shot_inv_range=0.1, seed=3, pair_index=1)
    s = o.Sensor(C_on=0.2, C_off=0.2, K=3, blend_mode=warp, noise=nz)
    L_ref = np.where(np.isfinite(pair.L_A), pair.L_A, F32(0)).astype(F32)
    want, R, _, _ = o.step(pair, s, L_ref.copy(), count_limit=evis.EVIS_MAX_CROSSINGS)
    d = U.device_pair(pair, torch)
    d.update(C_on=0.2, C_off=0.2, refractory_us=0, K=3, K_max=64, blend_mode=warp, env_id=2,
             noise=dataclasses.asdict(nz))
    d["L_ref"] = torch.from_numpy(L_ref.copy()).cuda()
    d["t_last"] = None
    out, n = evis.event_buffer(1 << 22)
    say("step_batch non-finite inputs, warp", hex(warp), "oracle events", len(want))
    evis.evis_step_batch(ctx, [d], out, n, None)
    torch.cuda.synchronize()
    ev = evis.decode_events(out, n)
    want[:, 4] = 2
    assert int(n.item()) == len(want)
    assert U.same_multiset(ev, want), U.multiset_diff(ev, want)
    got_R = d["L_ref"].cpu().numpy()
    assert np.array_equal(got_R.view(np.uint32), R.view(np.uint32))

"""evis_step_batch_noalloc, the fused step for callers that cannot allocate:
through the C ABI, against evis_step_batch on the same inputs (the same
event multiset, substep counts, reference levels and last-event times,
bit for bit), on two calls in a row, the second with a smaller batch; a
batch beyond the static scratch is refused with nothing enqueued; and the
call takes no device memory where evis_step_batch grows its scratch."""
import numpy as np
import pytest

import gpu_util as U

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_2607_08098_amd import evis
    c = evis.Context(0)
    evis.evis_set_tuning(c, tile_w=32, tile_h=16)
    yield c
    c.close()


def say(*a):
    print("[case]", *a, flush=True)


def make_envs(torch, specs):
    """Env dicts from (H, W, seed, extra) specs; extra: 'refractory' adds
    per-pixel thresholds and a 50 us refractory period."""
    from paper_2607_08098_amd import scenes
    envs = []
    for e, (H, W, seed, extra) in enumerate(specs):
        pair = U.oracle_pair(U.blob_scene(H, W, seed, flow="rotate", omega=8.0 + e))
        d = U.device_pair(pair, torch)
        d.update(C_on=0.2, C_off=0.2, K=0, K_max=64, refractory_us=0, env_id=e)
        d["L_ref"] = torch.from_numpy(pair.L_A.copy()).cuda()
        if extra == "refractory":
            on, off = scenes.mismatch_thresholds(H, W, 0.2, 0.03, 0.01, scenes.rng_for(seed + 1))
            d.update(theta_on=torch.from_numpy(on).cuda(), theta_off=torch.from_numpy(off).cuda(),
                     refractory_us=50,
                     t_last=torch.full((H, W), -(2 ** 30), dtype=torch.int32, device="cuda"))
        envs.append(d)
    return envs


def clone_state(torch, envs):
    out = []
    for d in envs:
        c = dict(d)
        c["L_ref"] = d["L_ref"].clone()
        if "t_last" in d:
            c["t_last"] = d["t_last"].clone()
        out.append(c)
    return out


def sorted_keys(torch, out, n):
    cnt = min(int(n.item()), out.shape[0])
    rec = out[:cnt].long()
    word = rec[:, 0] & 0xFFFFFFFF
    return torch.sort((word << 31) | rec[:, 1])[0]


def run_both(torch, ctx, specs):
    from paper_2607_08098_amd import evis
    a = make_envs(torch, specs)
    b = clone_state(torch, a)
    out_a, n_a = evis.event_buffer(1 << 22)
    out_b, n_b = evis.event_buffer(1 << 22)
    K_a = torch.zeros(len(a), dtype=torch.int32, device="cuda")
    K_b = torch.zeros(len(b), dtype=torch.int32, device="cuda")
    evis.evis_step_batch(ctx, a, out_a, n_a, K_a)
    evis.evis_step_batch_noalloc(ctx, b, out_b, n_b, K_b)
    torch.cuda.synchronize()
    assert 0 < int(n_a.item()) <= out_a.shape[0]
    assert int(n_a.item()) == int(n_b.item())
    assert torch.equal(K_a, K_b)
    assert torch.equal(sorted_keys(torch, out_a, n_a), sorted_keys(torch, out_b, n_b))
    for da, db in zip(a, b):
        assert torch.equal(da["L_ref"].view(torch.int32), db["L_ref"].view(torch.int32))
        if "t_last" in da:
            assert torch.equal(da["t_last"], db["t_last"])
    return int(n_a.item())


def test_noalloc_matches_step_batch_on_two_calls(torch, ctx):
    # first call: several sizes, ragged tiles, one env with mismatch and a
    # refractory period; second call: a smaller batch on the same scratch
    first = [(130, 170, 501, None), (96, 128, 502, "refractory"), (260, 346, 503, None),
             (47, 61, 504, None)]
    second = [(64, 80, 505, None), (33, 40, 506, "refractory")]
    say("noalloc: first call", [s[:2] for s in first])
    n1 = run_both(torch, ctx, first)
    say("noalloc: second call", [s[:2] for s in second], "after", n1, "events")
    run_both(torch, ctx, second)


def test_noalloc_refuses_a_batch_beyond_its_scratch(torch, ctx):
    from paper_2607_08098_amd import evis
    H, W = 720, 1280
    z = torch.zeros((H, W), dtype=torch.float32, device="cuda")
    one = torch.ones((H, W), dtype=torch.float32, device="cuda")
    m = torch.zeros((H, W, 2), dtype=torch.float32, device="cuda")
    envs = [dict(L_A=z, L_B=z, m_A=m, m_B=m, Z_A=one, Z_B=one, L_ref=z.clone(), K=0, K_max=64,
                 env_id=e) for e in range(5)]      # 4.6 M pixels: ~78 MB of scratch
    out, n = evis.event_buffer(1 << 16)
    n.fill_(7)
    with pytest.raises(evis.EvisError) as ei:
        evis.evis_step_batch_noalloc(ctx, envs, out, n, None, 0)
    assert ei.value.code == evis.EVIS_ERR_UNSUPPORTED
    assert "scratch" in ctx.last_error()
    torch.cuda.synchronize()
    assert int(n.item()) == 7                      # nothing ran


def test_noalloc_takes_no_device_memory(torch):
    """On fresh contexts: evis_step_batch grows its scratch (the free device
    memory drops by about its size), evis_step_batch_noalloc does not."""
    from paper_2607_08098_amd import evis
    specs = [(480, 640, 511 + e, None) for e in range(3)]     # ~0.9 M px: ~16 MB of scratch
    a = make_envs(torch, specs)
    b = clone_state(torch, a)
    out, n = evis.event_buffer(1 << 22)
    warm = evis.Context(0)                         # kernels loaded before measuring
    evis.evis_set_tuning(warm, tile_w=32, tile_h=16)
    evis.evis_step_batch_noalloc(warm, clone_state(torch, a), out, n, None)
    torch.cuda.synchronize()
    warm.close()

    def free_drop(fn):
        torch.cuda.synchronize()
        before = torch.cuda.mem_get_info()[0]
        fn()
        torch.cuda.synchronize()
        return before - torch.cuda.mem_get_info()[0]

    c1 = evis.Context(0)
    evis.evis_set_tuning(c1, tile_w=32, tile_h=16, use_graph=0)
    drop_plain = free_drop(lambda: evis.evis_step_batch(c1, a, out, n, None))
    c2 = evis.Context(0)
    evis.evis_set_tuning(c2, tile_w=32, tile_h=16)
    drop_noalloc = free_drop(lambda: evis.evis_step_batch_noalloc(c2, b, out, n, None))
    say("free device memory taken: step_batch", drop_plain, "noalloc", drop_noalloc)
    assert drop_plain >= 12 << 20
    assert drop_noalloc < 2 << 20
    c1.close()
    c2.close()

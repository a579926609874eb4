"""Host-detected errors of the C ABI: a negative status, a message in
evis_last_error, and nothing enqueued (the outputs and the state keep their
contents).  Device-detected capacity overflow is covered by the parity tests."""
import numpy as np
import pytest

from oracle import evis_oracle as o
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
    yield c
    c.close()


def env(torch, H=24, W=32, **kw):
    pair = U.oracle_pair(U.blob_scene(H, W, 71, flow="rotate", omega=6.0))
    d = U.device_pair(pair, torch)
    d.update(C_on=0.2, C_off=0.2, refractory_us=0, K=0, K_max=64, blend_mode=0, env_id=1)
    d["L_ref"] = torch.from_numpy(pair.L_A.copy()).cuda()
    d.update(kw)
    return d


def expect_error(ctx, code, fn, text):
    from paper_2607_08098_amd import evis
    with pytest.raises(evis.EvisError) as ei:
        fn()
    assert ei.value.code == code, (ei.value.code, str(ei.value))
    assert text in ctx.last_error(), ctx.last_error()


def test_step_batch_rejects_bad_envs_and_enqueues_nothing(torch, ctx):
    from paper_2607_08098_amd import evis
    out, n = evis.event_buffer(1 << 16)
    n.fill_(123)
    cases = [
        (dict(C_on=0.0), evis.EVIS_ERR_INVALID, "thresholds"),
        (dict(C_off=float("nan")), evis.EVIS_ERR_INVALID, "thresholds"),
        (dict(K_max=129), evis.EVIS_ERR_INVALID, "K_max"),
        (dict(K=200), evis.EVIS_ERR_UNSUPPORTED, "K > 128"),
        (dict(blend_mode=7), evis.EVIS_ERR_INVALID, "blend_mode"),
        (dict(refractory_us=100), evis.EVIS_ERR_INVALID, "t_last"),
        (dict(env_id=512), evis.EVIS_ERR_INVALID, "env_id"),
        (dict(t0=5, t1=5), evis.EVIS_ERR_INVALID, ""),
    ]
    good = env(torch)
    good_before = good["L_ref"].clone()
    for kw, code, text in cases:
        d = env(torch, **kw)
        before = d["L_ref"].clone()
        # the bad env second: the good one before it must not run either
        expect_error(ctx, code, lambda: evis.evis_step_batch(ctx, [good, d], out, n, None, 0), text)
        torch.cuda.synchronize()
        assert int(n.item()) == 123                     # nothing ran
        assert torch.equal(d["L_ref"], before)
        assert torch.equal(good["L_ref"], good_before)
    # too many envs
    d = env(torch)
    expect_error(ctx, evis.EVIS_ERR_UNSUPPORTED,
                 lambda: evis.evis_step_batch(ctx, [d] * 513, out, n, None, 0), "512")
    # a frame too large for the 11-bit coordinates
    big = env(torch)
    big_L = torch.zeros((2048, 4), dtype=torch.float32, device="cuda")
    for k in ("L_A", "L_B", "Z_A", "Z_B", "L_ref"):
        big[k] = big_L if k != "Z_A" and k != "Z_B" else big_L + 1.0
    big["m_A"] = torch.zeros((2048, 4, 2), dtype=torch.float32, device="cuda")
    big["m_B"] = big["m_A"]
    expect_error(ctx, evis.EVIS_ERR_UNSUPPORTED,
                 lambda: evis.evis_step_batch(ctx, [big], out, n, None, 0), "2047")
    torch.cuda.synchronize()
    assert int(n.item()) == 123


def test_other_entry_points_reject_bad_arguments(torch, ctx):
    from paper_2607_08098_amd import evis
    d = env(torch)
    L = torch.empty((3, 24, 32), dtype=torch.float32, device="cuda")
    expect_error(ctx, evis.EVIS_ERR_INVALID,
                 lambda: evis.evis_interpolate(ctx, d, 4, 3, 2, 0, L_out=L, want_holes=False),
                 "j_begin")
    expect_error(ctx, evis.EVIS_ERR_UNSUPPORTED,
                 lambda: evis.evis_interpolate(ctx, d, 129, 0, 1, 0, L_out=L, want_holes=False),
                 "K > 128")
    expect_error(ctx, evis.EVIS_ERR_INVALID,
                 lambda: evis.evis_log_luminance(ctx, d["L_A"], 0.0, out=L[0]), "eps")
    K_out = torch.zeros(1, dtype=torch.int32, device="cuda")
    expect_error(ctx, evis.EVIS_ERR_INVALID,
                 lambda: evis.evis_substep_count(ctx, d, 0, K_out), "K_max")
    C = torch.tensor([0.2], device="cuda")
    S = torch.empty_like(d["L_A"])
    envs = evis.soft_env_array(d["L_A"][None], d["L_B"][None], d["m_A"][None], d["m_B"][None],
                               d["Z_A"][None], d["Z_B"][None], d["L_ref"][None], S=S[None])
    expect_error(ctx, evis.EVIS_ERR_INVALID,
                 lambda: evis.evis_soft_count_forward(ctx, envs, 8, 0.0, 0, C), "tau")
    gC = torch.empty_like(C)
    expect_error(ctx, evis.EVIS_ERR_INVALID,
                 lambda: evis.evis_soft_count_backward(ctx, envs, 8, 0.02, 0, C, gC, flags=4), "")
    # the context is still usable after errors
    out, n = evis.event_buffer(1 << 16)
    evis.evis_step_batch(ctx, [env(torch)], out, n)
    torch.cuda.synchronize()
    assert int(n.item()) > 0

"""Defocus (separable Gaussian on linear intensity) through the C ABI
against the float64 oracle.  Bar, per output pixel: the float32 kernel sums
2r + 1 taps per pass in order, so each output is within
(4 (2r + 1) + 4) 2^-24 M of the exact blur, M the largest |x| in that
pixel's own (2r + 1) x (2r + 1) window (edge pixels repeated, as the blur
does): each pass rounds once per product and per partial sum, every
partial sum of the horizontal pass at a row of the window is bounded by
the largest |x| of that row's segment and every partial sum of the
vertical pass by the largest horizontal result in the window, since the
weights are positive and sum to 1; the weights themselves are rounded to
float32.  A dark pixel next to bright ones is held to its own window, not
to the image's maximum."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import evis_oracle as o

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


def pixel_bound(x, r):
    """(4 (2r + 1) + 4) 2^-24 times the largest |x| in each pixel's
    (2r + 1) x (2r + 1) window, per channel."""
    a = np.abs(x.astype(np.float64))
    size = (2 * r + 1, 2 * r + 1) + ((1,) if x.ndim == 3 else ())
    return (4 * (2 * r + 1) + 4) * 2.0 ** -24 * ndimage.maximum_filter(a, size=size, mode="nearest")


def within_bound(got, want, x, r):
    err = np.abs(got - want)
    bound = pixel_bound(x, r)
    worst = np.unravel_index(np.argmax(err - bound), err.shape)
    return bool(np.all(err <= bound)), (worst, float(err[worst]), float(bound[worst]))


def check(torch, ctx, x, sigma):
    from paper_2607_08098_amd import evis
    xd = torch.from_numpy(x).cuda()
    got = evis.evis_defocus(ctx, xd, sigma).cpu().numpy().astype(np.float64)
    want = o.defocus(x.astype(np.float64), sigma)
    ok, info = within_bound(got, want, x, o.defocus_radius(sigma))
    assert ok, (sigma, x.shape, info)


@pytest.mark.parametrize("shape", [(100, 130), (1, 1), (17, 300), (70, 90, 3), (300, 5)])
@pytest.mark.parametrize("sigma", [0.1, 0.5, 1.7, 4.0, 10.0])
def test_defocus_matches_oracle(torch, ctx, shape, sigma):
    rng = np.random.default_rng(hash((shape, sigma)) % 2 ** 32)
    x = (10.0 ** rng.uniform(-3, 3, size=shape)).astype(F32)    # six decades
    say("defocus", shape, sigma)
    check(torch, ctx, x, sigma)


def test_defocus_full_frame(torch, ctx):
    from paper_2607_08098_amd import scenes
    sc = scenes.blob_pair(720, 1280, 7)
    say("defocus 1280x720 sigma 0.5")
    check(torch, ctx, sc["I_A"], 0.5)


def test_defocus_batch(torch, ctx):
    """70 images of uneven size in batched launches (64, then 6), grey
    and RGB, against the oracle one by one."""
    from paper_2607_08098_amd import evis
    rng = np.random.default_rng(5)
    for ch in (1, 3):
        xs, outs, pairs = [], [], []
        for i in range(70):
            H, W = int(rng.integers(1, 90)), int(rng.integers(1, 130))
            shape = (H, W) if ch == 1 else (H, W, 3)
            x = (10.0 ** rng.uniform(-2, 2, size=shape)).astype(F32)
            xd = torch.from_numpy(x).cuda()
            od = torch.empty_like(xd)
            xs.append(x)
            pairs.append((xd, od))
        say("defocus batch of 70, channels", ch)
        evis.evis_defocus_batch(ctx, pairs, 1.3)
        torch.cuda.synchronize()
        r = o.defocus_radius(1.3)
        for x, (_, od) in zip(xs, pairs):
            got = od.cpu().numpy().astype(np.float64)
            want = o.defocus(x.astype(np.float64), 1.3)
            ok, info = within_bound(got, want, x, r)
            assert ok, (x.shape, info)


@pytest.mark.parametrize("sigma", [0.5, 2.0])
def test_defocus_batch_full_frames(torch, ctx, sigma):
    """The benchmark's 64 images in one launch (24 x 346x260, 24 x 640x480,
    16 x 1280x720: 12256 tiles, dealt to the XCDs in runs of consecutive
    tiles that cross image boundaries; sigma 2 needs more than one round of
    apron loads per thread), every image against the oracle."""
    from paper_2607_08098_amd import evis
    rng = np.random.default_rng(11)
    shapes = [(260, 346)] * 24 + [(480, 640)] * 24 + [(720, 1280)] * 16
    xs = [(10.0 ** rng.uniform(-2, 2, size=s)).astype(F32) for s in shapes]
    pairs = [(torch.from_numpy(x).cuda(), None) for x in xs]
    pairs = [(xd, torch.empty_like(xd)) for xd, _ in pairs]
    say("defocus batch of 64 full frames, sigma", sigma)
    evis.evis_defocus_batch(ctx, pairs, sigma)
    torch.cuda.synchronize()
    r = o.defocus_radius(sigma)
    for x, (_, od) in zip(xs, pairs):
        got = od.cpu().numpy().astype(np.float64)
        want = o.defocus(x.astype(np.float64), sigma)
        ok, info = within_bound(got, want, x, r)
        assert ok, (x.shape, sigma, info)


def test_defocus_argument_errors(torch, ctx):
    from paper_2607_08098_amd import evis
    x = torch.ones(8, 9, device="cuda")
    for sigma in (0.0, -1.0, 10.5, float("nan")):
        with pytest.raises(evis.EvisError) as ei:
            evis.evis_defocus(ctx, x, sigma)
        assert ei.value.code == evis.EVIS_ERR_INVALID
    with pytest.raises(evis.EvisError) as ei:
        evis.evis_defocus(ctx, x, 1.0, out=x)
    assert ei.value.code == evis.EVIS_ERR_INVALID and "overlap" in str(ei.value)

"""The seeded input generators (CPU): determinism and internal consistency
of the synthetic scenes.  They hold no arithmetic of the event path."""
import numpy as np
from scipy import ndimage

from paper_2607_08098_amd import scenes


def test_plane_scene_flow_is_consistent():
    """Keyframe B sampled at p + m_B(p) reproduces A's log radiance almost
    everywhere (exact projection; misses only at occlusion boundaries), and
    m_A and m_B of a static scene point are opposite."""
    sc = scenes.PlaneScene(120, 160, 2000, 1, focal=125.0)
    pr = sc.pair(0)
    yy, xx = np.mgrid[0:120, 0:160]
    la = np.log(pr["I_A"].astype(np.float64) + 1e-3)
    lb = np.log(pr["I_B"].astype(np.float64) + 1e-3)
    a_at = ndimage.map_coordinates(la, [yy + pr["m_B"][..., 1], xx + pr["m_B"][..., 0]], order=1,
                                   mode="nearest")
    assert np.mean(np.abs(a_at - lb) < 0.1) > 0.9
    assert np.all(pr["Z_A"] > 0) and np.all(np.isfinite(pr["m_A"]))
    # six decades of irradiance across the planes
    assert np.log10(pr["I_A"].max() / pr["I_A"].min()) > 4


def test_generators_are_seeded():
    a = scenes.blob_pair(32, 40, 7, flow="rotate")
    b = scenes.blob_pair(32, 40, 7, flow="rotate")
    for k in ("I_A", "I_B", "m_A", "Z_A"):
        assert np.array_equal(a[k], b[k])
    p1, p2 = scenes.PlaneScene(30, 40, 5, 2, focal=40.0), scenes.PlaneScene(30, 40, 5, 2, focal=40.0)
    assert np.array_equal(p1.pair(1)["m_B"], p2.pair(1)["m_B"])
    d1 = scenes.disc_pair(26, 34, 11, step=3)
    d2 = scenes.disc_pair(26, 34, 11, step=3)
    assert np.array_equal(d1["I_B"], d2["I_B"])


def test_threaded_plane_keyframes_equal_sequential():
    """render_keyframes on several threads returns the frames of one-at-a-time
    rendering, bit for bit (multithreaded BLAS entered from several Python
    threads at once has not)."""
    sc = scenes.PlaneScene(480, 640, 2000, 40)   # full size: BLAS runs threaded
    ks = list(range(20, 36))
    ref = [sc.keyframe(k) for k in ks]
    for _ in range(2):
        got = scenes.render_keyframes(sc, ks, threads=16)
        for a, b in zip(ref, got):
            for x, y in zip(a, b):
                assert (x is None and y is None) or np.array_equal(x.view(np.uint32), y.view(np.uint32))

"""Shared helpers of the GPU tests: seeded scenes as oracle pairs and as
device tensors, event-multiset comparison.  No arithmetic of the method."""
from __future__ import annotations

import numpy as np

from oracle import evis_oracle as o
from paper_2607_08098_amd import scenes

F32 = np.float32


def log_frames(scene: dict):
    """Log intensity of both keyframes (the oracle's float64 log intensity, stored as
    float32): the common input of both sides."""
    return (o.log_luminance(scene["I_A"]).astype(F32), o.log_luminance(scene["I_B"]).astype(F32))


def oracle_pair(scene: dict, t0=0, t1=16667) -> o.Pair:
    L_A, L_B = log_frames(scene)
    return o.Pair(L_A, L_B, scene["m_A"], scene["m_B"], scene["Z_A"], scene["Z_B"], t0, t1)


def device_pair(pair: o.Pair, torch, device="cuda") -> dict:
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return dict(L_A=t(pair.L_A), L_B=t(pair.L_B), m_A=t(pair.m_A), m_B=t(pair.m_B),
                Z_A=t(pair.Z_A), Z_B=t(pair.Z_B), t0=pair.t0_us, t1=pair.t1_us)


def blob_scene(H, W, seed, **kw):
    return scenes.blob_pair(H, W, seed, **kw)


def same_multiset(a: np.ndarray, b: np.ndarray) -> bool:
    a = o.canonical(a)
    b = o.canonical(b)
    return a.shape == b.shape and np.array_equal(a, b)


def multiset_diff(a: np.ndarray, b: np.ndarray, limit=10):
    from collections import Counter
    ca = Counter(map(tuple, np.asarray(a).tolist()))
    cb = Counter(map(tuple, np.asarray(b).tolist()))
    only_a = list((ca - cb).elements())[:limit]
    only_b = list((cb - ca).elements())[:limit]
    return only_a, only_b

"""Full-size parity cases and their expected digests.  TEST INFRASTRUCTURE.

The GPU tests run these cases at the benchmark's full sizes and compare
every env's event multiset and state with digests that the CPU oracle
alone computed from the same seeded scenes:

  python tests/golden/fullsize.py [--jobs N] [mixed64 disc512 planes640]

writes ``fullsize_digests.json`` next to this file.  Nothing here runs the
HIP library or reads anything it wrote: the inputs come from
``paper_2607_08098_amd.scenes`` (the seeded generator, which holds none of
the method's arithmetic), log intensity from the oracle's float64 a1
rounded to float32, and the expected values from ``oracle.evis_oracle``.

Cases:
  mixed64    the benchmark's 64 envs (24 x 346x260, 24 x 640x480,
             16 x 1280x720 rotating blob sequences, seeds 3000 + e), adaptive
             K <= 64, C = 0.2, keyframes 0..MIXED_STEPS chained through the
             state: every env at every step.
  disc512    512 rotating discs at 346x260 (seeds 4000 + e), adaptive
             K <= 128, C = 0.2, 200 keyframe pairs chained: DISC_ENVS (32
             envs spread over the batch) at every step.
  planes640  the textured-plane scene at 640x480 with per-pixel threshold
             mismatch (Eq. 8, C 0.25, sigma 0.03) and a 100 us refractory
             period, 100 keyframe pairs chained: every pair.

Digests: an env's events are packed into one int64 key per event,
t << 23 | y << 12 | x << 1 | p, sorted (the multiset in a fixed order) and
hashed with SHA-256 as little-endian bytes; a float32 state plane is
hashed as its little-endian bytes.  Hashes are kept to 16 hex digits.
A chained digest folds a step's event and state hashes into the previous
step's: d_s = sha256(d_{s-1} | events_s | state_s).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DIGEST_FILE = os.path.join(HERE, "fullsize_digests.json")
F32 = np.float32

MIXED_SEED_BASE = 3000
MIXED_STEPS = 3
MIXED_SENSOR = dict(C_on=0.2, C_off=0.2, K=0, K_max=64, refractory_us=0)

DISC_N, DISC_H, DISC_W, DISC_SEED_BASE, DISC_STEPS = 512, 260, 346, 4000, 200
# 32 envs spread over the batch: one in each run of 16 consecutive envs,
# at a different offset in each run (ranks, queue bands and XCDs differ)
DISC_ENVS = [16 * i + (7 * i) % 16 for i in range(32)]
DISC_CHECKPOINTS = sorted(set(list(range(9, DISC_STEPS, 10)) + [0, DISC_STEPS - 1]))
DISC_SENSOR = dict(C_on=0.2, C_off=0.2, K=0, K_max=128, refractory_us=0)

PLANES_H, PLANES_W, PLANES_SEED, PLANES_PAIRS, PLANES_ENV = 480, 640, 2000, 100, 9
PLANES_THETA = dict(C=0.25, sigma=0.03, theta_min=0.01, seed=2001)
PLANES_SENSOR = dict(K=0, K_max=64, refractory_us=100)


def h16(b: bytes) -> str:
    return hashlib.sha256(b).hexdigest()[:16]


def event_keys(ev: np.ndarray) -> np.ndarray:
    """[N, 5] (x, y, t, p, env) events of one env -> sorted int64 keys."""
    ev = np.asarray(ev, np.int64).reshape(-1, 5)
    k = (ev[:, 2] << 23) | (ev[:, 1] << 12) | (ev[:, 0] << 1) | ev[:, 3]
    return np.sort(k)


def keys_digest(sorted_keys: np.ndarray) -> str:
    return h16(np.ascontiguousarray(sorted_keys, dtype="<i8").tobytes())


def plane_digest(a: np.ndarray) -> str:
    return h16(np.ascontiguousarray(a).astype(a.dtype.newbyteorder("<")).tobytes())


def chain(prev: str, ev_digest: str, state_digest: str) -> str:
    return h16(f"{prev}|{ev_digest}|{state_digest}".encode())


def log_intensity(I: np.ndarray) -> np.ndarray:
    """The common input of both sides: the oracle's float64 a1, as float32."""
    from oracle import evis_oracle as o
    return o.log_luminance(I).astype(F32)


# ---------------------------------------------------------------------------
# case inputs (generator calls only)
# ---------------------------------------------------------------------------

def mixed_specs():
    from paper_2607_08098_amd import scenes
    return scenes.mixed_batch_specs(MIXED_SEED_BASE)


def disc_keyframe(e: int, i: int):
    """(radiance, backward motion, depth) of disc env e at keyframe i."""
    from paper_2607_08098_amd import scenes
    p = scenes.disc_scene_params(DISC_H, DISC_W, DISC_SEED_BASE + e)
    return scenes.disc_frame(DISC_H, DISC_W, p, i / 60.0)


def planes_thresholds():
    from paper_2607_08098_amd import scenes
    t = PLANES_THETA
    return scenes.mismatch_thresholds(PLANES_H, PLANES_W, t["C"], t["sigma"], t["theta_min"],
                                      scenes.rng_for(t["seed"]))


# ---------------------------------------------------------------------------
# oracle runs (one task each)
# ---------------------------------------------------------------------------

def _mixed_task(e: int):
    from oracle import evis_oracle as o
    from paper_2607_08098_amd import scenes
    H, W, seed = mixed_specs()[e]
    seq = scenes.RotatingSequence(H, W, seed)
    kf = [seq.keyframe(i) for i in range(MIXED_STEPS + 1)]
    L = [log_intensity(k[0]) for k in kf]
    R = L[0].copy()
    sensor = o.Sensor(**MIXED_SENSOR)
    steps = []
    for s in range(MIXED_STEPS):
        pair = o.Pair(L[s], L[s + 1], kf[s][1], kf[s + 1][1], kf[s][2], kf[s + 1][2],
                      scenes.frame_time_us(s), scenes.frame_time_us(s + 1))
        ev, R, _, K = o.step(pair, sensor, R, None, e)
        steps.append(dict(K=int(K), n=int(len(ev)), events=keys_digest(event_keys(ev)),
                          L_ref=plane_digest(R)))
    return "mixed64", e, dict(env=e, H=H, W=W, seed=seed, steps=steps)


def _disc_task(e: int):
    from oracle import evis_oracle as o
    from paper_2607_08098_amd import scenes
    sensor = o.Sensor(**DISC_SENSOR)
    I0, m, Z = disc_keyframe(e, 0)
    LA = log_intensity(I0)
    R = LA.copy()
    d, counts, marks, Ks = "", [], {}, set()
    for s in range(DISC_STEPS):
        IB, _, _ = disc_keyframe(e, s + 1)
        LB = log_intensity(IB)
        pair = o.Pair(LA, LB, m, m, Z, Z, scenes.frame_time_us(s), scenes.frame_time_us(s + 1))
        ev, R, _, K = o.step(pair, sensor, R, None, e)
        Ks.add(int(K))
        counts.append(int(len(ev)))
        d = chain(d, keys_digest(event_keys(ev)), plane_digest(R))
        if s in DISC_CHECKPOINTS:
            marks[str(s)] = d
        LA = LB
    return "disc512", e, dict(env=e, K=sorted(Ks), n=counts, chained=marks)


def _planes_task(_):
    from oracle import evis_oracle as o
    from paper_2607_08098_amd import scenes
    sc = scenes.PlaneScene(PLANES_H, PLANES_W, PLANES_SEED, PLANES_PAIRS)
    on, off = planes_thresholds()
    sensor = o.Sensor(theta_on=on, theta_off=off, **PLANES_SENSOR)
    I, m_next, _, Z = sc.keyframe(0)
    LA = log_intensity(I)
    R = LA.copy()
    tl = np.full((PLANES_H, PLANES_W), o.T_LAST_INIT, np.int32)
    pairs = []
    for k in range(PLANES_PAIRS):
        IB, m_next_B, m_prev_B, ZB = sc.keyframe(k + 1)
        LB = log_intensity(IB)
        pair = o.Pair(LA, LB, m_next, m_prev_B, Z, ZB, scenes.frame_time_us(k),
                      scenes.frame_time_us(k + 1))
        ev, R, tl, K = o.step(pair, sensor, R, tl, PLANES_ENV)
        pairs.append(dict(K=int(K), n=int(len(ev)), events=keys_digest(event_keys(ev)),
                          L_ref=plane_digest(R), t_last=plane_digest(tl)))
        LA, m_next, Z = LB, m_next_B, ZB
    return "planes640", 0, dict(H=PLANES_H, W=PLANES_W, pairs=pairs)


def _run(task):
    fn, arg = task
    t = time.time()
    out = fn(arg)
    print(f"[digests] {out[0]} {out[1]} done in {time.time() - t:.1f}s", flush=True)
    return out


def main(argv):
    import argparse
    import multiprocessing as mp
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*", default=["mixed64", "disc512", "planes640"])
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args(argv)
    tasks = []
    if "planes640" in args.cases:
        tasks.append((_planes_task, 0))
    if "disc512" in args.cases:
        tasks += [(_disc_task, e) for e in DISC_ENVS]
    if "mixed64" in args.cases:
        specs = mixed_specs()
        order = sorted(range(len(specs)), key=lambda e: -specs[e][0] * specs[e][1])
        tasks += [(_mixed_task, e) for e in order]
    old = {}
    if os.path.exists(DIGEST_FILE):
        with open(DIGEST_FILE) as fh:
            old = json.load(fh)
    res = {}
    left = {}
    for fn, _ in tasks:
        case = {_mixed_task: "mixed64", _disc_task: "disc512", _planes_task: "planes640"}[fn]
        left[case] = left.get(case, 0) + 1
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    out = dict(old)
    with mp.get_context("fork").Pool(args.jobs) as pool:
        for case, key, rec in pool.imap_unordered(_run, tasks):
            res.setdefault(case, {})[key] = rec
            left[case] -= 1
            if left[case] == 0:     # a case is complete: write it out now
                _store(out, case, res[case])
    print(f"[digests] wrote {DIGEST_FILE}")


def _store(out, case, recs):
    if case == "mixed64":
        out["mixed64"] = dict(seed_base=MIXED_SEED_BASE, steps=MIXED_STEPS, sensor=MIXED_SENSOR,
                              envs=[recs[e] for e in sorted(recs)])
    elif case == "disc512":
        out["disc512"] = dict(n_envs=DISC_N, H=DISC_H, W=DISC_W, seed_base=DISC_SEED_BASE,
                              steps=DISC_STEPS, sensor=DISC_SENSOR, checkpoints=DISC_CHECKPOINTS,
                              envs=[recs[e] for e in sorted(recs)])
    else:
        out["planes640"] = dict(recs[0], seed=PLANES_SEED, env=PLANES_ENV, sensor=PLANES_SENSOR,
                                thresholds=PLANES_THETA)
    with open(DIGEST_FILE, "w") as fh:
        json.dump(out, fh, indent=0, sort_keys=True)
        fh.write("\n")
    print(f"[digests] {case} written", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])

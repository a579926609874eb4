#!/usr/bin/env python3
"""Throughput of the fused event path on one MI355X.

Workload: 64 environments of mixed resolution in one batch (24 x 346x260,
24 x 640x480, 16 x 1280x720), each a rotating blob scene (omega U[0.5, 20]
rad/s at 60 Hz, N(0, 0.3) px flow noise, depth U[0.5, 5] m), adaptive K
(at most 64), C_on = C_off = 0.2.  Inputs are synthetic and resident in HBM
before timing.  One step = the whole path for one keyframe pair of every
env: log luminance of the new keyframe (one launch over all envs) and the
fused, graph-replayed substep count + warp + emit launch, events appended
to one device stream.

Printed: one JSON line.  value = Mpix-substeps/s (sum over envs of H*W*K
per step / step time); events/s beside it; the per-env-launch plain form
(interpolate every sub-frame to HBM, then emit, env by env) and the per-env
fused form on the same GPU; the roofline of the fused tile kernel, timed
live with HIP events; the same kernel with B splatted backward (the
two-splat warps: own z-buffer with B primary, and one joint z-buffer) and
with sensor noise (leak 0.1 Hz, shot 1 Hz, 0.1% hot pixels at 100 Hz);
the defocus blur of every env's keyframe (sigma 0.5 px); the 128-bin
voxel grid of one 1280x720 env from one step's event stream; the
HBM-bound forms (the event model over one env's materialised frames, the
fused step with every motion vector scaled to at most 1.9 px, so K <= 2);
the CPU oracle on a bounded sample of the same workload (rank 0, N = 1
only).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work of the fused path, per pixel and keyframe pair, from the
# operation counts of the method's formulas (splat ~14, resolve ~2, bilinear
# gather ~21, blend ~5, emission ~4 lane-ops per interior substep; emission
# alone at j = K) and its compulsory traffic (6 input planes, 32 B, plus the
# reference level read and written, 8 B) plus 8 B per event.
OPS_INTERIOR = 46
OPS_LAST = 4
# The two-splat warps: B splatted backward instead of gathered: two splats
# (~14 each), two resolves (~2 each), blend ~5 and emission ~4.
OPS_INTERIOR_TWO_SPLAT = 41
# Sensor noise adds one Philox4x32-10 draw per pixel-substep (10 rounds of
# two 32-bit high and low products, four xors and the key update, 98
# lane-ops) and ~10 for the three decisions.
OPS_NOISE = 108
BYTES_PER_PX = 40
BYTES_PER_EVENT = 8
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12      # plain VALU lane-ops: 39.3 T/s
HBM_PEAK_GBS = 8000.0

KERNEL_SOURCES = ["evis_common.h", "evis_internal.h", "evis_sink.h", "evis_warp.h", "evis_tile_kernel.h",
                  "evis_tile.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_tile_step_mixed64.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2607_08098_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile", type=str, default=None, help="WxH, skips the autotuner")
    ap.add_argument("--tuning-cache", type=str, default=os.path.join(ROOT, "tuning_cache.jsonl"),
                    help="the autotuner's cache file (empty string: no cache)")
    ap.add_argument("--quick", action="store_true", help="timed loop only (for profilers)")
    ap.add_argument("--variants", action="store_true",
                    help="timed loop and the variants only (for profilers)")
    ap.add_argument("--only", type=str, default=None,
                    choices=("generate_events", "events_batch", "small_motion", "defocus", "voxel",
                             "disc512"),
                    help="timed loop and this one variant only (for profilers): the event model "
                         "over one env's or every env's materialised samples, the small-motion "
                         "fused step, the batched defocus or the voxel grid; disc512: the "
                         "512-disc batch alone (--disc-steps pairs)")
    ap.add_argument("--warp-steps", type=int, default=10,
                    help="timed steps of each variant: two-splat warps, noise (0 skips them)")
    ap.add_argument("--disc-steps", type=int, default=200,
                    help="steps of the 512-disc sustained run reported beside the metric (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB three times (the reference kernel for HBM counters)")
    ap.add_argument("--traffic-from", type=str, default=None, metavar="DIR",
                    help="summarise rocprofv3 FETCH_SIZE / WRITE_SIZE runs in DIR/{fetch,write,"
                         "cal_fetch,cal_write} into the traffic record (no GPU)")
    ap.add_argument("--tile-label", type=str, default=None, help="WxH the counter runs used")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


COPY_BYTES = 1 << 30


def copy_calibration():
    """Three copies of 1 GiB: per dispatch the algorithmic traffic is
    exactly 1 GiB read and 1 GiB written, which calibrates the counters."""
    import torch
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_calibration_bytes=COPY_BYTES, dispatches=3)))


def _counter_means(run_dir, counter):
    """{kernel name: mean counter value per dispatch} from a rocprofv3 csv run."""
    import csv
    import glob
    tot, disp = {}, {}
    for f in glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                k = r["Kernel_Name"]
                tot[k] = tot.get(k, 0.0) + float(r["Counter_Value"])
                disp.setdefault(k, set()).add(r["Dispatch_Id"])
    return {k: tot[k] / len(disp[k]) for k in tot}


def traffic_from(d, tile_label):
    """HBM traffic of the fused tile kernel per launch, from rocprofv3 runs in
    DIR/{rd,write,cal_rd,cal_write}: reads as 32, 64 and 128 bytes times the
    L2-to-memory read requests of each size (TCC_EA0_RDREQ_{32B,64B,128B}),
    writes from WRITE_SIZE; the copy of exactly 1 GiB checks both (FETCH_SIZE
    is not used: its gfx950 formula takes 128-byte reads from TCC_BUBBLE, and
    counts this part's 128-byte reads as 64 bytes, half of a copy's)."""
    def pick(means, key):
        ks = [k for k in means if key(k)]
        assert ks, f"no dispatch matched in {sorted(means)[:8]}"
        ks.sort(key=lambda k: -means[k])
        return ks[0], means[ks[0]]
    is_tile = lambda k: "k_tile<" in k
    is_copy = lambda k: "copy" in k.lower() or "elementwise" in k

    def read_bytes(sub, key):
        n = {c: pick(_counter_means(os.path.join(d, sub), c), key) for c in
             ("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum")}
        kern = n["TCC_EA0_RDREQ_128B_sum"][0]
        return kern, (32 * n["TCC_EA0_RDREQ_32B_sum"][1] + 64 * n["TCC_EA0_RDREQ_64B_sum"][1]
                      + 128 * n["TCC_EA0_RDREQ_128B_sum"][1])

    kf, rb = read_bytes("rd", is_tile)
    _, crb = read_bytes("cal_rd", is_copy)
    kw, write = pick(_counter_means(os.path.join(d, "write"), "WRITE_SIZE"), is_tile)
    _, cw = pick(_counter_means(os.path.join(d, "cal_write"), "WRITE_SIZE"), is_copy)
    wb = write * 1024.0
    tw, th = (int(v) for v in tile_label.lower().split("x"))
    rec = dict(kernel=kf, kernel_hash=kernel_hash(), tuning=[tw, th], workload="mixed64_sequence",
               read_bytes=round(rb), write_bytes=round(wb), bytes_per_launch=round(rb + wb),
               copy_read_bytes=round(crb), copy_write_bytes=round(cw * 1024.0),
               copy_bytes=COPY_BYTES)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec))


def disc_sustained(ctx, steps):
    """512 rotating-disc envs at 346x260 (adaptive K <= 128, static background),
    `steps` consecutive keyframe pairs with the state kept on the device; each
    step's radiance is generated on the device before the step and only the
    fused step is timed (HIP events on the stream)."""
    import numpy as np
    import torch
    from paper_2607_08098_amd import evis, workloads
    t = time.time()
    batch = workloads.DiscBatch(ctx, n_envs=512, H=260, W=346, seed_base=4000)
    batch.start(0)
    sensor = dict(C_on=0.2, C_off=0.2, K=0, K_max=128, refractory_us=0)
    out, n = evis.event_buffer(1 << 26)
    K_used = torch.zeros(512, dtype=torch.int32, device="cuda")
    tuning = evis.evis_get_tuning(ctx).as_dict()
    log(f"disc512 ready in {time.time() - t:.1f}s")
    ms, events, work, overflow = 0.0, 0, 0.0, False
    px = 260 * 346
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for step in range(steps + 1):
        if step > 0:
            batch.advance()
        t0, t1 = batch.times()
        arr = evis.env_array(batch.env_dicts(sensor, t0, t1))
        e0.record()
        evis.evis_step_batch(ctx, arr, out, n, K_used, evis.EVIS_FLAG_RESET_CURSOR)
        e1.record()
        torch.cuda.synchronize()
        if step == 0:
            continue   # the first step also captures the graph
        ms += e0.elapsed_time(e1)
        cnt = int(n.item())
        overflow |= cnt > out.shape[0]
        events += cnt
        work += float(K_used.cpu().numpy().astype(np.int64).sum()) * px
        if step % 50 == 0:
            log(f"disc512 step {step}: {cnt} events")
    return dict(steps=steps, ms_per_step=round(ms / steps, 4),
                mpix_substeps_per_s=round(work / 1e6 / (ms / 1e3), 1),
                events_per_s=round(events / (ms / 1e3), 1), overflow=overflow, tuning=tuning)


def _oracle_pair_task(task):
    """The oracle on keyframes 0 -> 1 of one env of the sequence: (pixel-
    substeps, seconds in the oracle's step, name)."""
    e, H, W, seed = task
    import numpy as np
    from oracle import evis_oracle as o
    from paper_2607_08098_amd import scenes
    seq = scenes.RotatingSequence(H, W, seed)
    (I0, m0, Z0), (I1, m1, Z1) = seq.keyframe(0), seq.keyframe(1)
    L0 = o.log_luminance(I0).astype(np.float32)
    L1 = o.log_luminance(I1).astype(np.float32)
    pair = o.Pair(L0, L1, m0, m1, Z0, Z1, scenes.frame_time_us(0), scenes.frame_time_us(1))
    t0 = time.perf_counter()
    _, _, _, K = o.step(pair, o.Sensor(C_on=0.2, C_off=0.2, K=0, K_max=64), L0.copy(), None, e)
    return H * W * K, time.perf_counter() - t0, f"env{e}:{W}x{H},K={K}"


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(specs):
    """The CPU oracle, as it stands, on a bounded sample of the workload
    (keyframes 0 -> 1 of some envs): one process per env on every core this
    process may use (at most 16), and one env after another on one core.
    Runs before anything touches the GPU (the pool forks)."""
    import multiprocessing as mp
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    small = [e for e, (H, W, _) in enumerate(specs) if H * W <= 640 * 480]
    # one env per core, half of each of the two smaller classes
    par = [e for e in small if specs[e][0] == 260][: (cores + 1) // 2]
    par += [e for e in small if specs[e][0] == 480][: cores - len(par)]
    tasks = [(e,) + tuple(specs[e]) for e in par]
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_pair_task, tasks, chunksize=1)
    wall = time.perf_counter() - t0
    work = float(sum(r[0] for r in res))
    single = [_oracle_pair_task((e,) + tuple(specs[e])) for e in (0, 24)]
    s_work = float(sum(r[0] for r in single))
    s_secs = sum(r[1] for r in single)
    model = cpu_model()
    return dict(value=round(work / 1e6 / wall, 3), unit="Mpix-substeps/s", cores=cores, kind="oracle",
                cpu_model=model,
                sample=f"keyframes 0->1 of {len(tasks)} envs ({', '.join(r[2] for r in res)}), "
                       f"one process per env on {cores} cores of {model}, {wall:.1f}s wall; "
                       f"pixel-substeps over wall time",
                single_core=dict(value=round(s_work / 1e6 / s_secs, 3), cores=1,
                                 sample=f"keyframes 0->1 of {', '.join(r[2] for r in single)}, "
                                        f"{s_secs:.1f}s in the oracle's step"))


def main():
    args = parse()
    if args.only:
        args.variants = True
    want = lambda name: args.only is None or args.only == name
    if args.traffic_from:
        traffic_from(args.traffic_from, args.tile_label or "32x16")
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(environments are independent and would shard by env across GPUs)", file=sys.stderr)
        sys.exit(2)

    from paper_2607_08098_amd import scenes
    specs = scenes.mixed_batch_specs(3000)
    cpu = None
    if not (args.no_cpu_baseline or args.quick or args.variants or args.copy_calibration):
        cpu = cpu_baseline(specs)          # before anything touches the GPU
        log(f"cpu oracle: {cpu}")

    import numpy as np
    import torch
    from paper_2607_08098_amd import evis, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    ctx = evis.Context(0)
    if args.only == "disc512":   # the 512-disc batch alone (for profilers)
        tw, th = (int(v) for v in (args.tile or "32x16").lower().split("x"))
        evis.evis_set_tuning(ctx, tile_w=tw, tile_h=th)
        print(json.dumps(disc_sustained(ctx, max(1, args.disc_steps))))
        return
    t = time.time()
    W0, S = max(1, args.warmup), args.steps
    n_kf = W0 + S + 1
    seq = workloads.MixedSequence(ctx, n_kf, specs=specs)
    sensor = dict(C_on=0.2, C_off=0.2, K=0, K_max=64, refractory_us=0)
    arrs = [evis.env_array(seq.env_dicts(i, sensor)) for i in range(n_kf - 1)]
    n_envs = seq.n_envs
    shapes = np.array(seq.shapes, np.int64)
    px = shapes[:, 0] * shapes[:, 1]
    torch.cuda.synchronize()
    log(f"workload ready in {time.time() - t:.1f}s: {n_envs} envs, {seq.n_px} px, {n_kf} keyframes")

    K_all = torch.zeros((n_kf - 1, n_envs), dtype=torch.int32, device="cuda")
    out, n_total = evis.event_buffer(1 << 26)

    def step(i, flags=0):
        """Pair (i, i + 1): log intensity of keyframe i + 1 (one launch over
        every env), then the fused step."""
        seq.log_keyframe(i + 1)
        evis.evis_step_batch(ctx, arrs[i], out, n_total, K_all[i], flags)

    seq.reset_state(0)
    if args.tile:
        tw, th = (int(v) for v in args.tile.lower().split("x"))
        evis.evis_set_tuning(ctx, tile_w=tw, tile_h=th)
    autotune = None
    if not args.tile and not args.no_autotune:
        best, ms, trials, hit = evis.evis_autotune_ex(ctx, arrs[0], out, n_total, reps=3,
                                                      cache_path=args.tuning_cache or None)
        evis.evis_set_tuning(ctx, **best.as_dict())
        keys = ("tile_w", "tile_h", "grid_mult", "list_cap")
        autotune = dict(from_cache=hit, cache=os.path.basename(args.tuning_cache) if args.tuning_cache else None,
                        winner=dict({k: best.as_dict()[k] for k in keys}, ms=round(ms, 4)),
                        searched=[dict({k: t[k] for k in keys}, ms=round(m, 4)) for t, m in trials])
        log(f"autotune: {autotune}")
    tuning = evis.evis_get_tuning(ctx).as_dict()

    # warmup: pairs 0 .. W0-1 (the first step also captures the graph); size
    # the event buffer from the largest warmup step
    per_step = 0
    for i in range(W0):
        n_total.zero_()
        step(i)
        torch.cuda.synchronize()
        per_step = max(per_step, int(n_total.item()))
    need = per_step * S * 3 // 2 + 1024
    if need > out.shape[0]:
        out, n_total = evis.event_buffer(need)
    R_start = seq.L_ref.clone()      # the state at the start of the timed pairs

    # timed region: pairs W0 .. W0+S-1 of the sequence
    n_total.zero_()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for i in range(W0, W0 + S):
        step(i)
    e1.record()
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / S
    events_total = int(n_total.item())
    overflow = events_total > out.shape[0]
    Ks = K_all[W0:W0 + S].cpu().numpy().astype(np.int64)          # [S, n_envs]
    mpix_total = float((px[None, :] * Ks).sum()) / 1e6
    mpix_substeps = mpix_total / S
    value = mpix_total / (ms_total / 1e3)
    events_per_s = events_total / (ms_total / 1e3)
    log(f"batched: {ms_step:.3f} ms/step, {value:.0f} Mpix-substeps/s, {events_per_s:.3e} events/s")
    if args.quick and not args.variants:
        print(json.dumps(dict(ms_per_step=ms_step, value=value)))
        return

    def replay_timed(fn_step, pairs, kind=evis.EVIS_KERNEL_STEP, state=None):
        """Run fn_step over `pairs` from the timed region's start state (or
        state = (L_ref, start)) with the library's kernel timing on; (mean
        kernel ms, launches, events)."""
        lref, start = state if state is not None else (seq.L_ref, R_start)
        lref.copy_(start)
        torch.cuda.synchronize()
        evis.evis_profile_enable(ctx, True)
        n_total.zero_()
        for i in pairs:
            fn_step(i)
        torch.cuda.synchronize()
        kms, launches = evis.evis_profile_read(ctx, kind)
        evis.evis_profile_enable(ctx, False)
        return kms / max(launches, 1), launches, int(n_total.item())

    timed_pairs = list(range(W0, W0 + S))
    roof = None
    if not args.variants:
        # the fused tile kernel alone, timed with HIP events on its own stream,
        # over the same pairs from the same state
        tile_ms_avg, launches, ev = replay_timed(step, timed_pairs)
        ev_per_launch = ev / max(launches, 1)
        ops = float((px[None, :] * (OPS_INTERIOR * (Ks - 1) + OPS_LAST)).sum()) / S
        bytes_ = float(px.sum() * BYTES_PER_PX + BYTES_PER_EVENT * ev_per_launch)
        t_alu = ops / (ALU_PEAK_TOPS * 1e12)
        t_hbm = bytes_ / (HBM_PEAK_GBS * 1e9)
        traffic = None
        if os.path.exists(TRAFFIC_FILE):
            with open(TRAFFIC_FILE) as fh:
                tr = json.load(fh)
            if tr.get("kernel_hash") == kernel_hash() and tr.get("tuning") == [tuning["tile_w"], tuning["tile_h"]] \
                    and tr.get("workload") == "mixed64_sequence":
                traffic = tr.get("bytes_per_launch")
        if t_alu >= t_hbm:
            achieved = ops / (tile_ms_avg / 1e3) / 1e12
            roof = dict(bound="alu", achieved=round(achieved, 3), peak=round(ALU_PEAK_TOPS, 2),
                        unit="Tops/s", frac=round(achieved / ALU_PEAK_TOPS, 4), traffic=traffic)
        else:
            achieved = bytes_ / (tile_ms_avg / 1e3) / 1e9
            roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                        unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic)
        roof["kernel"] = "k_tile(step)"
        roof["kernel_ms"] = round(tile_ms_avg, 4)
        roof["ops_per_launch"] = ops
        roof["algorithmic_bytes_per_launch"] = bytes_
        roof["hbm_algorithmic_GBps"] = round(bytes_ / (tile_ms_avg / 1e3) / 1e9, 1)
        log(f"tile kernel {tile_ms_avg:.3f} ms; roofline {roof}")

    # the two-splat warps, and the gather warp with sensor noise, over the
    # first pairs of the same sequence and tile shape
    warps = {}
    n_var = max(0, min(args.warp_steps, S))
    var_pairs = timed_pairs[:n_var]
    Kv = Ks[:n_var]
    mpix_var = float((px[None, :] * Kv).sum()) / 1e6 / max(n_var, 1)
    if n_var > 0 and want("warps"):
        noise = dict(leak_rate_hz=0.1, shot_rate_hz=1.0, hot_rate_hz=100.0, hot_fraction=1e-3,
                     shot_L0=-7.0, shot_inv_range=0.1)
        for name, mode, nz in (("splat_b_primary", evis.EVIS_WARP_SPLAT | evis.EVIS_BLEND_B_PRIMARY,
                                None),
                               ("joint", evis.EVIS_WARP_JOINT, None),
                               ("gather_with_noise", evis.EVIS_WARP_GATHER, noise)):
            warrs = {}
            for i in var_pairs:
                wenvs = seq.env_dicts(i, dict(sensor, blend_mode=mode))
                if nz is not None:
                    for e, d in enumerate(wenvs):
                        d["noise"] = dict(nz, seed=9000 + e, pair_index=i)
                warrs[i] = evis.env_array(wenvs)
            wstep = lambda i: evis.evis_step_batch(ctx, warrs[i], out, n_total, None, 0)
            wstep(var_pairs[0])            # first launch of this kernel
            wms, wl, wev = replay_timed(wstep, var_pairs)
            if nz is None:
                wops = float((px[None, :] * (OPS_INTERIOR_TWO_SPLAT * (Kv - 1) + OPS_LAST)).sum())
            else:
                wops = float((px[None, :] * ((OPS_INTERIOR + OPS_NOISE) * (Kv - 1) + OPS_LAST
                                             + OPS_NOISE)).sum())
            wops /= n_var
            wach = wops / (wms / 1e3) / 1e12
            warps[name] = dict(kernel_ms=round(wms, 4), value=round(mpix_var / (wms / 1e3), 1),
                               events_per_step=round(wev / max(wl, 1), 1),
                               roofline=dict(bound="alu", achieved=round(wach, 3),
                                             peak=round(ALU_PEAK_TOPS, 2), unit="Tops/s",
                                             frac=round(wach / ALU_PEAK_TOPS, 4)))
            log(f"warp {name}: tile kernel {wms:.3f} ms")
            del warrs

    # defocus of every env's keyframe 1 (one batched launch, sigma 0.5 px):
    # HBM-bound, 8 algorithmic bytes per pixel (one read, one write)
    if n_var > 0 and want("defocus"):
        src = seq.I[1]
        blurred = torch.empty_like(src)
        views = [(seq.view(src, e), seq.view(blurred, e)) for e in range(n_envs)]

        def defocus_all():
            evis.evis_defocus_batch(ctx, views, 0.5)

        defocus_all()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.warp_steps):
            defocus_all()
        e1.record()
        torch.cuda.synchronize()
        eager_ms = e0.elapsed_time(e1) / args.warp_steps
        # the same launches captured once into a HIP graph and replayed
        gs = torch.cuda.Stream()
        gs.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(gs):
            defocus_all()
            gs.synchronize()
            with torch.cuda.graph(graph, stream=gs):
                defocus_all()
        torch.cuda.current_stream().wait_stream(gs)
        graph.replay()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.warp_steps):
            graph.replay()
        e1.record()
        torch.cuda.synchronize()
        dms = e0.elapsed_time(e1) / args.warp_steps
        gbs = 8.0 * float(px.sum()) / (dms / 1e3) / 1e9
        warps["defocus_sigma0.5"] = dict(ms_per_step=round(dms, 4), eager_ms_per_step=round(eager_ms, 4),
                                         images=n_envs, launches=(n_envs + 63) // 64,
                                         roofline=dict(bound="hbm", achieved=round(gbs, 1),
                                                       peak=HBM_PEAK_GBS, unit="GB/s",
                                                       frac=round(gbs / HBM_PEAK_GBS, 4)))
        log(f"defocus: {dms:.3f} ms (graph), {eager_ms:.3f} ms (eager) for {n_envs} images, {gbs:.0f} GB/s")
        del blurred, views, graph

    # voxel grid (128 bins per polarity) of one 1280x720 env from the stream
    # of the first timed pair: HBM-bound, 8 algorithmic bytes per event read
    # and per voxel written
    if n_var > 0 and want("voxel"):
        seq.L_ref.copy_(R_start)
        n_total.zero_()
        step(timed_pairs[0])
        torch.cuda.synchronize()
        ve = n_envs - 1
        vh, vw = seq.shapes[ve]
        vt0, vt1 = seq.times(timed_pairs[0])
        grid = torch.empty((2, 128, vh, vw), dtype=torch.float32, device="cuda")
        evis.evis_voxel_grid(ctx, out, n_total, ve, vh, vw, vt0, vt1, 128, out=grid)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.warp_steps):
            evis.evis_voxel_grid(ctx, out, n_total, ve, vh, vw, vt0, vt1, 128, out=grid)
        e1.record()
        torch.cuda.synchronize()
        vms = e0.elapsed_time(e1) / args.warp_steps
        nev = min(int(n_total.item()), out.shape[0])
        vbytes = 8.0 * nev + 8.0 * grid.numel()
        vgbs = vbytes / (vms / 1e3) / 1e9
        warps["voxel_grid_128"] = dict(ms=round(vms, 4), env=f"{vw}x{vh}", stream_events=nev,
                                       roofline=dict(bound="hbm", achieved=round(vgbs, 1),
                                                     peak=HBM_PEAK_GBS, unit="GB/s",
                                                     frac=round(vgbs / HBM_PEAK_GBS, 4)))
        log(f"voxel grid: {vms:.3f} ms ({nev} events scanned), {vgbs:.0f} GB/s")
        del grid

    # the HBM-bound forms: the event model over materialised frames (one
    # 1280x720 env, the K + 1 samples of the first timed pair written by
    # evis_interpolate first), and the fused step with small motion (K <= 2,
    # one warped substep) over the timed pairs
    if n_var > 0 and want("generate_events"):
        ve = n_envs - 1
        vh, vw = seq.shapes[ve]
        i0 = timed_pairs[0]
        Kg = int(Ks[0, ve])
        frames = torch.empty((Kg + 1, vh, vw), dtype=torch.float32, device="cuda")
        dv = seq.env_dicts(i0, sensor)[ve]
        vt0, vt1 = seq.times(i0)
        pair_v = dict(L_A=dv["L_A"], L_B=dv["L_B"], m_A=dv["m_A"], m_B=dv["m_B"], Z_A=dv["Z_A"],
                      Z_B=dv["Z_B"], t0=vt0, t1=vt1)
        evis.evis_interpolate(ctx, pair_v, Kg, 0, Kg + 1, evis.EVIS_BLEND_TIME, L_out=frames,
                              want_holes=False)
        lref = seq.view(R_start, ve).clone()
        st_v = dict(L_ref=lref)
        evis.evis_profile_enable(ctx, True)
        n_total.zero_()
        for _ in range(args.warp_steps):
            lref.copy_(seq.view(R_start, ve))
            evis.evis_generate_events(ctx, frames, vt0, vt1, sensor, st_v, ve, out, n_total, flags=0)
        torch.cuda.synchronize()
        gms, gl = evis.evis_profile_read(ctx, evis.EVIS_KERNEL_EVENTS)
        evis.evis_profile_enable(ctx, False)
        gms /= max(gl, 1)
        gev = int(n_total.item()) / max(gl, 1)
        gbytes = 4.0 * (Kg + 1) * vh * vw + 8.0 * vh * vw + 8.0 * gev
        ggbs = gbytes / (gms / 1e3) / 1e9
        warps["generate_events_1280x720"] = dict(
            kernel_ms=round(gms, 4), K=Kg, events=round(gev),
            roofline=dict(bound="hbm", achieved=round(ggbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                          frac=round(ggbs / HBM_PEAK_GBS, 4)))
        log(f"generate_events: {gms:.3f} ms, {ggbs:.0f} GB/s")
        del frames
    if n_var > 0 and want("events_batch"):
        i0 = timed_pairs[0]
        vt0, vt1 = seq.times(i0)
        # the same form over every env's samples of that pair in one launch
        # (evis_generate_events_batch): Σ 4 (K + 1) px bytes of samples, the
        # reference read and written, 8 B per event
        Kp = Ks[0]
        # each env's samples start on 256 bytes, as separate allocations
        # would (packed back to back, most planes would straddle lines)
        sizes = (Kp + 1) * px
        offs = np.concatenate([[0], np.cumsum((sizes + 63) // 64 * 64)])
        allf = torch.empty(int(offs[-1]), dtype=torch.float32, device="cuda")
        dicts = seq.env_dicts(i0, sensor)
        items = []
        for e, d in enumerate(dicts):
            H, W = seq.shapes[e]
            fr = allf[int(offs[e]):int(offs[e]) + int(sizes[e])].view(int(Kp[e]) + 1, H, W)
            evis.evis_interpolate(ctx, d, int(Kp[e]), 0, int(Kp[e]) + 1, evis.EVIS_BLEND_TIME,
                                  L_out=fr, want_holes=False)
            items.append(dict(L_seq=fr, t0=vt0, t1=vt1, env_id=e, C_on=0.2, C_off=0.2,
                              L_ref=seq.view(seq.L_ref, e)))
        def bstep(i):   # every repetition from the same state (outside the kernel's timing)
            seq.L_ref.copy_(R_start)
            evis.evis_generate_events_batch(ctx, items, out, n_total, flags=0)
        bstep(i0)
        bms, bl, bev = replay_timed(bstep, [i0] * args.warp_steps, kind=evis.EVIS_KERNEL_EVENTS)
        bev /= max(bl, 1)
        bbytes = 4.0 * float(sizes.sum()) + 8.0 * float(px.sum()) + 8.0 * bev
        bgbs = bbytes / (bms / 1e3) / 1e9
        warps["generate_events_batch64"] = dict(
            kernel_ms=round(bms, 4), samples_GB=round(4.0 * float(sizes.sum()) / 1e9, 3),
            events=round(bev),
            roofline=dict(bound="hbm", achieved=round(bgbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                          frac=round(bgbs / HBM_PEAK_GBS, 4)))
        log(f"generate_events batch of 64: {bms:.3f} ms, {bgbs:.0f} GB/s")
        del allf, items
    if n_var > 0 and want("small_motion"):
        # small motion: the same scenes turned by at most 1 px per keyframe
        # at the image corners, motion noise N(0, 0.15^2) px, so the
        # adaptive K is at most 2 (the form whose bytes per pixel-substep
        # are largest), content and motion vectors agreeing
        small = workloads.MixedSequence(
            ctx, n_var + 1, specs=specs,
            seq_kw=lambda e, H, W: dict(noise=0.15, theta=1.0 / np.hypot((W - 1) / 2, (H - 1) / 2)))
        small.reset_state(0)
        k2arrs = {W0 + i: evis.env_array(small.env_dicts(i, dict(sensor))) for i in range(n_var)}
        K2 = torch.zeros(n_envs, dtype=torch.int32, device="cuda")
        k2step = lambda i: evis.evis_step_batch(ctx, k2arrs[i], out, n_total, K2, 0)
        k2step(var_pairs[0])
        small.reset_state(0)
        kms, kl, kev = replay_timed(k2step, var_pairs, state=(small.L_ref, small.L_ref.clone()))
        kev /= max(kl, 1)
        kbytes = float(px.sum()) * BYTES_PER_PX + BYTES_PER_EVENT * kev
        kgbs = kbytes / (kms / 1e3) / 1e9
        kK = K2.cpu().numpy().astype(np.int64)
        warps["fused_K2"] = dict(kernel_ms=round(kms, 4), events=round(kev), max_K=int(kK.max()),
                                 mpix_substeps_per_s=round(float((px * kK).sum()) / 1e6 / (kms / 1e3), 1),
                                 roofline=dict(bound="hbm", achieved=round(kgbs, 1), peak=HBM_PEAK_GBS,
                                               unit="GB/s", frac=round(kgbs / HBM_PEAK_GBS, 4)))
        log(f"fused, small motion (K <= 2): {kms:.3f} ms, {kgbs:.0f} GB/s")
        del small, k2arrs

    if args.variants:
        print(json.dumps(dict(ms_per_step=ms_step, value=value, variants=warps)))
        return

    # per-env-launch forms over the first timed pairs from the same state:
    # plain (every sample to HBM, then the event model, env by env) and the
    # fused step launched env by env
    plain = None
    fused_per_env = None
    n_plain = max(0, min(args.plain_steps, S))
    if n_plain > 0:
        Kp = Ks[:n_plain]
        mpix_plain = float((px[None, :] * Kp).sum()) / 1e6
        Hmax_W = int(px.max())
        L_seq = torch.empty((int(Kp.max()) + 1) * Hmax_W, dtype=torch.float32, device="cuda")
        st = [dict(L_ref=seq.view(seq.L_ref, e)) for e in range(n_envs)]

        def plain_step(i):
            seq.log_keyframe(i + 1)
            t0_, t1_ = seq.times(i)
            for e, d in enumerate(seq.env_dicts(i, sensor)):
                H, W = seq.shapes[e]
                K = int(Ks[i - W0, e])
                Ls = L_seq[: (K + 1) * H * W].view(K + 1, H, W)
                evis.evis_interpolate(ctx, d, K, 0, K + 1, evis.EVIS_BLEND_TIME, L_out=Ls,
                                      want_holes=False)
                evis.evis_generate_events(ctx, Ls, t0_, t1_, sensor, st[e], e, out, n_total, flags=0)

        singles = {i: [evis.env_array([d]) for d in seq.env_dicts(i, sensor)]
                   for i in timed_pairs[:n_plain]}

        def fused_single_step(i):
            seq.log_keyframe(i + 1)
            for a in singles[i]:
                evis.evis_step_batch(ctx, a, out, n_total, None, 0)

        res = {}
        for name, fn in (("plain", plain_step), ("fused_per_env", fused_single_step)):
            seq.L_ref.copy_(R_start)
            fn(timed_pairs[0])                      # first launches of these shapes
            seq.L_ref.copy_(R_start)
            n_total.zero_()
            torch.cuda.synchronize()
            e0.record()
            for i in timed_pairs[:n_plain]:
                fn(i)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / n_plain
            res[name] = dict(ms_per_step=round(ms, 3), value=round(mpix_plain / n_plain / (ms / 1e3), 1),
                             pairs=n_plain)
            log(f"{name}: {ms:.3f} ms/step")
        plain, fused_per_env = res["plain"], res["fused_per_env"]

    disc = disc_sustained(ctx, args.disc_steps) if args.disc_steps > 0 else None

    rec = dict(
        metric="Mpix-substeps/s (64 mixed-res envs, batched persistent launch)",
        value=round(value, 1), unit="Mpix-substeps/s", n_gpus=1, steps=S,
        warmup=W0, ms_per_step=round(ms_step, 4), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload="mixed64_sequence: 24x346x260 + 24x640x480 + 16x1280x720 rotating blob "
                             "keyframe sequences at 60 Hz, one new keyframe per step (pairs "
                             f"{W0}..{W0 + S - 1}, state carried), adaptive K<=64, C=0.2",
                    n_envs=n_envs, px_per_step=int(px.sum()),
                    mean_K=round(float(Ks.mean()), 2), mpix_substeps_per_step=round(mpix_substeps, 2),
                    tuning=tuning, autotune=autotune),
        events_per_s=round(events_per_s, 1), events_per_step=round(events_total / S, 1),
        event_buffer_overflow=overflow,
        per_env_plain=plain, per_env_fused=fused_per_env,
        batched_vs_plain=(round(value / plain["value"], 2) if plain else None),
        batched_vs_fused_per_env=(round(value / fused_per_env["value"], 2) if fused_per_env else None),
        roofline=roof, cpu_baseline=cpu, variants=warps or None, disc512_sustained=disc,
    )
    print(json.dumps(rec))
    ctx.close()


if __name__ == "__main__":
    main()

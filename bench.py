#!/usr/bin/env python
"""ERP rasterizer benchmark: forward + L1 + backward iterations per second.

Workload: 1M Gaussians in the indoor room layout (70% on the faces of an
axis-aligned box, 30% in a shell, 20% of all moved into a 2-degree wedge at
world longitude pi), SH degree 3, 2048x1024 ERP images, 200 seeded poses
(centre in the unit ball, random yaw).  One step = one pose: omnigs_forward
(project, depth sort, emit, tile sort, ranges, blend; with instance and
block-entry capacities sized from the poses' counts, so no step reads
anything back), omnigs_l1_loss against a per-pose target image (the render
of a perturbed copy of the scene, prepared before timing), and
omnigs_backward (reverse blend, projection chain).  Inputs are resident in
HBM when timing starts.

Prints one JSON line (stdout) with the throughput; the roofline of the
dominant kernel (its stage bracketed with HIP events during the timed region;
no other stage is, since each event costs the stream a few microseconds; the
per-stage breakdown comes from a second pass over the same steps with every
stage timed); both blends against the FP32 peak and the bandwidth-bound
stages against the HBM peak, each also against the device's measured FMA
and copy ceilings; the per-pose fraction of Gaussians crossing the seam; and
the legs: the same workload with every pose at yaw 0 (the wedge across the
seam), 3M Gaussians at 3840x1920, the training iteration, pinhole crops,
masks and auxiliary outputs, the serving measurement (continuous batching
vs one request at a time on the same resident scene: renders/s and p50/p99
latency at Poisson arrival rates of 0.5, 1 and 2 times the one-at-a-time
capacity) and the FP64 CPU oracle timed on the host (all cores, and one core
against all on a sample).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-serve] [--no-stress] ...
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR = 157.3e12   # FLOP/s, MI355X published dense FP32 vector
PEAK_HBM = 8.0e12             # B/s
COPY_BYTES = 256 << 20        # plain copy used to calibrate the HBM counters
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "blend_bwd_1M_2048x1024_traffic.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2404_03202_amd", "csrc", "blend.hip")

# Algorithmic work of the blends, per (pixel, list position) pair walked up to
# the pixel's last contributor (sum of n_contrib): about 12 operations + one
# exp forward and 50 + one exp backward (alpha, transmittance, the colour and
# opacity terms and the moments of the conic gradient), each operation
# counted as one FLOP against the FP32 vector peak.
OPS_FWD_PAIR = 13
OPS_BWD_PAIR = 51
# Refined count: evaluating alpha (offsets, quadratic form, exp2, opacity,
# clamp; FMA = 2) = 12 FLOP per walked pair; the backward's gradient terms
# for a pair that was blended = 24 more.
FLOP_ALPHA = 12
FLOP_GRAD = 24
# HBM-bound stages, algorithmic bytes: per Gaussian for the projection (the
# 236 parameter bytes read, the 48-byte blend record and the sort key,
# depth, tile count and rectangle written) and its backward (parameters and
# the ten accumulators read, 59 gradients + dL/ds written).
BYTES_PROJECT = 300
BYTES_PROJECT_BWD = 600


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per blend_bwd launch from the committed counter summary, or
    None when the kernel source changed since the counters were taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    digest = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if kv.get("source_sha256") != digest:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def timed(step, ks, stages):
    """Seconds taken by step(k) for k in ks between two synchronisations,
    with the library's stage events on for `stages` only (None: every stage,
    (): none); returns (seconds, {stage: (ms, launches)})."""
    import torch
    from paper_2404_03202_amd import omnigs as B
    B.omnigs_profile_read()
    B.omnigs_profile_enable(stages is None or len(stages) > 0, stages=None if stages is None else list(stages))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in ks:
        step(k)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    B.omnigs_profile_enable(False)
    return dt, B.omnigs_profile_read()


def cpu_baseline(g, poses, gt_images):
    """FP64 oracle (forward + L1 + backward) on the host cores over a bounded
    sample of the benchmark's poses, plus one core against all of them on a
    quarter of one pose's tiles."""
    from oracle import oracle as O
    nproc = os.cpu_count()
    affinity = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else []
    cores = O.num_threads()
    t0 = time.perf_counter()
    for pose, gt_image in zip(poses, gt_images):
        sc = O.Scene(g, pose)
        r = O.render(sc, alt=False)
        _, dl = O.l1(r["image"], gt_image)
        O.backward(sc, dl, with_abs=False)
    dt = time.perf_counter() - t0
    n = len(poses)

    # one core vs all cores: forward + L1 + backward of pose 0 restricted to
    # a seeded quarter of its tiles (the projection still covers every
    # Gaussian)
    sc = O.Scene(g, poses[0])
    ntiles = sc.tiles_x * sc.tiles_y
    mask = np.zeros(ntiles, bool)
    mask[np.random.default_rng(11).choice(ntiles, ntiles // 4, replace=False)] = True

    def sample():
        t = time.perf_counter()
        r = O.render(sc, alt=False, tile_mask=mask)
        _, dl = O.l1(r["image"], gt_images[0])
        O.backward(sc, dl, with_abs=False, tile_mask=mask)
        return time.perf_counter() - t

    t_all = sample()
    O.set_num_threads(1)
    try:
        t_one = sample()
    finally:
        O.set_num_threads(cores)

    # serving: the oracle's forward of the first request of each resolution
    # in the serving stream (the requests the serving accuracy test samples)
    from paper_2404_03202_amd import scenes
    stream = scenes.serve_cameras(4, 64)
    serve_s = {}
    for w, h in scenes.SERVE_RESOLUTIONS:
        cam = next(c for c in stream if (c["width"], c["height"]) == (w, h))
        t = time.perf_counter()
        O.render(O.Scene(g, cam), alt=False)
        serve_s[f"{w}x{h}"] = time.perf_counter() - t
    return dict(value=n / dt, unit="iters/s", cores=cores, kind="oracle",
                sample=f"{n} of 200 poses (poses 0-{n - 1}), full 1M Gaussians at 2048x1024: forward + L1 + backward, "
                       f"{dt:.1f} s on {cores} threads",
                nproc=nproc, affinity=f"{len(affinity)} cpus: {affinity[0]}-{affinity[-1]}" if affinity else None,
                one_core=dict(sample="pose 0, forward + L1 + backward over a seeded quarter of its 8192 tiles "
                                     "(projection of all 1M Gaussians)",
                              seconds_1_thread=t_one, seconds_all_threads=t_all, threads=cores,
                              speedup=t_one / t_all,
                              implied_1core_iters_per_s=(n / dt) * t_all / t_one),
                serving=dict(sample="forward of the first request of each serving resolution (resident 1M-Gaussian "
                                    f"scene), {cores} threads", seconds=serve_s,
                             renders_per_s=len(serve_s) / sum(serve_s.values())),
                note="baseline only")


def serving_bench(gd, n_requests, slots, max_batch, log):
    """Continuous-batching server vs one-request-at-a-time on the resident
    1M-Gaussian scene: resolutions uniform over 512x256 .. 3840x1920, forward
    only.  mu1 = the one-at-a-time capacity (all requests queued at once);
    then Poisson arrivals at 0.5, 1 and 2 x mu1, the same requests for both."""
    import torch
    from paper_2404_03202_amd import omnigs as B
    from paper_2404_03202_amd import scenes, serve

    res = scenes.SERVE_RESOLUTIONS
    cams = scenes.serve_cameras(4, n_requests)

    def server(batched):
        srv = serve.Server(gd, slots=slots if batched else 1, max_batch=max_batch if batched else 1,
                           hbm_budget=32 << 30, keep_images=False)
        srv.calibrate([scenes.camera(w, h) for (w, h) in res])
        return srv

    # warm the caching allocator and the code paths
    for batched in (False, True):
        server(batched).run(serve.make_requests(cams[:64]))
    torch.cuda.synchronize()
    sat = {}
    for name, batched in (("one_at_a_time", False), ("batched", True)):
        sat[name] = server(batched).run(serve.make_requests(cams))
        log(f"serving saturated {name}: {sat[name]}")
    mu1 = sat["one_at_a_time"]["renders_per_s"]
    rates = []
    for k, mult in enumerate((0.5, 1.0, 2.0)):
        arr = scenes.arrival_times(4, n_requests, mult * mu1, run=k)
        row = dict(multiplier=mult, rate_hz=mult * mu1)
        for name, batched in (("one_at_a_time", False), ("batched", True)):
            srv = server(batched)
            keep = set(range(0, n_requests, max(1, n_requests // 24))) if (batched and mult == 2.0) else False
            srv.keep_images = keep
            reqs = serve.make_requests(cams, arr)
            row[name] = srv.run(reqs)
            log(f"serving {mult} x mu1 {name}: {row[name]}")
            if keep:
                # every kept result equals the render of that request alone
                same = 0
                for r in reqs:
                    if r.image is not None:
                        same += int(torch.equal(r.image, B.omnigs_forward(gd, r.camera).image))
                row["identical_alone"] = f"{same}/{len(keep)}"
        rates.append(row)
    return dict(workload=f"resident 1M-Gaussian room scene, {n_requests} requests, resolution uniform over "
                         + ", ".join(f"{w}x{h}" for w, h in res) + ", forward only",
                slots=slots, max_batch=max_batch, mu1_renders_per_s=mu1, saturated=sat, poisson=rates)


def hbm_stages(ms, n, S, M, W, H, ceilings=None):
    """Algorithmic HBM bytes, GB/s and fraction of the 8 TB/s peak (and of
    the measured copy rate) of the bandwidth-bound stages: u32 keys and
    values; a sort reads its keys once for the digit histograms of all its
    passes, then each pass reads and writes key + value (the depth sort's
    first pass generates its values); the scan of the block counts in depth
    order reads the count and rectangle of every Gaussian; block entries (S)
    are emitted, sorted by block and ranged; the expansion reads every entry
    and its rectangle twice (count, write) and writes each instance (M) once."""
    supers = ((W // 16 + 7) // 8) * ((H // 16 + 7) // 8)
    passes = -(-max(1, int(np.ceil(np.log2(supers)))) // 8)
    algo = dict(project=BYTES_PROJECT * n, depth_sort=(4 + 4 * 16 - 4) * n, emit_count=12 * n,
                super_emit=8 * S + 20 * n, super_sort=(4 + passes * 16) * S + 4 * S, tile_bin=24 * S + 4 * M,
                project_bwd=BYTES_PROJECT_BWD * n)
    out = {}
    for k, b in algo.items():
        if k not in ms or ms[k] <= 0:
            continue
        rate = b / (ms[k] * 1e-3)
        row = dict(ms=ms[k], algo_bytes=b, GBps=rate / 1e9, frac=rate / PEAK_HBM)
        if ceilings and ceilings.get("copy_gbps"):
            row["frac_of_measured_copy"] = rate / (ceilings["copy_gbps"] * 1e9)
        out[k] = row
    return out, passes


def blend_rates(walked, blended, ms_fwd, ms_bwd, ceilings=None):
    """The two blends against the FP32 vector peak: work counted as a fixed
    number of ops per walked pair, and as the refined FLOP count."""
    out = {}
    for name, ms, ops, flops in (("blend_fwd", ms_fwd, OPS_FWD_PAIR * walked, FLOP_ALPHA * walked),
                                 ("blend_bwd", ms_bwd, OPS_BWD_PAIR * walked, FLOP_ALPHA * walked + FLOP_GRAD * blended)):
        if not ms:
            continue
        a = ops / (ms * 1e-3)
        r = flops / (ms * 1e-3)
        row = dict(ms=ms, TFLOPs=a / 1e12, frac=a / PEAK_FP32_VECTOR, refined_TFLOPs=r / 1e12,
                   refined_frac=r / PEAK_FP32_VECTOR)
        if ceilings and ceilings.get("fma_tflops"):
            row["frac_of_measured_fma"] = a / (ceilings["fma_tflops"] * 1e12)
        out[name] = row
    return out


def pair_counts(gd, cams):
    """Mean (walked, blended) pixel-instance pairs per forward over `cams`:
    walked = sum of n_contrib, blended = sum of n_blended."""
    import torch
    from paper_2404_03202_amd import omnigs as B
    walked = blended = 0
    for c in cams:
        f = B.omnigs_forward(gd, c, with_blended=True)
        walked += int(f.n_contrib.sum(dtype=torch.int64))
        blended += int(f.n_blended.sum(dtype=torch.int64))
    return walked / len(cams), blended / len(cams)


def seam_fractions(gd, cams):
    from paper_2404_03202_amd import omnigs as B
    fr = np.array([B.omnigs_forward(gd, c).seam_fraction() for c in cams])
    return dict(mean=float(fr.mean()), min=float(fr.min()), p50=float(np.median(fr)), max=float(fr.max()))


def stress_bench(steps, log, ceilings=None):
    """Large scene: 3M Gaussians (room layout, scales log-uniform [0.002,
    0.5]) at 3840x1920, forward + L1 + backward per pose.  Reports stage
    times, the algorithmic HBM rate of the sort and binning stages, the
    algorithmic FP32 rate of the two blends and the backward's atomics."""
    import torch
    from paper_2404_03202_amd import omnigs as B
    from paper_2404_03202_amd import scenes

    g, poses, gt = scenes.config3(n_poses=4)
    dev = "cuda:0"
    gd = {k: (torch.from_numpy(v).to(dev) if k != "sh_degree" else v) for k, v in g.items()}
    gtd = {k: (torch.from_numpy(v).to(dev) if k != "sh_degree" else v) for k, v in gt.items()}
    targets = [B.omnigs_forward(gtd, p).image.clone() for p in poses]
    del gtd
    n = int(g["means"].shape[0])
    W, H = 3840, 1920
    inst, entries = [], []

    def step(k):
        p = poses[k % len(poses)]
        fwd = B.omnigs_forward(gd, p)
        inst.append(fwd.n_instances)
        entries.append(fwd.n_entries)
        _, dl = B.omnigs_l1_loss(fwd.image, targets[k % len(poses)])
        B.omnigs_backward(gd, p, None, fwd, dl)

    step(0)
    torch.cuda.synchronize()
    inst.clear()
    entries.clear()
    dt, _ = timed(step, range(steps), ())
    _, prof = timed(step, range(steps), None)  # stage breakdown
    ms = {k: v[0] / steps for k, v in prof.items() if v[1]}
    M = float(np.mean(inst))
    S = float(np.mean(entries))
    walked, blended = pair_counts(gd, [poses[k % len(poses)] for k in range(steps)])
    stages, passes = hbm_stages(ms, n, S, M, W, H, ceilings)
    out = dict(workload="3M Gaussians, room layout, scales log-uniform [0.002, 0.5], SH degree 3, 3840x1920 ERP, "
                        f"{len(poses)} poses, forward + L1 + backward per pose (instance counts read back)",
               steps=steps, ms_per_step=dt * 1e3 / steps, iters_per_s=steps / dt, instances_per_step=M,
               block_entries_per_step=S, block_sort_passes=passes, stage_ms=ms, hbm_stages=stages,
               blend_pairs=dict(walked=walked, blended=blended),
               blends=blend_rates(walked, blended, ms.get("blend_fwd"), ms.get("blend_bwd"), ceilings),
               seam_fraction=seam_fractions(gd, poses))
    log(f"stress: {out}")
    return out


def seam_stress_bench(gd, gt, steps, warmup, n_poses, log):
    """The benchmark workload with every pose at yaw 0, where the wedge of
    Gaussians placed at world longitude pi straddles the image seam: centres
    uniform in the unit ball as in the benchmark, forward + L1 + backward
    per pose with capacities (no read-back)."""
    import torch
    from paper_2404_03202_amd import omnigs as B
    from paper_2404_03202_amd import scenes

    poses = scenes.poses(2, n_poses, 2048, 1024, yaw_zero=True)
    used = [poses[k % len(poses)] for k in range(warmup + steps)]
    gtd = {k: (torch.from_numpy(v).to("cuda:0") if k != "sh_degree" else v) for k, v in gt.items()}
    targets = {id(p): B.omnigs_forward(gtd, p).image.clone() for p in used}
    del gtd
    m_max = s_max = 0
    for p in used:
        f = B.omnigs_forward(gd, p)
        m_max, s_max = max(m_max, f.n_instances), max(s_max, f.n_entries)
    cap = (int(1.05 * m_max) + 1, int(1.05 * s_max) + 1)
    overflow = []

    def step(k):
        p = poses[k % len(poses)]
        fwd = B.omnigs_forward(gd, p, capacity=cap)
        overflow.append(fwd.overflow)
        _, dl = B.omnigs_l1_loss(fwd.image, targets[id(p)])
        B.omnigs_backward(gd, p, None, fwd, dl)

    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    dt, _ = timed(step, range(warmup, warmup + steps), ())
    _, prof = timed(step, range(warmup, warmup + steps), None)
    if int(torch.cat(overflow).sum()):
        raise SystemExit("bench.py: the seam-stress leg overflowed its capacities")
    out = dict(workload=f"1M Gaussians, room layout, 2048x1024 ERP, {n_poses} poses at yaw 0 (centre in the unit "
                        "ball), forward + L1 + backward per pose",
               steps=steps, iters_per_s=steps / dt, ms_per_step=dt * 1e3 / steps,
               stage_ms={k: v[0] / steps for k, v in prof.items() if v[1]},
               seam_fraction=seam_fractions(gd, poses))
    log(f"seam stress: {out}")
    return out


def train_bench(g, poses, targets, steps, log):
    """The full iteration of Alg. 1 on the benchmark workload: forward, L1,
    backward, densification statistics and the Adam step (train.Trainer),
    plus one densification event on the 1M-Gaussian set."""
    import torch
    from paper_2404_03202_amd import omnigs as B
    from paper_2404_03202_amd.train import Trainer, TrainSettings

    # no densification inside the timing; forwards with capacities (no count
    # read-back), overflows settled two iterations later
    tr = Trainer(g, TrainSettings(extent=10.0, densify_from=10 ** 9), capacity_slack=1.1)
    for k in range(3):
        tr.step(poses[k % len(poses)], targets[k % len(poses)])
    torch.cuda.synchronize()

    def it(k):
        tr.step(poses[k % len(poses)], targets[k % len(poses)])

    dt, _ = timed(it, range(steps), ())
    _, prof = timed(it, range(steps), None)  # stage breakdown
    tr.flush()
    n0 = tr.n
    torch.cuda.synchronize()
    B.omnigs_profile_enable(True)
    t1 = time.perf_counter()
    tr.densify(screen=False)  # as before the first opacity reset
    torch.cuda.synchronize()
    dens = time.perf_counter() - t1
    B.omnigs_profile_enable(False)
    dprof = B.omnigs_profile_read()
    out = dict(workload="forward + photometric loss (L1 + 0.2 SSIM term) + backward + densification statistics + "
                        "Adam per pose, 1M Gaussians, 2048x1024, the benchmark poses; forwards with capacities "
                        "(1.1x the counts read so far), overflowed iterations run again",
               steps=steps, iters_per_s=steps / dt, ms_per_step=dt * 1e3 / steps, redone=tr.redone,
               stage_ms={k: v[0] / steps for k, v in prof.items() if v[1]},
               densify=dict(gaussians_before=n0, gaussians_after=tr.n, ms=dens * 1e3,
                            kernel_ms=dprof["densify"][0]))
    log(f"train: {out}")
    return out


def pinhole_bench(gd, crops, crop_targets, poses, steps, log):
    """The pinhole camera of Eq. 2 on the benchmark scene: (1) forward + L1 +
    backward of 1024x1024 perspective crops (90 degree field of view, seeded
    poses inside the room); (2) the six 512x512 faces of a cube map around
    each benchmark pose rendered as one batch, against the 2048x1024 ERP
    forward of the same pose (the same pixel count on the sphere)."""
    import torch
    from paper_2404_03202_amd import omnigs as B
    from paper_2404_03202_amd import scenes

    def crop_step(k):
        c = crops[k % len(crops)]
        fwd = B.omnigs_forward(gd, c)
        loss, dl = B.omnigs_l1_loss(fwd.image, crop_targets[k % len(crops)])
        B.omnigs_backward(gd, c, None, fwd, dl)

    for k in range(5):
        crop_step(k)
    torch.cuda.synchronize()
    dt, _ = timed(crop_step, range(steps), ())
    _, prof = timed(crop_step, range(steps), None)  # stage breakdown
    crop = dict(workload="1M Gaussians, 1024x1024 pinhole crops (90 deg), forward + L1 + backward per crop",
                steps=steps, iters_per_s=steps / dt, ms_per_step=dt * 1e3 / steps,
                stage_ms={k: v[0] / steps for k, v in prof.items() if v[1]})
    n = min(steps, len(poses))
    faces = [scenes.cube_faces(p, 512) for p in poses[:n]]
    for k in range(3):
        B.omnigs_forward_batch(gd, faces[k])
        B.omnigs_forward(gd, poses[k])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n):
        B.omnigs_forward_batch(gd, faces[k])
    torch.cuda.synchronize()
    t_cube = time.perf_counter() - t0
    t0 = time.perf_counter()
    for k in range(n):
        B.omnigs_forward(gd, poses[k])
    torch.cuda.synchronize()
    t_erp = time.perf_counter() - t0
    cube = dict(workload="six 512x512 cube-map faces per benchmark pose, one batched forward",
                poses=n, poses_per_s=n / t_cube, ms_per_pose=t_cube * 1e3 / n,
                erp_forward_poses_per_s=n / t_erp, erp_ms_per_pose=t_erp * 1e3 / n)
    out = dict(crop=crop, cube_map=cube)
    log(f"pinhole: {out}")
    return out


def aux_bench(g, gd, masked, steps, log):
    """Loss masks and auxiliary outputs: (1) training at 1520x760 with the
    bottom 48 rows left out of the loss (the 360Roam setting: 712 rows used),
    once with the camera's row crop (the rows are never rendered) and once
    rendering all 760 rows with a loss mask of zeros there; (2) forward +
    backward at 2048x1024 with the depth image and depth / alpha cotangents
    against the plain colour pass."""
    import torch
    from paper_2404_03202_amd import omnigs as B
    from paper_2404_03202_amd.train import Trainer, TrainSettings

    cams, targets_full = masked
    out = {}
    H, rows = 760, 712
    mask = torch.zeros(H, 1520, device="cuda:0")
    mask[:rows] = 1.0
    for name, use_rows in (("rows_712_of_760", True), ("mask_712_of_760", False)):
        tr = Trainer(g, TrainSettings(extent=10.0, densify_from=10 ** 9))

        def it(k):
            c = cams[k % len(cams)]
            t = targets_full[k % len(cams)]
            if use_rows:
                return tr.step(dict(c, rows=rows), t[:, :rows].contiguous())
            return tr.step(c, t, mask=mask)

        for k in range(3):
            it(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            it(k)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = dict(iters_per_s=steps / dt, ms_per_step=dt * 1e3 / steps)
        del tr
    from paper_2404_03202_amd import scenes
    poses = scenes.poses(2, 50, 2048, 1024)
    rng = torch.Generator(device="cuda:0").manual_seed(7)
    GD = torch.randn(1024, 2048, device="cuda:0", generator=rng) * 1e-6
    GA = torch.randn(1024, 2048, device="cuda:0", generator=rng) * 1e-6
    G = torch.randn(3, 1024, 2048, device="cuda:0", generator=rng) * 1e-6
    for name, aux in (("colour", False), ("colour_depth_alpha", True)):
        def it(k):
            p = poses[k % len(poses)]
            fwd = B.omnigs_forward(gd, p, with_depth=aux)
            B.omnigs_backward(gd, p, None, fwd, G, dL_ddepth=GD if aux else None, dL_dalpha=GA if aux else None)

        for k in range(3):
            it(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            it(k)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["fwd_bwd_2048x1024_" + name] = dict(iters_per_s=steps / dt, ms_per_step=dt * 1e3 / steps)
    log(f"aux: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--poses", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-stress", action="store_true", help="skip the 3M-Gaussian 3840x1920 workload")
    ap.add_argument("--no-seam-stress", action="store_true", help="skip the yaw-0 seam-stress workload")
    ap.add_argument("--no-ceilings", action="store_true", help="skip the measured FMA/exp/atomic/copy ceilings")
    ap.add_argument("--no-train", action="store_true", help="skip the full training-iteration measurement")
    ap.add_argument("--no-pinhole", action="store_true", help="skip the pinhole-camera measurement")
    ap.add_argument("--no-aux", action="store_true", help="skip the loss-mask / depth-output measurement")
    ap.add_argument("--stress-steps", type=int, default=8)
    ap.add_argument("--serve-requests", type=int, default=800)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-max-batch", type=int, default=4)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run plain 256 MiB device copies (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (the rasterizer has no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2404_03202_amd import omnigs as B
    from paper_2404_03202_amd import scenes

    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes=COPY_BYTES, copies=5)))
        return
    ceilings = None
    if not args.no_ceilings:
        ceilings = B.omnigs_measure_ceilings(atomic_words=10 << 20, copy_bytes=COPY_BYTES)
        log(f"ceilings: {ceilings}")
    t0 = time.perf_counter()
    g, poses, gt = scenes.config2(n_poses=args.poses)
    log(f"scene: {g['means'].shape[0]} Gaussians, {len(poses)} poses ({time.perf_counter() - t0:.1f} s)")
    gd = {k: (torch.from_numpy(v).to(dev) if k != "sh_degree" else v) for k, v in g.items()}
    gtd = {k: (torch.from_numpy(v).to(dev) if k != "sh_degree" else v) for k, v in gt.items()}
    targets = []
    for p in poses:
        targets.append(B.omnigs_forward(gtd, p).image.clone())
    crops = scenes.crop_poses(2, 100, 1024, 1024, 90.0)
    crop_targets = [] if args.no_pinhole else [B.omnigs_forward(gtd, c).image.clone() for c in crops]
    masked_cams = scenes.poses(2, 50, 1520, 760)
    masked = (masked_cams, [] if args.no_aux else [B.omnigs_forward(gtd, c).image.clone() for c in masked_cams])
    del gtd
    torch.cuda.synchronize()
    log("targets rendered")

    # instance and block-entry capacities from one counted forward of every
    # pose (5% headroom): the timed forwards then read nothing back, and every
    # step's overflow flag is checked after the timed region
    m_max = s_max = 0
    m_pose, s_pose = [], []
    for p in poses:
        f = B.omnigs_forward(gd, p)
        m_pose.append(f.n_instances)
        s_pose.append(f.n_entries)
        m_max, s_max = max(m_max, f.n_instances), max(s_max, f.n_entries)
    del f
    cap = (int(1.05 * m_max) + 1, int(1.05 * s_max) + 1)
    overflow = []

    def step(k):
        p = poses[k % len(poses)]
        fwd = B.omnigs_forward(gd, p, capacity=cap)
        overflow.append(fwd.overflow)
        loss, dl = B.omnigs_l1_loss(fwd.image, targets[k % len(poses)])
        B.omnigs_backward(gd, p, None, fwd, dl)
        return fwd

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    ks = range(args.warmup, args.warmup + args.steps)
    # the timed region: only the dominant kernel's stage carries events
    dt, prof_bwd = timed(step, ks, ("blend_bwd",))
    # stage breakdown: the same steps again, every stage bracketed
    dt_prof, prof = timed(step, ks, None)
    n_over = int(torch.cat(overflow).sum())
    if n_over:
        raise SystemExit(f"bench.py: {n_over} steps overflowed the capacities {cap}")
    log(f"{args.steps / dt:.1f} iters/s ({args.steps / dt_prof:.1f} with every stage timed), capacities {cap}")
    log("stages (ms per step): " + ", ".join(f"{k} {v[0] / args.steps:.3f}" for k, v in prof.items() if v[1]))

    # pairs walked / blended by the timed steps (deterministic re-render)
    timed_poses = [poses[k % len(poses)] for k in ks]
    walked, blended = pair_counts(gd, timed_poses)
    bwd_ms, bwd_n = prof_bwd["blend_bwd"]
    bwd_avg = bwd_ms / max(bwd_n, 1)
    stage_ms = {k: v[0] / args.steps for k, v in prof.items() if v[1]}
    blends = blend_rates(walked, blended, stage_ms.get("blend_fwd"), bwd_avg, ceilings)
    dominant = max(((k, v[0]) for k, v in prof.items()), key=lambda kv: kv[1])[0]
    rb = blends["blend_bwd"]
    roofline = dict(kernel="blend_bwd", bound="alu", achieved=rb["TFLOPs"], peak=PEAK_FP32_VECTOR / 1e12,
                    unit="TFLOP/s", frac=rb["frac"], traffic=measured_traffic(),
                    work=f"{OPS_BWD_PAIR} ops per walked pixel-instance pair (sum of n_contrib), one op = one FLOP",
                    refined_achieved=rb["refined_TFLOPs"], refined_frac=rb["refined_frac"],
                    frac_of_measured_fma=rb.get("frac_of_measured_fma"),
                    avg_launch_ms=bwd_avg, pairs_walked_per_launch=walked, pairs_blended_per_launch=blended,
                    dominant_stage=dominant)
    M = float(np.mean([m_pose[k % len(poses)] for k in ks]))
    S = float(np.mean([s_pose[k % len(poses)] for k in ks]))
    stages, _ = hbm_stages(stage_ms, int(g["means"].shape[0]), S, M, 2048, 1024, ceilings)
    seam = seam_fractions(gd, poses)

    out = dict(metric="ERP fwd+bwd iters/s @1M Gaussians 2048x1024", value=args.steps / dt, unit="iters/s",
               n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=dt * 1e3 / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload="1M Gaussians, room layout (20% of them in a 2-degree wedge at world longitude "
                                    f"pi; at random yaw {100 * seam['mean']:.1f}% of the visible ones cross the "
                                    "seam), SH degree 3, 2048x1024 ERP, 200 poses, forward + L1 + backward per pose",
                           gaussians=int(g["means"].shape[0]), width=2048, height=1024, poses=len(poses),
                           forward="caller capacities, no host read-back (overflow checked: none)",
                           instance_capacity=cap[0], entry_capacity=cap[1]),
               stage_ms=stage_ms,
               ms_per_step_all_stages_timed=dt_prof * 1e3 / args.steps,
               roofline=roofline, blends=blends, hbm_stages=stages,
               instances_per_step=M, block_entries_per_step=S, seam_fraction=seam, ceilings=ceilings)
    if not args.no_train:
        out["train"] = train_bench(g, poses, targets, min(args.steps, 100), log)
    if not args.no_pinhole:
        out["pinhole"] = pinhole_bench(gd, crops, crop_targets, poses, min(args.steps, 100), log)
    if not args.no_aux:
        out["aux"] = aux_bench(g, gd, masked, min(args.steps, 50), log)
    if not args.no_seam_stress:
        out["seam_stress"] = seam_stress_bench(gd, gt, args.steps, args.warmup, args.poses, log)
    if not args.no_stress:
        out["stress"] = stress_bench(args.stress_steps, log, ceilings)
    if not args.no_serve:
        out["serving"] = serving_bench(gd, args.serve_requests, args.serve_slots, args.serve_max_batch, log)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, 3 poses)...")
        out["cpu_baseline"] = cpu_baseline(g, poses[:3], [t.cpu().numpy().astype(np.float64) for t in targets[:3]])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

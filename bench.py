"""Benchmark of the S-BKI per-scan map update on one MI355X.

Workload: one spinning-LiDAR-shaped scan (64 beams x 2048 azimuth steps,
~1.29e5 labelled hits, free samples every 0.3 m, ~4.0e6 training rows),
K = 20, 0.1 m voxels in 8^3 blocks, l = 0.3 m, sigma0 = 0.1.  Data is
synthetic and seeded (scenes.make_config(1)).

A step is one pass of the per-scan path into a fresh map: clear the map,
validate the scan, generate free samples, bucket (keys + radix sort + block
tables), splat the rows' kernel weights Eq. (7)-(8) onto the voxel centroids
of their (class, block) regions, allocate blocks, merge the partial sums into
the map, and read out Eq. (3)-(4) at the voxels of the scan's hits.  Inputs
are resident in HBM before timing starts.

metric value = voxel updates per second = V / (time per step), V = voxels
with at least one training row within l.  Also reported: input points/s, the
roofline fraction of the dominant kernel (the splat, VALU-bound) and of the
whole step, the copy bandwidth of the device, the model variants (counting
model, soft measurements, per-class kernels, extended block), the batched town
(64 scans: sequential, one batched insert, the batched insert replayed as a
recorded HIP graph), the stereo sequence (100 scans into one map, per-scan
times), the differentiable form's forward/backward times on the LiDAR scan and
on the tiny scene, and the CPU oracle on the host's cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

VALU_PEAK = 256 * 64 * 2.4e9          # non-packed FP32 VALU lane-operations per second
HBM_PEAK = 8.0e12                     # bytes per second
OPS_PER_PAIR = 24                     # algorithmic VALU lane-operations per in-support pair


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu():
    """Host CPU model and the threads this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return model, n


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the differentiable-form lines and the steps without timing events")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the S-CSM, extended-block and soft-measurement lines")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-scan batched line")
    ap.add_argument("--no-stereo", action="store_true", help="skip the 100-scan stereo line")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer 5 times (scale for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import scenes
    # every workload is generated before the GPU is touched (the stereo
    # sequence casts its scans in forked worker processes)
    t0 = time.time()
    sc = scenes.make_config(1)
    s = sc.scans[0]
    p = sc.params
    log(f"[bench] lidar scan generated in {time.time() - t0:.1f}s: {s.xyz.shape[0]} hits")
    town = stereo = None
    if not args.no_batched and not args.copy_calibration:
        t0 = time.time()
        town = scenes.make_config(3)
        log(f"[bench] town generated in {time.time() - t0:.1f}s: {len(town.scans)} scans")
    if not args.no_stereo and not args.copy_calibration:
        t0 = time.time()
        stereo = scenes.make_config(2, workers=min(16, host_cpu()[1]))
        log(f"[bench] stereo sequence generated in {time.time() - t0:.1f}s: "
            f"{len(stereo.scans)} scans")

    import torch
    from paper_1909_04631_amd import SemanticMap

    torch.cuda.init()
    dev = torch.device("cuda", 0)
    if args.copy_calibration:
        n = args.copy_calibration << 18          # float32 elements
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n}))
        return
    xyz = torch.from_numpy(s.xyz).to(dev)
    lab = torch.from_numpy(s.label).to(dev)
    vox = torch.from_numpy(np.floor(s.xyz / np.float32(p.res)).astype(np.int32)).to(dev)
    B_l, ub_l = tuned("lidar", p)
    m = SemanticMap(p.res, B_l, p.l, p.sigma0, p.K, p.alpha0, p.free_class,
                    initial_blocks=1 << 15, unit_budget=ub_l)
    stream = torch.cuda.current_stream()

    def step():
        m.reset()
        m.insert_scan(xyz, lab, s.origin, p.free_step)
        return m.query(vox, alpha=False, var=False, mean=True, label=True, p_occ=True)

    for i in range(args.warmup):
        step()
        log(f"[bench] warmup {i + 1}/{args.warmup}")
    torch.cuda.synchronize()
    st = m.stats()
    log(f"[bench] stats {st}")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    w0 = time.perf_counter()
    for i in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    # the splat and merge times of these steps (the last 64 at most), from the
    # HIP events the library records around them on the map's stream, read
    # after the loop so that the timed region holds no extra synchronisation
    splat_ms, merge_ms = m.kernel_times(min(args.steps, 64))
    assert len(splat_ms) == min(args.steps, 64)
    ev_ms = e0.elapsed_time(e1)
    ms = max(ev_ms, 1e3 * wall) / args.steps
    # the same steps without the insert's timing events (outside the timed
    # region; what an insert costs when nobody asks for kernel times; not in
    # the profiling runs, which trace the timed steps only)
    ms_no_events = None
    if not args.no_extras:
        m.set_kernel_timing(False)
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        f0.record(stream)
        for i in range(args.steps):
            step()
        f1.record(stream)
        torch.cuda.synchronize()
        m.set_kernel_timing(True)
        ms_no_events = f0.elapsed_time(f1) / args.steps
    log(f"[bench] {args.steps} steps: {ms:.3f} ms/step (events {ev_ms / args.steps:.3f}, "
        f"wall {1e3 * wall / args.steps:.3f}); splat {np.mean(splat_ms):.3f} ms, "
        f"alloc+merge {np.mean(merge_ms):.3f} ms")
    V, P = st["n_updated_voxels"], st["n_pairs"]
    value = V / (ms * 1e-3)
    g_ms = float(np.mean(splat_ms))
    achieved = OPS_PER_PAIR * P / (g_ms * 1e-3)
    copy_bw = copy_bandwidth(torch, dev)
    # whole step against its roof: algorithmic bytes (hits read once, every updated
    # voxel's K float32 concentrations read and written once) and VALU work
    b_alg = 16.0 * st["n_hits"] + 8.0 * p.K * V
    t_roof = max(b_alg / HBM_PEAK, OPS_PER_PAIR * P / VALU_PEAK)
    out = {
        "metric": "voxel updates/sec per scan (1 GPU)",
        "value": value,
        "unit": "voxel updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded ray-cast street scene, LiDAR-shaped)",
        "config": {
            "workload": f"lidar_scan_64x2048_K20_res0.1_B{B_l}_l0.3_s0.1_step0.3",
            "block_size": B_l, "unit_budget": ub_l,
            "hits": st["n_hits"], "free_samples": st["n_free"], "voxels_updated": V,
            "pairs_in_support": P, "blocks_allocated": st["n_new_blocks"],
            "splat_units": st["n_units"], "stencil_lane_util": st["n_candidates"] / max(st["n_lane_slots"], 1),
        },
        "points_per_s": st["n_hits"] / (ms * 1e-3),
        "roofline": {
            "kernel": "k_splat",
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": VALU_PEAK / 1e12,
            "unit": "T VALU lane-op/s",
            "frac": achieved / VALU_PEAK,
            "traffic": None,
            "kernel_ms": g_ms,
            "merge_ms": float(np.mean(merge_ms)),
            "ops_per_pair": OPS_PER_PAIR,
        },
        "step_roofline": {"t_roof_ms": 1e3 * t_roof, "t_step_ms": ms, "frac": 1e3 * t_roof / ms,
                          "algorithmic_bytes": b_alg, "algorithmic_valu_ops": OPS_PER_PAIR * P},
        "hbm": {"peak_GBps": HBM_PEAK / 1e9, "copy_GBps": copy_bw / 1e9},
        "ms_per_step_without_timing_events": ms_no_events,
    }

    out["roofline"]["traffic"] = splat_traffic()
    kt = kernel_table(st, p, copy_bw)
    if kt is not None:
        out["kernels"] = kt
    if not args.no_variants:
        out["scsm"] = bench_scsm(torch, m, xyz, lab, vox, s, p, SemanticMap, args.steps)
        out["face_blocks"] = bench_face_blocks(torch, m, xyz, lab, vox, s, p, SemanticMap,
                                               args.steps)
        out["soft"] = bench_soft(torch, xyz, vox, s, p, SemanticMap, args.steps)
        out["per_class"] = bench_per_class(torch, xyz, lab, vox, s, p, SemanticMap, args.steps)
    if not args.no_extras:
        out["fwd_bwd"] = bench_loss_lidar(torch, dev, sc)
        from paper_1909_04631_amd import predictive_loss
        out["fwd_bwd_tiny"] = bench_loss(torch, dev, predictive_loss)
    if town is not None:
        out["batched"] = bench_batched(torch, dev, SemanticMap, town)
    if stereo is not None:
        out["stereo"] = bench_stereo(torch, dev, SemanticMap, stereo)
    del m
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, V)
    print(json.dumps(out), flush=True)


def tuned(workload, p):
    """(block size, unit budget) the autotuner chose for a workload
    (paper_1909_04631_amd/tuned.json), else the workload's own block size and
    the library's default unit budget."""
    from paper_1909_04631_amd import autotune
    s = autotune.settings(workload)
    return (int(s[0]), int(s[1])) if s else (int(p.block_size), 0)


def copy_bandwidth(torch, dev, mib=1024, reps=10):
    """Achievable HBM bandwidth: a device-to-device copy of mib MiB (bytes read +
    written per second), timed with events."""
    n = mib << 18
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) * 1e-3 / reps
    del src, dst
    return 8.0 * n / sec


def bench_loss_lidar(torch, dev, sc, reps=10):
    """Differentiable form on the LiDAR scan with a seeded 20 % of hits held out
    (their beams removed): forward with alpha kept for backward, the same
    forward without keeping it (plain), and the backward (d/dl, d/dsigma0,
    d/dx of every training row and query), each timed with events on the
    stream with a preallocated workspace."""
    import scenes
    from paper_1909_04631_amd import free_samples
    from paper_1909_04631_amd.loss import loss_backward, loss_forward, workspace
    d = scenes.differentiable_scene(seed=1, base=sc)
    p = d.params
    tr = d.scans[0]
    txh = torch.from_numpy(tr.xyz).to(dev)
    tyh = torch.from_numpy(tr.label).to(dev)
    fq, _ = free_samples(txh, tyh, tr.origin, p.free_step, p.K)
    tx = torch.cat([txh, fq]).contiguous()
    ty = torch.cat([tyh, torch.full((fq.shape[0],), p.free_class, dtype=torch.int32,
                                    device=dev)]).contiguous()
    qx = torch.from_numpy(d.holdout.xyz).to(dev)
    qy = torch.from_numpy(d.holdout.label).to(dev)
    ws = workspace(tx.shape[0], qx.shape[0], p.K, dev)
    l, s0, a0, K = float(np.float32(p.l)), float(np.float32(p.sigma0)), float(np.float32(p.alpha0)), p.K
    g1 = torch.ones((1,), dtype=torch.float32, device=dev)
    _, aq = loss_forward(tx, ty, qx, qy, l, s0, a0, K, ws=ws)

    def timeit(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    t_plain = timeit(lambda: loss_forward(tx, ty, qx, qy, l, s0, a0, K, keep_alpha=False, ws=ws))
    t_fwd = timeit(lambda: loss_forward(tx, ty, qx, qy, l, s0, a0, K, ws=ws))
    t_bwd = timeit(lambda: loss_backward(tx, ty, qx, qy, l, s0, a0, K, aq, g1, ws=ws))
    log(f"[bench] lidar loss: fwd {t_fwd:.2f} ms, bwd {t_bwd:.2f} ms, plain {t_plain:.2f} ms")
    return {"workload": "lidar scan, 20% of hits held out (beams removed), K=20",
            "train_rows": int(tx.shape[0]), "queries": int(qx.shape[0]),
            "t_fwd_ms": t_fwd, "t_bwd_ms": t_bwd, "t_plain_ms": t_plain,
            "bwd_over_fwd": t_bwd / t_fwd, "fwd_bwd_over_plain": (t_fwd + t_bwd) / t_plain}


def bench_stereo(torch, dev, SemanticMap, stereo):
    """The stereo sequence: every scan inserted into one persistent map, each
    insert timed with events on the stream (its host waits included)."""
    p = stereo.params
    B_s, ub_s = tuned("stereo", p)
    m = SemanticMap(p.res, B_s, p.l, p.sigma0, p.K, p.alpha0, p.free_class,
                    initial_blocks=1 << 17, unit_budget=ub_s)
    stream = torch.cuda.current_stream()
    xyz = [torch.from_numpy(x.xyz).to(dev) for x in stereo.scans]
    lab = [torch.from_numpy(x.label).to(dev) for x in stereo.scans]
    # warm-up on a separate map (same shapes)
    w = SemanticMap(p.res, B_s, p.l, p.sigma0, p.K, p.alpha0, p.free_class,
                    initial_blocks=1 << 17, unit_budget=ub_s)
    for i in range(2):
        w.insert_scan(xyz[i], lab[i], stereo.scans[i].origin, p.free_step)
    torch.cuda.synchronize()
    del w
    ms, V, H, P = [], [], [], []
    for i, sc in enumerate(stereo.scans):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        m.insert_scan(xyz[i], lab[i], sc.origin, p.free_step)
        b.record(stream)
        st = m.stats()
        ms.append(a.elapsed_time(b))
        V.append(st["n_updated_voxels"])
        H.append(st["n_hits"])
        P.append(st["n_pairs"])
    ms = np.array(ms)
    splat_ms, _ = m.kernel_times(64)
    tot = ms.sum() * 1e-3
    log(f"[bench] stereo: {len(ms)} scans, median {np.median(ms):.2f} ms, max {ms.max():.2f} ms")
    return {"workload": "stereo_1242x375_100scans_K11_res0.1_l0.3_s0.1_step0.3",
            "block_size": B_s, "unit_budget": ub_s,
            "scans": len(ms), "hits_per_scan_mean": float(np.mean(H)),
            "ms_per_scan_median": float(np.median(ms)), "ms_per_scan_max": float(ms.max()),
            "ms_per_scan_mean": float(ms.mean()),
            "voxel_updates_per_s": float(np.sum(V) / tot), "points_per_s": float(np.sum(H) / tot),
            "pairs_per_scan_mean": float(np.mean(P)),
            "splat_frac_of_valu_peak": float(OPS_PER_PAIR * np.sum(P[-len(splat_ms):]) /
                                             (np.sum(splat_ms) * 1e-3) / VALU_PEAK)}


def bench_loss(torch, dev, predictive_loss, reps=20):
    """Differentiable form on the tiny scene with 20 % of hits held out."""
    import scenes
    sc = scenes.make_config(4)
    p = sc.params
    tr = sc.scans[0]
    from paper_1909_04631_amd import free_samples
    txh = torch.from_numpy(tr.xyz).to(dev)
    tyh = torch.from_numpy(tr.label).to(dev)
    fq, _ = free_samples(txh, tyh, tr.origin, p.free_step, p.K)
    tx = torch.cat([txh, fq]).contiguous()
    ty = torch.cat([tyh, torch.zeros(fq.shape[0], dtype=torch.int32, device=dev)]).contiguous()
    qx = torch.from_numpy(sc.holdout.xyz).to(dev)
    qy = torch.from_numpy(sc.holdout.label).to(dev)
    l = torch.tensor(p.l, device=dev, requires_grad=True)
    s0 = torch.tensor(p.sigma0, device=dev, requires_grad=True)
    txg = tx.clone().requires_grad_(True)

    def timeit(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t) / reps

    def plain():
        with torch.no_grad():
            return predictive_loss(tx, ty, qx, qy, l, s0, p.alpha0, p.K)

    def fwd():
        return predictive_loss(txg, ty, qx, qy, l, s0, p.alpha0, p.K)

    def fwd_bwd():
        L = predictive_loss(txg, ty, qx, qy, l, s0, p.alpha0, p.K)
        L.backward()
        return L

    t_plain = timeit(plain)
    t_fwd = timeit(fwd)
    t_fb = timeit(fwd_bwd)
    t_bwd = max(t_fb - t_fwd, 0.0)
    return {"workload": "tiny scene, 20% of hits held out (1600 hits + free samples, 400 queries)",
            "train_rows": int(tx.shape[0]), "queries": int(qx.shape[0]),
            "t_fwd_ms": t_fwd, "t_bwd_ms": t_bwd, "t_plain_ms": t_plain,
            "bwd_over_fwd": t_bwd / t_fwd if t_fwd > 0 else None,
            "fwd_bwd_over_plain": t_fb / t_plain if t_plain > 0 else None}


def bench_scsm(torch, m_bki, xyz, lab, vox, s, p, SemanticMap, steps):
    """The counting model (Eq. 2) on the same scan and step (reset, insert, readout)."""
    m = SemanticMap.from_params(p, initial_blocks=1 << 15, model="scsm")

    def step():
        m.reset()
        m.insert_scan(xyz, lab, s.origin, p.free_step)
        return m.query(vox, alpha=False, var=False, mean=True, label=True, p_occ=True)

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t) / steps
    st = m.stats()
    return {"model": "S-CSM (Eq. 2)", "ms_per_step": ms, "voxels_updated": st["n_updated_voxels"],
            "voxel_updates_per_s": st["n_updated_voxels"] / (ms * 1e-3),
            "points_per_s": st["n_hits"] / (ms * 1e-3)}


def bench_soft(torch, xyz, vox, s, p, SemanticMap, steps):
    """Soft measurements (Sec. VI) on the same scan: every hit carries a
    classifier-like weight vector truncated to its 3 largest classes."""
    import scenes
    probs = torch.from_numpy(scenes.soft_measurements(s.label, p.K, seed=1, top=3)).to(xyz.device)
    m = SemanticMap.from_params(p, initial_blocks=1 << 15)

    def step():
        m.reset()
        m.insert_scan_soft(xyz, probs, s.origin, p.free_step)
        return m.query(vox, alpha=False, var=False, mean=True, label=True, p_occ=True)

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t) / steps
    st = m.stats()
    return {"measurements": "soft, top-3 class weights per hit", "ms_per_step": ms,
            "hit_rows": st["n_hits"], "voxels_updated": st["n_updated_voxels"],
            "voxel_updates_per_s": st["n_updated_voxels"] / (ms * 1e-3),
            "pairs_in_support": st["n_pairs"], "splat_ms": st["splat_ms"],
            "merge_ms": st["merge_ms"]}


def bench_per_class(torch, xyz, lab, vox, s, p, SemanticMap, steps):
    """Per-class kernels on the same scan: l_k from 0.2 to 0.3 m and sigma0_k
    from 0.05 to 0.2 (seeded); the stencil follows the largest l_k."""
    rng = np.random.default_rng(20)
    lk = rng.choice([0.2, 0.25, 0.3], p.K).tolist()
    lk[p.free_class] = 0.3
    sk = rng.choice([0.05, 0.1, 0.2], p.K).tolist()
    m = SemanticMap.from_params(p, initial_blocks=1 << 15)
    m.set_class_params(lk, sk)

    def step():
        m.reset()
        m.insert_scan(xyz, lab, s.origin, p.free_step)
        return m.query(vox, alpha=False, var=False, mean=True, label=True, p_occ=True)

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t) / steps
    st = m.stats()
    return {"kernels": "per class, l_k in {0.2, 0.25, 0.3}, sigma0_k in {0.05, 0.1, 0.2}",
            "ms_per_step": ms, "voxels_updated": st["n_updated_voxels"],
            "voxel_updates_per_s": st["n_updated_voxels"] / (ms * 1e-3),
            "pairs_in_support": st["n_pairs"], "splat_ms": st["splat_ms"],
            "merge_ms": st["merge_ms"]}


def bench_face_blocks(torch, m_exact, xyz, lab, vox, s, p, SemanticMap, steps):
    """The paper's extended-block selection on the same scan: its time, and how
    far its concentrations depart from the exact support at the hit voxels."""
    m = SemanticMap.from_params(p, initial_blocks=1 << 15, selection="face_blocks")

    def step():
        m.reset()
        m.insert_scan(xyz, lab, s.origin, p.free_step)
        return m.query(vox, alpha=False, var=False, mean=True, label=True, p_occ=True)

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t) / steps
    st = m.stats()
    m_exact.reset()
    m_exact.insert_scan(xyz, lab, s.origin, p.free_step)
    a_face = m.query(vox, mean=False, var=False, label=True, p_occ=False)
    a_ex = m_exact.query(vox, mean=False, var=False, label=True, p_occ=False)
    rel = ((a_face["alpha"] - a_ex["alpha"]).abs() / a_ex["alpha"]).max(dim=1).values
    return {"selection": "own block + 6 face-adjacent blocks", "ms_per_step": ms,
            "voxels_updated": st["n_updated_voxels"],
            "voxel_updates_per_s": st["n_updated_voxels"] / (ms * 1e-3),
            "hit_voxels_changed_frac": float((rel > 1e-6).float().mean()),
            "hit_voxels_max_rel_alpha_drop": float(rel.max()),
            "hit_voxels_label_changed_frac": float((a_face["label"] != a_ex["label"]).float().mean())}


def splat_traffic():
    """HBM bytes per k_splat launch on this workload from the committed counter
    profile (FETCH_SIZE and WRITE_SIZE, each scaled by a 1 GiB copy measured the
    same way), or None when the kernel source changed since it was taken."""
    import hashlib
    prof = os.path.join(HERE, "profiles", "k_splat_lidar_hbm_traffic.txt")
    src = os.path.join(HERE, "paper_1909_04631_amd", "csrc", "splat.hip")
    if not os.path.exists(prof):
        return None
    fields = {}
    for line in open(prof):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            fields[k.strip()] = v.strip()
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if fields.get("splat_hip_sha256") != digest or "hbm_bytes_per_launch" not in fields:
        return None
    return float(fields["hbm_bytes_per_launch"])


def bench_batched(torch, dev, SemanticMap, town, reps=3):
    """64 scans of a synthetic town (U[10k, 130k] hits each), each form into a
    fresh map: 64 sequential inserts, one batched insert, and the batched insert
    recorded as a HIP graph and replayed (no host synchronisation inside).
    V = sum over scans of each scan's updated voxels (from the sequential run)."""
    sc = town
    p = sc.params
    xyz = [torch.from_numpy(s.xyz).to(dev) for s in sc.scans]
    lab = [torch.from_numpy(s.label).to(dev) for s in sc.scans]
    cat_xyz, cat_lab = torch.cat(xyz).contiguous(), torch.cat(lab).contiguous()
    offs = [0]
    for s in sc.scans:
        offs.append(offs[-1] + s.xyz.shape[0])
    origins = [s.origin for s in sc.scans]
    B_t, ub_t = tuned("town", p)
    m = SemanticMap(p.res, B_t, p.l, p.sigma0, p.K, p.alpha0, p.free_class,
                    initial_blocks=1 << 18, unit_budget=ub_t)

    def sequential():
        m.reset()
        v = 0
        for i, s in enumerate(sc.scans):
            m.insert_scan(xyz[i], lab[i], s.origin, p.free_step)
            v += m.stats()["n_updated_voxels"]
        return v

    def batched():
        m.reset()
        m.insert_scans(cat_xyz, cat_lab, offs, origins, p.free_step)

    def timed(fn, n):
        r = fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t = time.perf_counter()
        a.record()
        for _ in range(n):
            r = fn()
        b.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / n
        return max(wall, a.elapsed_time(b) * 1e-3 / n), r

    t_seq, V = timed(sequential, reps)
    t_bat, _ = timed(batched, reps)
    st = m.stats()
    splat_ms, merge_ms = m.kernel_times(reps)
    # the recorded form: captured after one ordinary batched insert, replayed
    m.reset()
    g = m.batch_capture(cat_xyz, cat_lab, offs, origins, p.free_step)
    torch.cuda.synchronize()

    def replay():
        m.reset()
        g.replay(offs, origins)

    t_graph, _ = timed(replay, 2 * reps)
    m.sync()
    sg = m.stats()
    assert sg["n_updated_voxels"] == st["n_updated_voxels"] and sg["n_pairs"] == st["n_pairs"]
    g.close()
    sp = float(np.mean(splat_ms))
    log(f"[bench] batched: graph {t_graph * 1e3:.1f} ms, batched {t_bat * 1e3:.1f} ms, "
        f"sequential {t_seq * 1e3:.1f} ms")
    return {"workload": "town_64_scans_K20_res0.2_l0.3_s0.1_step0.3",
            "block_size": B_t, "unit_budget": ub_t,
            "hits": int(offs[-1]), "rows": int(st["n_hits"] + st["n_free"]),
            "voxel_updates_sum_over_scans": int(V), "voxels_updated_union": int(st["n_updated_voxels"]),
            "t_graph_replay_ms": t_graph * 1e3, "t_batched_ms": t_bat * 1e3,
            "t_sequential_ms": t_seq * 1e3,
            "graph_voxel_updates_per_s": V / t_graph, "batched_voxel_updates_per_s": V / t_bat,
            "sequential_voxel_updates_per_s": V / t_seq,
            "points_per_s_graph": offs[-1] / t_graph,
            "speedup_graph_vs_sequential": t_seq / t_graph, "speedup": t_seq / t_bat,
            "batched_splat_ms": sp, "batched_merge_ms": float(np.mean(merge_ms)),
            "splat_roofline": {"bound": "alu", "achieved": OPS_PER_PAIR * st["n_pairs"] / (sp * 1e-3) / 1e12,
                               "peak": VALU_PEAK / 1e12, "unit": "T VALU lane-op/s",
                               "frac": OPS_PER_PAIR * st["n_pairs"] / (sp * 1e-3) / VALU_PEAK,
                               "pairs_in_support": int(st["n_pairs"])}}


def kernel_table(st, p, copy_bw):
    """Per-kernel achieved HBM bandwidth of the LiDAR step's bucketing, merge and
    readout kernels: algorithmic bytes per launch (from this run's counts) over
    the mean durations of the committed kernel trace of the same workload, as a
    fraction of the 8 TB/s peak and of the measured copy bandwidth; None when
    the trace is missing or older than the sources it names."""
    import hashlib
    import re
    prof = os.path.join(HERE, "profiles", "lidar_scan_kernel_trace.txt")
    if not os.path.exists(prof):
        return None
    fields, dur = {}, {}
    for line in open(prof):
        line = line.strip()
        if line.startswith("#") or not line:
            continue
        if line.startswith("|"):   # | kernel | calls | avg_us | ...
            cells = [c.strip() for c in line.strip("|").split("|")]
            name = re.search(r"\b(k_\w+)", cells[0]) if cells else None
            if name and len(cells) >= 3:
                try:
                    dur.setdefault(name.group(1), float(cells[2]))
                except ValueError:
                    pass
        elif "=" in line:
            k, v = line.split("=", 1)
            fields[k.strip()] = v.strip()
    srcdir = os.path.join(HERE, "paper_1909_04631_amd", "csrc")
    digest = hashlib.sha256(b"".join(open(os.path.join(srcdir, f), "rb").read()
                                     for f in sorted(os.listdir(srcdir)))).hexdigest()
    if fields.get("csrc_sha256") != digest:
        return None
    nh, nf = st["n_hits"], st["n_free"]
    nt = nh + nf
    V = st["n_updated_voxels"]
    # algorithmic bytes per launch
    alg = {
        "k_count": 16.0 * nh + 12.0 * nh,                  # read xyz+label, write counts/flags
        "k_free_keys": 24.0 * nf,                          # write key, index, record per sample
        "k_hit_keys": 16.0 * nh + 24.0 * nh,
        "k_hist": 4.0 * nt,                                # one key read per row
        "k_scatter": 16.0 * nt,                            # key + index in and out
        "k_query": 12.0 * nh + 4.0 * (2 * p.K + 2) * nh,   # ijk in; K alpha read, mean out, label, p_occ
        "k_merge": 8.0 * p.K * V,                          # every updated voxel's alpha read + written
    }
    out = {}
    for k, b in alg.items():
        us = dur.get(k)
        if us:
            out[k] = {"algorithmic_bytes": b, "mean_us": us, "GBps": b / (us * 1e-6) / 1e9,
                      "frac_of_peak": b / (us * 1e-6) / HBM_PEAK,
                      "frac_of_copy": b / (us * 1e-6) / copy_bw}
    return {"source": "profiles/lidar_scan_kernel_trace.txt", "per_kernel": out}


def cpu_baseline(sc, V_full, stride=4):
    """The oracle's map update (plain double-precision C, split over voxel-column
    tiles with OpenMP; the same sums in the same order at any thread count) on
    the host: the whole scan with every thread, and every stride-th beam with
    one thread (scaled to the scan by training rows)."""
    import oracle
    model, ncpu = host_cpu()
    p = sc.params.f32()
    s = sc.scans[0]
    oracle.set_num_threads(ncpu)
    threads = oracle.num_threads()
    om = oracle.OracleMap.from_params(p)
    t = time.perf_counter()
    om.insert_scan(s.xyz, s.label, s.origin, p.free_step, p.free_class)
    T_all = time.perf_counter() - t
    del om
    sub = slice(0, None, stride)
    _, nf_full = oracle.free_counts(s.xyz, s.label, s.origin, p.free_step, p.K)
    _, nf_sub = oracle.free_counts(s.xyz[sub], s.label[sub], s.origin, p.free_step, p.K)
    rows_full = s.xyz.shape[0] + nf_full
    rows_sub = s.xyz[sub].shape[0] + nf_sub
    oracle.set_num_threads(1)
    om = oracle.OracleMap.from_params(p)
    t = time.perf_counter()
    om.insert_scan(s.xyz[sub], s.label[sub], s.origin, p.free_step, p.free_class)
    T1 = time.perf_counter() - t
    oracle.set_num_threads(ncpu)
    T1_full = T1 * rows_full / rows_sub
    log(f"[bench] cpu oracle: full scan {T_all:.2f}s on {threads} threads; "
        f"1 thread est. {T1_full:.1f}s")
    return {"value": V_full / T_all, "unit": "voxel updates/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole scan ({rows_full} training rows) on {threads} threads, "
                      f"{T_all:.2f} s",
            "cpu_model": model, "seconds_full_scan": T_all,
            "points_per_s": s.xyz.shape[0] / T_all,
            "one_thread": {"sample": f"every {stride}th beam ({rows_sub} of {rows_full} rows), "
                                     f"{T1:.2f} s, scaled by training rows",
                           "seconds_full_scan_est": T1_full,
                           "value": V_full / T1_full}}


if __name__ == "__main__":
    main()

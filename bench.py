#!/usr/bin/env python3
"""Benchmark of the per-frame mapping path on one MI355X.

Workload: the 64-beam street sequence (64x2048 range images, +2/-24.8 deg, 100 m, four
1280x720 label cameras with 19 classes, 0.1 m voxels, 0.3 m truncation, 10 Hz at 1 m/s),
synthetic and seeded.  One step = one frame of the whole path: block allocation + TSDF
integration of the scan, label fusion of the four images, and marching cubes of the dirty
blocks (the triangle count is read back, as a caller must).  Inputs are uploaded to HBM
before the timed region.

Printed (one JSON line): voxel-updates/s over the timed frames (U_k from an untimed
counting pass of the same frames), ms per frame, per-kernel averages from HIP events on
the launch stream, the HBM roofline of the dominant kernel (algorithmic bytes per launch
over its average duration) and the CPU oracle timed on a bounded sample of the same
frames on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12  # MI355X HBM3E, bytes/s
PROF_EVERY = 8      # timed frames per event-bracketed frame of the dominant kernel group
METRIC = "voxel-updates/s and ms/frame (64-beam scan, 0.1 m voxels) vs oracle"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_frames(w, n, with_labels=True):
    frames = []
    t0 = time.time()
    for k in range(n):
        frames.append(w.frame(k, with_labels=with_labels))
        if (k + 1) % 10 == 0:
            log(f"[bench] generated {k + 1}/{n} frames ({time.time() - t0:.1f} s)")
    return frames


def h2d_inputs(torch, frames, n=20):
    """Upload time of a frame's inputs (range image and label images) from pinned host
    memory to HBM, outside the timed region: the first n frames, one copy per image."""
    host = []
    for f in frames[:n]:
        imgs = [f.range] + [np.ascontiguousarray(l) for _, l, _ in f.cams]
        host.append([torch.from_numpy(a).pin_memory() for a in imgs])
    dev = [[torch.empty_like(h, device="cuda") for h in hs] for hs in host]
    for d, h in zip(dev[0], host[0]):  # first use of the buffers, untimed
        d.copy_(h, non_blocking=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for ds, hs in zip(dev, host):
        for d, h in zip(ds, hs):
            d.copy_(h, non_blocking=True)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / len(host)
    nbytes = sum(h.numel() * h.element_size() for h in host[0])
    return {"bytes_per_frame": nbytes, "ms_per_frame": ms, "GBps": nbytes / (ms * 1e-3) / 1e9,
            "note": "pinned host to HBM, one copy per image; outside the timed region"}


def run_frames(torch, m, w, dev_frames, lidar, cams, ks, pos, lab, stats=False, step_times=None, prof=None):
    """One step per frame k in ks.  prof = (mask, frames): the library's HIP events bracket
    the kernel groups in mask on those frames only."""
    from paper_2412_00291_amd import MAP_MESH_DIRTY
    out = []
    for k in ks:
        rng_d, labs_d, T, Tcs = dev_frames[k]
        sampled = prof is not None and k in prof[1]
        if sampled:
            m.profile(prof[0])
        t0 = time.perf_counter()
        m.integrate_lidar(lidar, rng_d, T)
        m.integrate_labels_multi(cams, labs_d, Tcs)
        st, n = m.extract_mesh(MAP_MESH_DIRTY, pos, lab, None)
        if sampled:
            m.profile(0)
        if step_times is not None:
            step_times.append(time.perf_counter() - t0)
        if stats:
            st2, s = m.stats()
            out.append(s)
    return out


def algorithmic_bytes(kernel, s, rows, cols, cams):
    """Bytes the method must move per frame for one kernel (the HBM-roofline model)."""
    U, V, T, M, Tri = s["updates"], s["votes"], s["touched"], s["mesh_blocks"], s["triangles"]
    if kernel == "tsdf":       # read + write (D, W) per update, the range image, the touched list
        return 16 * U + 4 * rows * cols + 16 * T
    if kernel == "mesh":       # 9^3 halo of (D, W, fused) per block, 3 x (12 B + 1 B) per triangle
        return 6561 * M + 39 * Tri
    if kernel == "labels":     # count r/w, fused r/w, count of the fused label; the label images
        return 8 * V + sum(c.width * c.height for c in cams)
    if kernel == "alloc":      # the range image, one probe + list entry per touched block
        return 4 * rows * cols + 16 * T
    if kernel == "tsdf_labels":  # the TSDF launch with the frame's camera labels fused in
        return algorithmic_bytes("tsdf", s, rows, cols, cams) + algorithmic_bytes("labels", s, rows, cols, cams)
    return 0


def group_ms(prof, k):
    """Milliseconds of a kernel group in a profile read; the TSDF group includes the fused
    TSDF-and-labels launch."""
    if k == "tsdf":
        return prof["tsdf"][0] + prof["tsdf_labels"][0]
    return prof[k][0]


TRAFFIC_JSON = os.path.join("profiles", "street_64x2048_traffic.json")


def kernel_group(name, sch):
    """The kernel group of a rocprofv3 kernel name (instances of the chosen schedules only),
    or None: k_alloc -> alloc; k_tsdf<S, lds, np, lab> -> tsdf_labels when lab != 0, else
    tsdf; k_labels<S, ...> -> labels; k_mesh_count and k_mesh_emit<S> -> mesh."""
    args = name[name.index("<") + 1:name.rindex(">")].replace(" ", "").split(",") if "<" in name else []
    if name.startswith("k_alloc"):
        return "alloc"
    if name.startswith("k_tsdf<"):
        if int(args[0]) != sch["tsdf"]:
            return None
        return "tsdf_labels" if len(args) > 3 and args[3] != "0" else "tsdf"
    if name.startswith("k_labels<"):
        return "labels" if int(args[0]) == sch["labels"] else None
    if name.startswith("k_mesh_count"):
        return "mesh"
    if name.startswith("k_mesh_emit<"):
        return "mesh" if int(args[0]) == sch["mesh"] else None
    return None


def sources_sha256(root):
    """Hash of the kernel sources (csrc *.hip, *.h and the case-table generator)."""
    import hashlib
    csrc = os.path.join(root, "paper_2412_00291_amd", "csrc")
    names = sorted(n for n in os.listdir(csrc) if n.endswith((".hip", ".h"))) + ["gen_mc_table.py"]
    h = hashlib.sha256()
    for n in sorted(os.path.join("paper_2412_00291_amd/csrc", x) for x in names):
        h.update(open(os.path.join(root, n), "rb").read())
    return h.hexdigest()


def _counter_rows(path):
    import csv
    rows = []
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"].replace("void ", "").split("(")[0].replace("mc::", "")
        rows.append((int(r["Dispatch_Id"]), name, float(r["Counter_Value"])))
    rows.sort()
    return rows


def write_traffic(out_dir):
    """Summarise the rocprofv3 FETCH_SIZE / WRITE_SIZE runs under out_dir (pmc_<C>/street_*
    of `bench.py --steps K --warmup W --no-cpu-baseline --no-extensions`, cal_<C>/copy_* of
    `bench.py --calibrate-copy`) into the HBM bytes per launch of each kernel group: the
    last K dispatches of each kernel instance of the schedules that run chose (its
    per-kernel breakdown pass), each counter scaled by the copy calibration."""
    import glob
    bench = json.load(open(os.path.join(out_dir, "pmc_FETCH_SIZE.json")))
    K = bench["steps"]
    sch = bench["schedules"]
    per = {}
    factors = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        cal = _counter_rows(glob.glob(os.path.join(out_dir, f"cal_{c}", "*counter_collection.csv"))[0])
        copy_kib = max(v for _, n, v in cal if "copyBuffer" in n)
        factors[c] = (256 << 10) / copy_kib  # a 256 MiB copy reads and writes 262144 KiB
        rows = _counter_rows(glob.glob(os.path.join(out_dir, f"pmc_{c}", "*counter_collection.csv"))[0])
        by = {}
        for _, n, v in rows:
            by.setdefault(n, []).append(v)
        per[c] = by
    out = {}
    kernels = {}
    for n in per["FETCH_SIZE"]:
        g = kernel_group(n, sch)
        if g is None:
            continue
        f = per["FETCH_SIZE"][n][-K:]
        w = per["WRITE_SIZE"].get(n, [0.0])[-K:]
        fb = 1024 * factors["FETCH_SIZE"] * sum(f) / len(f)
        wb = 1024 * factors["WRITE_SIZE"] * sum(w) / len(w)
        kernels[n] = {"group": g, "fetch_kib": sum(f) / len(f), "write_kib": sum(w) / len(w), "bytes": fb + wb}
        out[g] = out.get(g, 0.0) + fb + wb
    rec = {"workload": "street-64x2048-v0.1", "sources_sha256": sources_sha256(ROOT),
           "fetch_factor": factors["FETCH_SIZE"], "write_factor": factors["WRITE_SIZE"],
           "bytes_per_launch": out, "kernels": kernels, "dispatches_per_kernel": K,
           "schedules": {k: sch[k] for k in ("tsdf", "labels", "mesh")},
           "note": "FETCH_SIZE and WRITE_SIZE KiB per dispatch x the copy-calibrated factors, "
                   "summed over the group's kernels (street_64x2048_traffic.md gives the commands)"}
    path = os.path.join(ROOT, TRAFFIC_JSON)
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def measured_traffic(kernel, sched):
    """HBM bytes per launch of a kernel group from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, or None when the kernel sources (or the group's schedule) differ
    from the ones the counters were taken on."""
    try:
        rec = json.load(open(os.path.join(ROOT, TRAFFIC_JSON)))
    except (OSError, ValueError):
        return None
    if sources_sha256(ROOT) != rec.get("sources_sha256"):
        return None
    if kernel in sched and rec.get("schedules", {}).get(kernel) != sched[kernel]:
        return None
    return rec.get("bytes_per_launch", {}).get(kernel)


def _cpu_run(w, frames, budget_s, variant):
    import oracle
    om = oracle.OracleMap(w.voxel, w.trunc, w.n_classes, w.max_blocks, variant=variant)
    U = 0
    t_total = 0.0
    n = 0
    per_frame = []
    for k, f in enumerate(frames):
        t0 = time.perf_counter()
        om.integrate_lidar(w.lidar, f.range, f.T_wl)
        for T, lab, cam in f.cams:
            om.integrate_labels(cam, lab, T)
        om.extract_mesh(oracle.MESH_DIRTY, with_keys=False)
        t_total += time.perf_counter() - t0
        s = om.stats()
        per_frame.append(s)
        U += s["updates"]
        n += 1
        if t_total >= budget_s:
            break
    om.close()
    return U / t_total, 1e3 * t_total / n, n, per_frame


def campus_oracle(campus):
    """The oracle's OpenMP build on the first campus frames (scan, both label images, dirty
    meshing; room for 200K blocks as on the GPU): each frame's counts against the GPU's, and
    its time per frame on this host."""
    import oracle
    w, host, gpu = campus
    n = len(host)
    om = oracle.OracleMap(w.voxel, w.trunc, w.n_classes, CAMPUS_CHECK_BLOCKS, variant="omp")
    cpu, t = [], 0.0
    for k in range(n):
        rng, labs, Tcs = host[k]
        t0 = time.perf_counter()
        om.integrate_lidar(w.lidar, rng, w.poses[k])
        for c, l, T in zip(w.cameras, labs, Tcs):
            om.integrate_labels(c, l, T)
        om.extract_mesh(oracle.MESH_DIRTY, with_keys=False)
        t += time.perf_counter() - t0
        cpu.append(om.stats())
    om.close()
    keys = ("updates", "votes", "touched", "new_blocks", "mesh_blocks", "triangles", "allocated")
    bad = [(k, key, gpu[k][key], cpu[k][key]) for k in range(n) for key in keys if gpu[k][key] != cpu[k][key]]
    U = sum(s["updates"] for s in cpu)
    return ({"frames": n, "counts": list(keys), "equal": not bad, "mismatches": bad[:5]},
            {"value": U / t, "unit": "voxel-updates/s", "cores": oracle.threads("omp"), "ms_per_frame": 1e3 * t / n,
             "sample": f"campus frames 0-{n - 1} (128x2048 scan, 2 x 1920x1080 label images, dirty mesh), "
                       "OpenMP build"})


def cpu_baseline(w, frames, budget_s, campus=None):
    """The oracle on this host's cores, whole path per frame, on the first frames of the same
    sequence: its OpenMP build (every host thread; loops over rows, touched blocks and meshed
    blocks in parallel, identical results) and its plain single-threaded build; with
    `campus`, also the first campus frames, checked against the GPU's counts."""
    import oracle
    threads = oracle.threads("omp")
    v_omp, ms_omp, n_omp, per_frame = _cpu_run(w, frames, budget_s, "omp")
    v_one, ms_one, n_one, _ = _cpu_run(w, frames, budget_s, "plain")
    extra = {}
    if campus is not None:
        extra["campus_check"], extra["campus"] = campus_oracle(campus)
    return per_frame, extra, {"value": v_omp, "unit": "voxel-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"street frames 0-{n_omp - 1} of the same sequence, whole path per frame "
                      f"(scan + 4 label images + dirty mesh), OpenMP build on {threads} threads",
            "ms_per_frame": ms_omp, "frames": n_omp,
            "single_thread": {"value": v_one, "unit": "voxel-updates/s", "cores": 1, "ms_per_frame": ms_one,
                              "frames": n_one, "sample": f"street frames 0-{n_one - 1}, plain build"},
            "cpu": _cpu_model(), "host_threads_available": len(os.sched_getaffinity(0)),
            **({"campus": extra["campus"]} if "campus" in extra else {})}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_adjoint(torch, reps=5):
    """Differentiation workload: 64 poses x 131072 points against the tiny-scene map."""
    import synth
    from paper_2412_00291_amd import KERNEL_NAMES, LidarModel, Map
    w = synth.tiny_workload()
    f = w.frame(0, with_labels=False)
    m = Map(w.voxel, w.trunc, w.n_classes, w.max_blocks)
    lidar = LidarModel(w.lidar.rows, w.lidar.cols, w.lidar.elev_rad, w.lidar.r_max)
    m.integrate_lidar(lidar, torch.from_numpy(f.range).cuda(), f.T_wl)
    pts = synth.scan_points(w, synth.uniform_lidar(64, 2048, 15.0, -15.0, 40.0), f.T_wl, 131072, seed=4)
    B, N = 64, 131072
    P = torch.from_numpy(np.broadcast_to(pts, (B, N, 3)).copy()).cuda()
    X = torch.from_numpy(synth.perturbed_poses(B, seed=4)).cuda()
    loss = torch.empty(B, device="cuda")
    gxi = torch.empty(B, 6, device="cuda")
    gp = torch.empty_like(P)
    m.sdf_pose_adjoint(X, P, loss, gxi, gp)
    torch.cuda.synchronize()
    m.profile(1 << KERNEL_NAMES.index("adjoint"))
    t0 = time.perf_counter()
    for _ in range(reps):
        m.sdf_pose_adjoint(X, P, loss, gxi, gp)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    prof = m.profile_read()["adjoint"]
    k_ms = prof[0] / max(prof[1], 1)
    bytes_ = B * N * (12 + 12) + B * 6 * 4 * 2  # points in, point gradients out, poses
    m.close()
    return {"workload": "64 poses x 131072 points, tiny-scene map (0.2 m voxels)",
            "ms_per_call": 1e3 * dt, "points_per_s": B * N / dt, "kernel_ms": k_ms,
            "roofline": {"bound": "hbm", "achieved": bytes_ / (k_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                         "unit": "GB/s", "frac": bytes_ / (k_ms * 1e-3) / PEAK_HBM}}


def bench_range_image(torch, reps=50):
    """Measurement preprocessing: raw street point clouds (64 x 2048 scan, one return per
    beam and column plus 10% second returns and 1% invalid points) to depth and height
    images, the clouds resident in HBM."""
    import synth
    from paper_2412_00291_amd import KERNEL_NAMES, LidarModel, Map
    w = synth.street_workload(n_frames=4, n_cams=1)
    lidar = LidarModel(w.lidar.rows, w.lidar.cols, w.lidar.elev_rad, w.lidar.r_max)
    clouds = [torch.from_numpy(synth.cloud_points(w, k, 200 + k)).cuda() for k in range(4)]
    D = torch.empty(w.lidar.rows, w.lidar.cols, device="cuda")
    H = torch.empty_like(D)
    m = Map(w.voxel, w.trunc, w.n_classes, 1 << 12)
    for P in clouds:
        m.range_image(lidar, P, D, H)
    torch.cuda.synchronize()
    m.profile(1 << KERNEL_NAMES.index("range"))
    t0 = time.perf_counter()
    for i in range(reps):
        m.range_image(lidar, clouds[i % 4], D, H)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    prof = m.profile_read()["range"]
    k_ms = prof[0] / max(prof[1], 1)
    n = sum(int(clouds[i % 4].shape[0]) for i in range(reps)) / reps
    bytes_ = 12 * n + 8 * w.lidar.rows * w.lidar.cols  # points in; depth and height out
    m.close()
    return {"workload": "street clouds, 64x2048 scan, ~145k points each", "points": n,
            "ms_per_call": 1e3 * dt, "points_per_s": n / dt, "kernel_ms": k_ms,
            "roofline": {"bound": "hbm", "achieved": bytes_ / (k_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                         "unit": "GB/s", "frac": bytes_ / (k_ms * 1e-3) / PEAK_HBM}}


def bench_lidar_labels(torch, frames=24):
    """Label fusion from label range images (the scan's points labelled by a segmentation
    network): street frames, each integrated (64 x 2048 scan) and then fused with its
    label range image; the label call alone is timed with events."""
    import synth
    from paper_2412_00291_amd import KERNEL_NAMES, LidarModel, Map
    w = synth.street_workload(n_frames=frames, n_cams=1)
    lidar = LidarModel(w.lidar.rows, w.lidar.cols, w.lidar.elev_rad, w.lidar.r_max)
    data = [(torch.from_numpy(w.frame(k, with_labels=False).range).cuda(),
             torch.from_numpy(w.lidar_labels(k)).cuda(), w.poses[k]) for k in range(frames)]
    m = Map(w.voxel, w.trunc, w.n_classes, w.max_blocks)
    votes, warm = 0, 4
    for k, (rng, lab, T) in enumerate(data):
        if k == warm:
            torch.cuda.synchronize()
            m.profile(1 << KERNEL_NAMES.index("labels"))
        m.integrate_lidar(lidar, rng, T)
        m.integrate_labels_lidar(lidar, lab, T)
        if k >= warm:
            votes += m.stats()[1]["votes"]
    prof = m.profile_read()["labels"]
    m.close()
    k_ms = prof[0] / max(prof[1], 1)
    per = votes / max(prof[1], 1)
    bytes_ = 8 * per + w.lidar.rows * w.lidar.cols
    return {"workload": "street frames, 64x2048 label range images, L=19", "frames_timed": frames - warm,
            "votes_per_frame": per, "kernel_ms": k_ms, "votes_per_s": per / (k_ms * 1e-3),
            "roofline": {"bound": "hbm", "achieved": bytes_ / (k_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                         "unit": "GB/s", "frac": bytes_ / (k_ms * 1e-3) / PEAK_HBM}}


def bench_nonprojective(torch, frames=24, warm=4):
    """The paper's own distance (non-projective, Eq. 4): street frames (64x2048 scan, four
    1280x720 label cameras, dirty meshing every frame) into a map in that mode; ms per
    frame over the last frames, and the allocation + TSDF kernels (normal image, point
    filter, gradients) timed with events and priced at their algorithmic bytes."""
    import synth
    from paper_2412_00291_amd import (CameraModel, KERNEL_NAMES, LidarModel, Map, MAP_DIST_NONPROJECTIVE,
                                      MAP_MESH_DIRTY)
    w = synth.street_workload(n_frames=frames)
    lid = LidarModel(w.lidar.rows, w.lidar.cols, w.lidar.elev_rad, w.lidar.r_max)
    cams = [CameraModel(c.width, c.height, c.fx, c.fy, c.cx, c.cy) for c in w.cameras]
    dev = []
    for k in range(frames):
        f = w.frame(k)
        dev.append((torch.from_numpy(f.range).cuda(),
                    [torch.from_numpy(np.ascontiguousarray(l)).cuda() for _, l, _ in f.cams], f.T_wl,
                    [T for T, _, _ in f.cams]))
    cap = 4_000_000
    pos = torch.empty((cap, 3, 3), dtype=torch.float32, device="cuda")
    lab = torch.empty((cap, 3), dtype=torch.uint8, device="cuda")
    m = Map(w.voxel, w.trunc, w.n_classes, w.max_blocks)
    m.set_distance(MAP_DIST_NONPROJECTIVE, float(np.deg2rad(80.0)))
    times, stats = [], []
    mask = sum(1 << KERNEL_NAMES.index(k) for k in ("alloc", "tsdf", "tsdf_labels"))
    for k, (r, labs, T, Tcs) in enumerate(dev):
        if k == warm:
            torch.cuda.synchronize()
            m.profile_read()
        timed_frame = k >= warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.integrate_lidar(lid, r, T)
        m.integrate_labels_multi(cams, labs, Tcs)
        m.extract_mesh(MAP_MESH_DIRTY, pos, lab, None)
        torch.cuda.synchronize()
        if timed_frame:
            times.append(time.perf_counter() - t0)
            stats.append(m.stats()[1])
    # kernel events on a second pass over the same frames (a fresh map)
    m.close()
    m = Map(w.voxel, w.trunc, w.n_classes, w.max_blocks)
    m.set_distance(MAP_DIST_NONPROJECTIVE, float(np.deg2rad(80.0)))
    for k, (r, labs, T, Tcs) in enumerate(dev):
        if k == warm:
            torch.cuda.synchronize()
            m.profile(mask)
        m.integrate_lidar(lid, r, T)
        m.integrate_labels_multi(cams, labs, Tcs)
        m.extract_mesh(MAP_MESH_DIRTY, pos, lab, None)
    prof = m.profile_read()
    m.close()
    R, C = w.lidar.rows, w.lidar.cols
    n = len(stats)
    U = sum(s["updates"] for s in stats)
    Tk = sum(s["touched"] for s in stats)
    V = sum(s["votes"] for s in stats)
    # alloc: range + its two neighbours' rows through the caches (4 B), normal image write
    # (16 B), probe + list per touched block; TSDF: (D, W) and the gradient read and
    # written per update, the normal image read, the touched list; with the frame's camera
    # labels fused into the TSDF launch, the label bytes of the projective model as well
    alloc_b = n * (4 * R * C + 16 * R * C) + 16 * Tk
    tsdf_b = 16 * U + 24 * U + n * 16 * R * C + 16 * Tk
    fused = prof["tsdf_labels"][1] > 0
    if fused:
        tsdf_b += 8 * V + n * sum(c.width * c.height for c in cams)
    out = {"workload": "street-64x2048-v0.1, non-projective distance (Eq. 4), 80 deg point filter, 4 cameras",
           "frames_timed": n, "ms_per_frame_p50": float(np.median(times) * 1e3),
           "ms_per_frame_p90": float(np.percentile(times, 90) * 1e3),
           "voxel_updates_per_s": U / sum(times), "updates_per_frame": U / n,
           "tsdf_launch": "TSDF with the camera labels fused in" if fused else "TSDF"}
    for name, key, b in (("alloc", "alloc", alloc_b), ("tsdf", "tsdf_labels" if fused else "tsdf", tsdf_b)):
        ms, launches = prof[key]
        out[f"{name}_avg_us"] = 1e3 * ms / max(launches, 1)
        out[f"{name}_roofline"] = {"bound": "hbm", "achieved": b / (ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                                   "unit": "GB/s", "frac": b / (ms * 1e-3) / PEAK_HBM}
    return out


def bench_label_modes(torch, frames=12, warm=2):
    """Label fusion modes on street frames: the latest label (four 1280x720 label images
    per frame) and Eq. 6 on two 1280x720x19 fp32 log-probability images per frame; the
    label kernels alone are timed with events and priced at their algorithmic bytes."""
    import synth
    from paper_2412_00291_amd import (CameraModel, KERNEL_NAMES, LidarModel, Map, MAP_LABELS_BAYES,
                                      MAP_LABELS_LATEST)
    w = synth.street_workload(n_frames=frames)
    lid = LidarModel(w.lidar.rows, w.lidar.cols, w.lidar.elev_rad, w.lidar.r_max)
    cams = [CameraModel(c.width, c.height, c.fx, c.fy, c.cx, c.cy) for c in w.cameras]
    hf = [w.frame(k) for k in range(frames)]
    L = w.n_classes
    out = {}
    mask = 1 << KERNEL_NAMES.index("labels")
    # latest label wins: the four label images are fused into the frame's TSDF launch, so
    # that launch is timed and priced at the TSDF bytes plus the label bytes
    fmask = (1 << KERNEL_NAMES.index("tsdf_labels")) | mask
    m = Map(w.voxel, w.trunc, L, w.max_blocks)
    m.set_label_fusion(MAP_LABELS_LATEST)
    dev = [(torch.from_numpy(f.range).cuda(), [torch.from_numpy(np.ascontiguousarray(l)).cuda() for _, l, _ in f.cams],
            f.T_wl, [T for T, _, _ in f.cams]) for f in hf]
    votes = upd = touched = 0
    for k, (r, labs, T, Tcs) in enumerate(dev):
        if k == warm:
            torch.cuda.synchronize()
            m.profile(fmask)
        m.integrate_lidar(lid, r, T)
        m.integrate_labels_multi(cams, labs, Tcs)
        if k >= warm:
            st = m.stats()[1]
            votes += st["votes"]
            upd += st["updates"]
            touched += st["touched"]
    prof = m.profile_read()
    m.close()
    fused = prof["tsdf_labels"][1] > 0
    ms, launches = prof["tsdf_labels"] if fused else prof["labels"]
    b = 2 * votes + launches * sum(c.width * c.height for c in cams)  # fused read + write per vote, images
    if fused:
        b += 16 * upd + launches * 4 * w.lidar.rows * w.lidar.cols + 16 * touched
    out["latest"] = {"workload": "street-64x2048-v0.1, 4 x 1280x720 label images, latest label wins",
                     "kernel": "TSDF with the labels fused in" if fused else "labels",
                     "launches": launches, "kernel_us": 1e3 * ms / max(launches, 1),
                     "votes_per_s": votes / (ms * 1e-3),
                     "roofline": {"bound": "hbm", "achieved": b / (ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                                  "unit": "GB/s", "frac": b / (ms * 1e-3) / PEAK_HBM}}
    del dev
    # Eq. 6 on log-probability images: two cameras (front, back), a 1 M-block map
    m = Map(w.voxel, w.trunc, L, 1 << 20)
    m.set_label_fusion(MAP_LABELS_BAYES)
    hb = hf[:6]
    lp = [[torch.from_numpy(synth.logprob_image(f.cams[i][1], L, seed=7 * k + i)).cuda() for i in (0, 2)]
          for k, f in enumerate(hb)]
    votes = 0
    for k, f in enumerate(hb):
        if k == warm:
            torch.cuda.synchronize()
            m.profile(mask)
        m.integrate_lidar(lid, torch.from_numpy(f.range).cuda(), f.T_wl)
        for j, i in enumerate((0, 2)):
            m.integrate_logprobs(cams[i], lp[k][j], f.cams[i][0])
        if k >= warm:
            votes += m.stats()[1]["votes"]
    ms, launches = m.profile_read()["labels"]
    m.close()
    b = votes * (12 * L + 1)  # log-posteriors read + written, the pixel's vector read, fused write
    out["bayes"] = {"workload": "street-64x2048-v0.1, 2 x 1280x720x19 fp32 log-probability images, Eq. 6",
                    "launches": launches, "kernel_us": 1e3 * ms / max(launches, 1),
                    "votes_per_s": votes / (ms * 1e-3),
                    "roofline": {"bound": "hbm", "achieved": b / (ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                                 "unit": "GB/s", "frac": b / (ms * 1e-3) / PEAK_HBM}}
    return out


_BATCHED = {}


def _one_thread_worker():
    """Frame-generation workers each ray-cast on one thread (the pool supplies the
    parallelism; an OpenMP team per worker would oversubscribe the host)."""
    os.environ["OMP_NUM_THREADS"] = "1"


def _batched_frame(args):
    """One frame of one batched map (worker process): (m, k, range, T_wl, label image, T_wc)."""
    import synth
    m, k = args
    ws = _BATCHED.get("ws")
    if ws is None:
        ws = _BATCHED["ws"] = synth.batched_workloads(seed=3, n_maps=16)
    f = ws[m].frame(k)
    T, lab, _ = f.cams[0]
    return m, k, f.range, f.T_wl, np.ascontiguousarray(lab), T


def batched_max_blocks(voxel):
    """Pool size of a batched map: room for its whole sequence at its voxel size."""
    return {0.05: 1 << 19, 0.1: 1 << 18, 0.2: 1 << 17}.get(round(voxel, 2), 1 << 16)


def bench_batched(torch, workers=None):
    """Batched form at the batched workload's own frame counts: 16 street maps of uneven size
    (voxel 0.05-0.4 m, 16/32/64 beams, 1024-2048 columns, 10-200 frames each, one 1280x720
    camera), autotuned schedule, against the same frames integrated by sequential plain
    calls.  A step integrates one frame into every map that still has frames; the frames
    are generated in worker processes and resident in HBM before the timed runs."""
    import multiprocessing as mp
    import synth
    from paper_2412_00291_amd import Batch, CameraModel, LidarModel, Map, MAP_MESH_DIRTY
    from paper_2412_00291_amd import autotune
    ws = synth.batched_workloads(seed=3, n_maps=16)
    workers = workers or min(16, len(os.sched_getaffinity(0)))
    jobs = [(m, k) for m, w in enumerate(ws) for k in range(w.n_frames)]
    frames = [[None] * w.n_frames for w in ws]
    t0 = time.time()
    with mp.get_context("spawn").Pool(workers, initializer=_one_thread_worker) as pool:
        for i, (m, k, r, T, lab, Tc) in enumerate(pool.imap_unordered(_batched_frame, jobs, chunksize=8)):
            frames[m][k] = (torch.from_numpy(r).cuda(), T, torch.from_numpy(lab).cuda(), Tc)
            if (i + 1) % 500 == 0:
                log(f"[bench] batched: {i + 1}/{len(jobs)} frames generated ({time.time() - t0:.0f} s)")
    data = []
    for m, w in enumerate(ws):
        lid = LidarModel(w.lidar.rows, w.lidar.cols, w.lidar.elev_rad, w.lidar.r_max)
        cam = CameraModel(*(getattr(w.cameras[0], k) for k in ("width", "height", "fx", "fy", "cx", "cy")))
        data.append((w, lid, cam, frames[m]))
    log(f"[bench] batched: {len(jobs)} frames over {len(data)} maps generated")
    torch.cuda.synchronize()
    cap = 1 << 21
    bufs = [(torch.empty((cap, 3, 3), dtype=torch.float32, device="cuda"),
             torch.empty((cap, 3), dtype=torch.uint8, device="cuda")) for _ in data]
    n_steps = max(len(d[3]) for d in data)
    stream = torch.cuda.Stream()

    def items_for(k):
        out = []
        for mi, (w, lid, cam, fr) in enumerate(data):
            if k < len(fr):
                r, T, lab, Tc = fr[k]
                out.append({"map_index": mi, "lidar": lid, "range": r, "T_wl": T, "cams": [cam],
                            "labels": [lab], "T_wc": [Tc], "pos": bufs[mi][0], "lab": bufs[mi][1]})
        return out

    def new_maps():
        return [Map(w.voxel, w.trunc, w.n_classes, batched_max_blocks(w.voxel)) for w, *_ in data]

    def build():
        return Batch(new_maps())

    def run_step(batch, k):
        with torch.cuda.stream(stream):
            batch.step(items_for(k))

    # every candidate runs the whole workload (every step after the first timed, compared by
    # the mean): steps whose maps have run out of frames are part of what a schedule costs
    sig = "street16-seed3-real-" + "-".join(str(len(d[3])) for d in data)
    sched, grid, timings = autotune.tune(sig, build, run_step, n_steps=n_steps - 1, score="mean")
    log(f"[bench] batched: autotuner chose schedule {sched}, grid {grid}")

    # batched, all steps (items prepared beforehand, as a caller holding its frames would);
    # HIP events on the step stream give the device time beside the wall time
    step_items = [items_for(k) for k in range(n_steps)]
    batch = build()
    batch.configure(sched, grid, True)
    with torch.cuda.stream(stream):
        batch.step(step_items[0])  # first step: scratch sizing and graph capture (untimed)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        e0.record(stream)
        for k in range(1, n_steps):
            batch.step(step_items[k])
        e1.record(stream)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    gpu_batch = e0.elapsed_time(e1)
    U = 0
    for m in batch.maps:
        U += m.stats()[1]["allocated"]
    for m in batch.maps:
        m.close()
    batch.close()
    # sequential plain calls over the same frames, on fresh maps
    maps = new_maps()

    def seq_step(k):
        for mi, (w, lid, cam, fr) in enumerate(data):
            if k < len(fr):
                r, T, lab, Tc = fr[k]
                m = maps[mi]
                m.integrate_lidar(lid, r, T)
                m.integrate_labels_multi([cam], [lab], [Tc])
                m.extract_mesh(MAP_MESH_DIRTY, bufs[mi][0], bufs[mi][1], None)

    seq_step(0)
    torch.cuda.synchronize()
    cur = torch.cuda.current_stream()
    t0 = time.perf_counter()
    e0.record(cur)
    for k in range(1, n_steps):
        seq_step(k)
    e1.record(cur)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    gpu_seq = e0.elapsed_time(e1)
    blocks_seq = sum(m.stats()[1]["allocated"] for m in maps)
    frames_timed = sum(max(len(d[3]) - 1, 0) for d in data)
    for m in maps:
        m.close()
    return {"workload": "16 street maps, voxel 0.05-0.4 m, 16/32/64 x 1024-2048, "
                        f"{min(len(d[3]) for d in data)}-{max(len(d[3]) for d in data)} frames each, 1 camera",
            "steps_timed": n_steps - 1, "map_frames_timed": frames_timed,
            "schedule": ({"tsdf": ["workgroup-per-block", "wavefront-per-block"][sched & 1],
                          "labels": ["workgroup-per-block", "wavefront-per-block"][sched >> 1],
                          "meshing": "wavefront-per-block", "grid": grid} if sched < 4 else
                         {"concurrent": "each map's own kernels", "streams": grid}),
            "autotune_ms": {f"{k[0]},{k[1]}": 1e3 * v for k, v in timings.items()},
            "ms_per_step_batched": 1e3 * t_batch / (n_steps - 1),
            "ms_per_step_sequential": 1e3 * t_seq / (n_steps - 1),
            "speedup_vs_sequential": t_seq / t_batch,
            "stream_ms_per_step_batched": gpu_batch / (n_steps - 1),
            "stream_ms_per_step_sequential": gpu_seq / (n_steps - 1),
            "ms_per_map_frame_batched": 1e3 * t_batch / frames_timed,
            "ms_per_map_frame_sequential": 1e3 * t_seq / frames_timed,
            "allocated_blocks_end": {"batched": U, "sequential": blocks_seq}}


_CAMPUS = {}


def _campus_frame(args):
    """One campus frame (worker process): (k, range, [label images]) with or without labels."""
    import synth
    k, n_frames, with_labels = args
    w = _CAMPUS.get(n_frames)
    if w is None:
        w = _CAMPUS[n_frames] = synth.campus_workload(n_frames=n_frames)
    f = w.frame(k, with_labels=with_labels)
    return k, f.range, [np.ascontiguousarray(l) for _, l, _ in f.cams], [T for T, _, _ in f.cams]


def bench_campus(torch, warm=1300, timed=200, window=100, n_check=30, workers=None):
    """Large-scale form: 128x2048 scans and two 1920x1080 cameras on the campus loop, in a
    map with room for 2M blocks (~50 GB).  Frames 0..warm-1 grow the map (scan and dirty
    meshing; no labels); meshing alone is timed with events over two windows of the growth,
    early (frames 300-399) and late (the last `window` growth frames), to compare its cost
    per meshed block at two map sizes.  Then frames warm..warm+timed-1 (scan, both label
    images, dirty meshing) are timed one by one, wall clock: the steady state once the map
    has grown.  The frames are generated in worker processes before the GPU work and
    uploaded to HBM first."""
    import multiprocessing as mp
    import synth
    from paper_2412_00291_amd import CameraModel, KERNEL_NAMES, LidarModel, Map, MAP_MESH_DIRTY
    n = warm + timed
    w = synth.campus_workload(n_frames=n)
    lid = LidarModel(w.lidar.rows, w.lidar.cols, w.lidar.elev_rad, w.lidar.r_max)
    cams = [CameraModel(c.width, c.height, c.fx, c.fy, c.cx, c.cy) for c in w.cameras]
    workers = workers or min(16, len(os.sched_getaffinity(0)))
    t0 = time.time()
    frames = {}
    with mp.get_context("spawn").Pool(workers, initializer=_one_thread_worker) as pool:
        jobs = [(k, n, k >= warm or k < n_check) for k in range(n)]
        host = {}
        for k, rng, labs, Tcs in pool.imap_unordered(_campus_frame, jobs, chunksize=4):
            frames[k] = (torch.from_numpy(rng).cuda(), [torch.from_numpy(l).cuda() for l in labs], Tcs)
            if k < n_check:
                host[k] = (rng, labs, Tcs)
            if len(frames) % 100 == 0:
                log(f"[bench] campus: {len(frames)}/{n} frames generated ({time.time() - t0:.0f} s)")
    torch.cuda.synchronize()
    cap = 4_000_000
    pos = torch.empty((cap, 3, 3), dtype=torch.float32, device="cuda")
    lab = torch.empty((cap, 3), dtype=torch.uint8, device="cuda")
    m = Map(w.voxel, w.trunc, w.n_classes, w.max_blocks)
    mesh_mask = 1 << KERNEL_NAMES.index("mesh")
    windows = {"early": (300, 300 + window), "late": (warm - window, warm)}
    win = {}
    times, U, alloc, mesh_blocks = [], 0, [], []
    for k in range(n):
        r, labs, Tcs = frames[k]
        T = w.poses[k]
        for name, (a, b) in windows.items():
            if k == a:
                torch.cuda.synchronize()
                m.profile(mesh_mask)
                win[name] = {"frames": f"{a}-{b - 1}", "allocated_blocks_start": m.stats()[1]["allocated"],
                             "mesh_blocks": 0}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.integrate_lidar(lid, r, T)
        if k >= warm:
            m.integrate_labels_multi(cams, labs, Tcs)
        m.extract_mesh(MAP_MESH_DIRTY, pos, lab, None)
        torch.cuda.synchronize()  # the frame ends when its triangles are written
        t1 = time.perf_counter()
        for name, (a, b) in windows.items():
            if a <= k < b:
                win[name]["mesh_blocks"] += m.stats()[1]["mesh_blocks"]
            if k == b - 1:
                torch.cuda.synchronize()
                ms, launches = m.profile_read()["mesh"]
                m.profile(0)
                d = win[name]
                d["allocated_blocks_end"] = m.stats()[1]["allocated"]
                d["mesh_us_per_frame"] = 1e3 * ms / launches
                d["mesh_blocks_per_frame"] = d["mesh_blocks"] / launches
                d["mesh_ns_per_block"] = 1e6 * ms / max(d.pop("mesh_blocks"), 1)
        if k >= warm:
            times.append(t1 - t0)
            st, s = m.stats()
            U += s["updates"]
            alloc.append(s["allocated"])
            mesh_blocks.append(s["mesh_blocks"])
        if (k + 1) % 100 == 0:
            log(f"[bench] campus: frame {k + 1}/{n}")
    m.close()
    same = campus_same_frames(torch, w, lid, frames, pos, lab, window)
    check = (w, host, campus_gpu_counts(torch, w, lid, cams, frames, len(host), pos, lab))
    del pos, lab
    fine = bench_campus_fine(torch, w, lid, frames, warm, window)
    t = np.array(times) * 1e3
    return {"workload": f"{w.name}, 2 x 1920x1080 cameras, L=20, max_blocks {w.max_blocks}",
            "frames": f"{warm} frames of growth (scan and meshing), then frames {warm}-{n - 1} timed",
            "frames_timed": len(times), "ms_per_frame_p50": float(np.median(t)),
            "ms_per_frame_p90": float(np.percentile(t, 90)), "voxel_updates_per_s": U / (t.sum() * 1e-3),
            "mesh_blocks_per_frame": float(np.mean(mesh_blocks)),
            "allocated_blocks_start": int(alloc[0]), "allocated_blocks_end": int(alloc[-1]),
            "mesh_windows": win, "mesh_same_frames": same, "fine_voxels": fine}, check


def campus_gpu_counts(torch, w, lid, cams, frames, n, pos, lab):
    """The first campus frames (scan, both label images, dirty meshing) on the GPU into a map
    with room for 200K blocks: each frame's counts, for the CPU baseline's oracle run on the
    same frames to compare."""
    from paper_2412_00291_amd import Map, MAP_MESH_DIRTY
    m = Map(w.voxel, w.trunc, w.n_classes, CAMPUS_CHECK_BLOCKS)
    out = []
    for k in range(n):
        r, labs, Tcs = frames[k]
        m.integrate_lidar(lid, r, w.poses[k])
        m.integrate_labels_multi(cams, labs, Tcs)
        m.extract_mesh(MAP_MESH_DIRTY, pos, lab, None)
        out.append(m.stats()[1])
    m.close()
    return out


CAMPUS_CHECK_BLOCKS = 200_000


def campus_same_frames(torch, w, lid, frames, pos, lab, window):
    """Meshing of the same frames in a small and in a larger map: frames 0..399 (scan and
    dirty meshing) into a fresh map, and into a map that first took frames 900..1299 (the
    far side of the loop, beyond the scan's range from frames 300..399, so the dirty blocks
    of those frames are the same blocks in both maps); meshing timed with events over
    frames 300..399 in each."""
    from paper_2412_00291_amd import KERNEL_NAMES, Map, MAP_MESH_DIRTY
    mesh_mask = 1 << KERNEL_NAMES.index("mesh")
    first = 400 - window
    out = {"frames_timed": f"{first}-399"}
    for name, pre in (("small", []), ("large", list(range(900, 1300)))):
        m = Map(w.voxel, w.trunc, w.n_classes, w.max_blocks)
        for k in pre:
            m.integrate_lidar(lid, frames[k][0], w.poses[k])
            m.extract_mesh(MAP_MESH_DIRTY, pos, lab, None)
        blocks = 0
        for k in range(400):
            if k == first:
                torch.cuda.synchronize()
                m.profile(mesh_mask)
                a0 = m.stats()[1]["allocated"]
            m.integrate_lidar(lid, frames[k][0], w.poses[k])
            m.extract_mesh(MAP_MESH_DIRTY, pos, lab, None)
            if k >= first:
                blocks += m.stats()[1]["mesh_blocks"]
        torch.cuda.synchronize()
        ms, launches = m.profile_read()["mesh"]
        out[name] = {"allocated_blocks_start": a0, "allocated_blocks_end": m.stats()[1]["allocated"],
                     "mesh_us_per_frame": 1e3 * ms / launches, "mesh_blocks_per_frame": blocks / launches}
        m.close()
        log(f"[bench] campus, same frames in the {name} map: {out[name]}")
    return out


def bench_campus_fine(torch, w, lid, frames, warm, window):
    """Dirty meshing of a map of millions of blocks: the campus growth frames (scan and
    dirty meshing) at 0.05 m voxels (tau 0.15 m, one class) into a map of up to 4M blocks,
    once with the dirty blocks found in the dirty bitmap (the default above 2^19 blocks) and
    once by the sweep of the slots (threshold never reached); meshing timed with events
    over the last `window` frames of each run."""
    from paper_2412_00291_amd import KERNEL_NAMES, Map, MAP_MESH_DIRTY
    cap = 16_000_000
    pos = torch.empty((cap, 3, 3), dtype=torch.float32, device="cuda")
    lab = torch.empty((cap, 3), dtype=torch.uint8, device="cuda")
    mesh_mask = 1 << KERNEL_NAMES.index("mesh")
    out = {"workload": f"campus frames 0-{warm - 1}, 0.05 m voxels, tau 0.15 m, max_blocks 4000000",
           "frames_timed": f"{warm - window}-{warm - 1}"}
    for name, threshold in (("bitmap", -1), ("sweep", 1 << 40)):
        m = Map(0.05, 0.15, 1, 4_000_000)
        m.set_dirty_bitmap(threshold)
        from_bits = blocks = over = 0
        for k in range(warm):
            if k == warm - window:
                torch.cuda.synchronize()
                m.profile(mesh_mask)
                a0 = m.stats()[1]["allocated"]
            m.integrate_lidar(lid, frames[k][0], w.poses[k])
            st, n = m.extract_mesh(MAP_MESH_DIRTY, pos, lab, None, allow_small=True)
            over += n > cap
            if k >= warm - window:
                s = m.stats()[1]
                from_bits += s["mesh_from_bitmap"]
                blocks += s["mesh_blocks"]
            if (k + 1) % 100 == 0:
                log(f"[bench] campus at 0.05 m, {name}: frame {k + 1}/{warm}")
        torch.cuda.synchronize()
        ms, launches = m.profile_read()["mesh"]
        out[name] = {"allocated_blocks_start": a0, "allocated_blocks_end": m.stats()[1]["allocated"],
                     "mesh_us_per_frame": 1e3 * ms / launches, "mesh_blocks_per_frame": blocks / launches,
                     "extractions_from_bitmap": from_bits, "extractions_over_capacity": over}
        m.close()
        log(f"[bench] campus at 0.05 m, {name}: {out[name]}")
    return out


def calibrate_copy(torch):
    """A plain copy of known size, for scaling HBM counters (FETCH_SIZE / WRITE_SIZE)."""
    n = 256 << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": n, "bytes_written": n, "launches": 3}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=90)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-baseline-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extensions", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--write-traffic", metavar="DIR",
                    help="summarise rocprofv3 FETCH_SIZE/WRITE_SIZE runs under DIR into " + TRAFFIC_JSON)
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args.write_traffic)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU; runs on several GPUs are not implemented "
              "(a map would shard by block ownership)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        calibrate_copy(torch)
        return
    import synth
    from paper_2412_00291_amd import CameraModel, LidarModel, Map, KERNEL_NAMES

    K, W = args.steps, args.warmup
    nfr = K + W
    w = synth.street_workload(n_frames=nfr)
    log(f"[bench] workload {w.name}: {nfr} frames, {len(w.cameras)} cameras")
    frames = make_frames(w, nfr)
    lidar = LidarModel(w.lidar.rows, w.lidar.cols, w.lidar.elev_rad, w.lidar.r_max)
    cams = [CameraModel(c.width, c.height, c.fx, c.fy, c.cx, c.cy) for c in w.cameras]
    dev_frames = []
    for f in frames:
        labs = torch.from_numpy(np.stack([np.ascontiguousarray(l) for _, l, _ in f.cams])).cuda()
        dev_frames.append((torch.from_numpy(f.range).cuda(), [labs[c] for c in range(len(f.cams))], f.T_wl,
                           [T for T, _, _ in f.cams]))
    torch.cuda.synchronize()
    cap = 4_000_000
    pos = torch.empty((cap, 3, 3), dtype=torch.float32, device="cuda")
    lab = torch.empty((cap, 3), dtype=torch.uint8, device="cuda")

    # counting pass (untimed): per-frame U_k, V_k, |T_k|, |M_k|, triangles
    m = Map(w.voxel, w.trunc, w.n_classes, w.max_blocks)
    per_frame = run_frames(torch, m, w, dev_frames, lidar, cams, range(nfr), pos, lab, stats=True)
    m.close()
    log(f"[bench] counting pass done: frame {W} has U={per_frame[W]['updates']} "
        f"T={per_frame[W]['touched']} M={per_frame[W]['mesh_blocks']} tris={per_frame[W]['triangles']}")

    # schedule choice per phase (workgroup or wavefront per block): the warm-up frames on
    # fresh maps with each uniform schedule, kernel time per phase compared
    all_kernels = (1 << len(KERNEL_NAMES)) - 1
    phase_ms = {}
    for sc in (0, 1):
        mt = Map(w.voxel, w.trunc, w.n_classes, w.max_blocks)
        mt.set_schedule(sc, sc, sc)
        run_frames(torch, mt, w, dev_frames, lidar, cams, range(max(W // 2, 1)), pos, lab)
        mt.profile(all_kernels)
        run_frames(torch, mt, w, dev_frames, lidar, cams, range(max(W // 2, 1), W), pos, lab)
        phase_ms[sc] = mt.profile_read()
        mt.close()
    sched = [0 if group_ms(phase_ms[0], k) <= group_ms(phase_ms[1], k) else 1 for k in ("tsdf", "labels", "mesh")]
    log(f"[bench] schedules (tsdf, labels, mesh): {sched}")

    # dominant kernel group (by warm-up time under the chosen schedules): the only one whose
    # launches the timed pass brackets with HIP events, so the frame time carries no
    # other event records.  Camera labels are fused into the TSDF launch when they follow
    # the scan (one launch, "tsdf_labels").
    fused = phase_ms[sched[0]]["tsdf_labels"][1] > 0
    groups = ("alloc", "tsdf_labels" if fused else "tsdf", "labels", "mesh")
    sched_of = {"alloc": 0, "tsdf": sched[0], "tsdf_labels": sched[0], "labels": sched[1], "mesh": sched[2]}
    dominant = max(groups, key=lambda k: phase_ms[sched_of[k]][k][0])

    # timed pass
    m = Map(w.voxel, w.trunc, w.n_classes, w.max_blocks)
    m.set_schedule(*sched)
    run_frames(torch, m, w, dev_frames, lidar, cams, range(W), pos, lab)
    torch.cuda.synchronize()
    # the dominant group is bracketed by HIP events on every PROF_EVERY-th timed frame (a
    # pair of events around a group costs the frame several microseconds)
    prof_frames = set(range(W, nfr, PROF_EVERY))
    step_times = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_frames(torch, m, w, dev_frames, lidar, cams, range(W, nfr), pos, lab, step_times=step_times,
               prof=(1 << KERNEL_NAMES.index(dominant), prof_frames))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof_dom = m.profile_read()[dominant]
    m.close()
    elapsed = t1 - t0
    timed = per_frame[W:]
    U = sum(s["updates"] for s in timed)
    value = U / elapsed

    # per-kernel breakdown: the same frames again on a fresh map, every kernel bracketed
    m = Map(w.voxel, w.trunc, w.n_classes, w.max_blocks)
    m.set_schedule(*sched)
    run_frames(torch, m, w, dev_frames, lidar, cams, range(W), pos, lab)
    torch.cuda.synchronize()
    m.profile(all_kernels)
    run_frames(torch, m, w, dev_frames, lidar, cams, range(W, nfr), pos, lab)
    torch.cuda.synchronize()
    prof = m.profile_read()
    m.close()

    kern = {k: {"avg_us": 1e3 * prof[k][0] / prof[k][1], "launches": prof[k][1], "total_ms": prof[k][0]}
            for k in KERNEL_NAMES if prof[k][1] > 0}
    for k, v in kern.items():
        ab = sum(algorithmic_bytes(k, s, w.lidar.rows, w.lidar.cols, w.cameras) for s in per_frame[W:])
        v["alg_GBps"] = ab / (v["total_ms"] * 1e-3) / 1e9
        v["hbm_frac"] = v["alg_GBps"] * 1e9 / PEAK_HBM
    alg = sum(algorithmic_bytes(dominant, per_frame[k], w.lidar.rows, w.lidar.cols, w.cameras) for k in prof_frames)
    launches = prof_dom[1]
    assert launches == len(prof_frames), (launches, len(prof_frames))
    dom_avg_us = 1e3 * prof_dom[0] / launches
    achieved = (alg / launches) / (dom_avg_us * 1e-6)
    sch = {"tsdf": sched[0], "labels": sched[1], "mesh": sched[2]}
    traffic = measured_traffic(dominant, sch)
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": achieved / PEAK_HBM,
                "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE, WRITE_SIZE, copy-calibrated)",
                "alg_bytes_per_launch": alg / launches, "avg_us_timed_region": dom_avg_us,
                "event_frames": f"{launches} of the {K} timed frames (every {PROF_EVERY}th)"}
    # every kernel group's HBM roofline from the breakdown pass, with its counter traffic
    roofline_groups = {}
    for k in ("alloc", "tsdf", "tsdf_labels", "labels", "mesh"):
        if k in kern:
            roofline_groups[k] = {"bound": "hbm", "achieved": kern[k]["alg_GBps"], "peak": PEAK_HBM / 1e9,
                                  "unit": "GB/s", "frac": kern[k]["hbm_frac"], "avg_us": kern[k]["avg_us"],
                                  "traffic": measured_traffic(k, sch)}
    integ_ms = sum(kern[k]["total_ms"] for k in ("alloc", "tsdf", "tsdf_labels", "labels") if k in kern)
    mesh_ms = kern.get("mesh", {"total_ms": float("nan")})["total_ms"]
    st = np.array(step_times) * 1e3
    result = {
        "metric": METRIC, "value": value, "unit": "voxel-updates/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": 1e3 * elapsed / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name + "-tau0.3-4cam-1280x720-L19", "frames_timed": K,
                   "scan": "64x2048 +2/-24.8 deg, 100 m", "voxel_m": w.voxel, "truncation_m": w.trunc,
                   "cameras": "4 x 1280x720, 19 classes", "meshing": "dirty blocks every frame"},
        "ms_per_frame_p50": float(np.median(st)), "ms_per_frame_p90": float(np.percentile(st, 90)),
        "integration_updates_per_s": U / (integ_ms * 1e-3),
        "mesh_blocks_per_s": sum(s["mesh_blocks"] for s in timed) / (mesh_ms * 1e-3),
        "per_frame_means": {k: float(np.mean([s[k] for s in timed])) for k in
                            ("updates", "votes", "touched", "new_blocks", "mesh_blocks", "triangles")},
        "kernels": kern,
        "schedules": {"tsdf": sched[0], "labels": sched[1], "mesh": sched[2],
                      "meaning": "0 = workgroup per block, 1 = wavefront per block",
                      "warmup_kernel_ms": {str(sc): {k: phase_ms[sc][k][0] for k in ("tsdf", "labels", "mesh")}
                                           for sc in (0, 1)}},
        "roofline": roofline,
        "roofline_groups": roofline_groups,
        "h2d_inputs": h2d_inputs(torch, frames),
    }
    campus = None  # the first campus frames' inputs and GPU counts, for the oracle check
    if not args.no_extensions:
        result["extensions"] = {"pose_adjoint": bench_adjoint(torch), "range_image": bench_range_image(torch),
                                "lidar_labels": bench_lidar_labels(torch),
                                "nonprojective": bench_nonprojective(torch),
                                "label_modes": bench_label_modes(torch),
                                "batched": bench_batched(torch),
                                "large_scale": None}
        result["extensions"]["large_scale"], campus = bench_campus(torch)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        oracle_frames, extra, result["cpu_baseline"] = cpu_baseline(w, frames, args.cpu_baseline_seconds, campus)
        if "campus_check" in extra:
            result["oracle_check_campus"] = extra["campus_check"]
        # the per-frame counts behind `value` (the GPU counting pass) against the oracle's
        keys = ("updates", "votes", "touched", "new_blocks", "mesh_blocks", "triangles", "allocated")
        bad = [(k, key, per_frame[k][key], o[key]) for k, o in enumerate(oracle_frames) for key in keys
               if per_frame[k][key] != o[key]]
        result["oracle_check"] = {"frames": len(oracle_frames), "counts": list(keys), "equal": not bad,
                                  "mismatches": bad[:5]}
    print(json.dumps(result))


if __name__ == "__main__":
    main()

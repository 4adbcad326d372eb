#!/usr/bin/env python3
"""Voxel-grid downsampling throughput on one MI355X (libvg).

Step = one batched call over the uneven 64-frame RGB-D batch (every frame
through bbox, histogram, radix sort and segmented reduce; the call's launch
sequence replayed from a hipGraph), inputs resident in HBM.  Prints one JSON
line: Mpoints/s (input points, valid and invalid), the roofline of the
dominant kernel (HIP event pairs around each launch, in a second timed region
of the same steps), the whole step's roofline, the plain per-frame path and the
backward on the same GPU, and the CPU oracle on a bounded sample.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "Mpoints/s voxel downsample + % HBM roofline; batched vs plain at 1e-6 tol"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def frame_passes(x, y, z, leaf, radix_bits, with_bits=False):
    """Radix passes (and key bits) of a frame under the library's rule
    (host-side byte accounting only)."""
    v = np.isfinite(x) & np.isfinite(y) & np.isfinite(z)
    if not v.any():
        return (0, 0) if with_bits else 0
    inv = np.float32(1.0) / np.float32(leaf)
    dims = []
    for a in (x, y, z):
        av = a[v]
        t = (av.max() - av.min()) * inv
        dims.append(int(np.floor(t)) + 1)
    top = dims[0] * dims[1] * dims[2] - 1
    bits = top.bit_length()
    passes = max(1, math.ceil(bits / radix_bits))
    return (passes, bits) if with_bits else passes


def algorithmic_bytes(n, nv, passes, m, point_cell=False):
    """Bytes the sort-based method moves per call: bbox and key read xyz of every
    point (12 + 12 B), the key pass writes (key, index) of valid points (8 B),
    the histogram reads keys (4 B), each radix pass reads and writes pairs
    (16 B), the reduce reads pairs (8 B) and gathers xyz + rgb (15 B), and every
    cell writes xyz, rgb, count, key (27 B); the per-point row adds 4 B."""
    return 24 * n + (8 + 4 + 16 * passes + 8 + 15 + (4 if point_cell else 0)) * nv + 27 * m


def kernel_bytes(n, nv, passes, m, narrow, point_cell=False):
    """Algorithmic bytes per step of each kernel of the phased pipeline, summed
    over frames (lists indexed like the frames):
      bbox    reads xyz of every point                      12 B x n
      hist    reads xyz of every point to form the keys      12 B x n
              and stores them when they fit 31 bits          +4 B x n
      sort    pass 0 reads the stored keys (else xyz) and    4 B (12 B) x n
              writes (key, index) pairs                      + 8 B x n_v
              pass p > 0 reads and writes the pairs          16 B x n_v of frames with > p passes
      reduce  reads the pairs, gathers xyz + rgb             23 B x n_v (+4 B x n_v point rows)
              writes xyz, rgb, count, key per cell           27 B x m
    """
    n, nv, passes, m = (np.asarray(a, dtype=np.int64) for a in (n, nv, passes, m))
    narrow = np.asarray(narrow, dtype=bool)
    live = passes > 0
    key_in = np.where(narrow & live, 4, 12)
    sort = int((key_in * n).sum() + (8 * nv[live]).sum() +
               (16 * nv * np.maximum(passes - 1, 0)).sum())
    red = int(((23 + (4 if point_cell else 0)) * nv).sum() + (27 * m).sum())
    hist = int((12 * n).sum() + (4 * n[narrow & live]).sum())
    b = {"init": 0, "bbox": int(12 * n.sum()), "hist": hist, "sort": sort,
         "reduce": red, "fixup": 0}
    b["pipeline"] = sum(b.values())
    return b


def step_bytes_by_kernel(n, nv, passes, m, point_cell=False):
    """Algorithmic bytes per step of each kernel, by the per-step byte counts of
    the sort-based method (the method's own traffic, not this design's):
      bbox    validity and box: xyz of every point            12 B x n
      hist    key formation: xyz of every point               12 B x n
              digit histograms over the keys                   + 4 B x n_v
      sort    every radix pass reads and writes pairs          16 B x P x n_v
      reduce  pairs + gathered xyz/rgb                         23 B x n_v (+4 B x n_v rows)
              one row per cell: xyz, rgb, count, key           + 27 B x m
    The key step's (key, index) write of 8 B x n_v (done by radix pass 0 here)
    is counted in the step total but in no kernel's row.  Summed over frames."""
    n, nv, passes, m = (np.asarray(a, dtype=np.int64) for a in (n, nv, passes, m))
    b = {"init": 0, "bbox": int(12 * n.sum()), "hist": int(12 * n.sum() + 4 * nv.sum()),
         "sort": int((16 * passes * nv).sum()),
         "reduce": int(((23 + (4 if point_cell else 0)) * nv).sum() + (27 * m).sum()),
         "fixup": 0}
    b["pipeline"] = sum(b.values()) + int(8 * nv.sum())
    return b


def source_digest():
    """Digest of the device code, the header and the tuning choice: counter
    figures taken under another digest no longer describe these kernels."""
    import hashlib
    h = hashlib.sha256()
    files = [os.path.join(ROOT, "include", "vg.h")]
    csrc = os.path.join(ROOT, "paper_2102_11084_amd", "csrc")
    files += [os.path.join(csrc, f) for f in sorted(os.listdir(csrc))
              if f.endswith((".hip", ".hpp", ".h"))]
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + fh.read())
    # the tuning choice itself, not the timings the autotuner recorded with it
    with open(os.path.join(ROOT, "paper_2102_11084_amd", "tuning_gfx950.json")) as fh:
        h.update(b"tuning\0" + json.dumps(json.load(fh).get("tuning"), sort_keys=True).encode())
    return h.hexdigest()[:16]


def read_traffic(kind, workload_tag):
    """HBM bytes per launch of `kind` from the committed counter summary, or
    None when it is missing or was taken on other kernels."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload_tag}.txt")
    try:
        rows = dict(line.split(":", 1) for line in open(path) if ":" in line and not line.startswith("#"))
    except OSError:
        return None, "no counter summary"
    rows = {k.strip(): v.strip() for k, v in rows.items()}
    if rows.get("source_digest") != source_digest():
        return None, "counter summary taken on other kernels"
    v = rows.get(f"{kind}_bytes_per_launch")
    return (int(float(v)), path) if v else (None, f"no {kind} row")


def copy_calibration(steps):
    """A plain device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(steps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": steps}),
          flush=True)


def plan_kernel_times(plan, args_run, steps):
    """Per-kind launch times of `steps` runs of a plan, each launch between a
    HIP event pair on the plan's stream: {kind: [total ms, launches]} and the
    per-launch list of the last run."""
    plan.set_timing(True)
    per_kind, last = {}, None
    for _ in range(max(steps, 1)):
        plan.run(*args_run[0], **args_run[1])
        last = plan.kernel_times()
        for kind, ms in last:
            t = per_kind.setdefault(kind, [0.0, 0])
            t[0] += ms
            t[1] += 1
    plan.set_timing(False)
    return per_kind, last


def kernel_table(per_kind, steps, kbytes):
    ks = max(steps, 1)
    return {k: {"ms_per_step": round(v[0] / ks, 4), "launches_per_step": v[1] // ks,
                "avg_launch_ms": round(v[0] / v[1], 4),
                "algorithmic_bytes_per_step": kbytes[k],
                "gbs": round(kbytes[k] / (v[0] / ks * 1e-3) / 1e9, 1) if v[0] > 0 else None}
            for k, v in per_kind.items()}


def single_cloud_leg(name, cloud, leaf, tuning, dev, reps, oracle_runs, cpu_jobs):
    """One cloud through the plain path (synchronous vg_downsample_ex calls,
    m read back) and its kernels timed through a one-frame plan; the oracle's
    timing on the same cloud is registered in cpu_jobs for the CPU-baseline
    leg."""
    import torch

    from paper_2102_11084_amd import vg
    x, y, z, rgb = cloud
    n = x.size
    d = [torch.from_numpy(a).to(dev) for a in (x, y, z, rgb.reshape(-1))]
    ws = torch.empty(vg.workspace_bytes(n, 1, tuning), dtype=torch.uint8, device=dev)
    out_set = ("xyz", "rgb", "count", "key")
    for _ in range(2):
        r = vg.voxel_downsample(*d, leaf=leaf, tuning=tuning, outputs=out_set, workspace=ws)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = vg.voxel_downsample(*d, leaf=leaf, tuning=tuning, outputs=out_set, workspace=ws)
        ts.append(time.perf_counter() - t0)
    med = float(np.median(ts))
    m = int(r["m"])
    nv = int((np.isfinite(x) & np.isfinite(y) & np.isfinite(z)).sum())
    passes, bits = frame_passes(x, y, z, leaf, tuning.radix_bits, with_bits=True)
    # kernels: the same kernels through a one-frame plan with per-launch events
    plan = vg.BatchPlan(1, n, vg.KEY_LINEAR, tuning)
    outs = plan.alloc_outputs(n, 1, dev, outputs=out_set)
    offs = np.array([0, n], np.int64)
    lv = np.array([leaf], np.float32)
    per_kind, _ = plan_kernel_times(plan, ((*d, offs, lv), {"out": outs}), max(3, reps // 2))
    plan.close()
    kb = step_bytes_by_kernel([n], [nv], [passes], [m])
    kt = kernel_table(per_kind, max(3, reps // 2), kb)
    sort = kt.get("sort")
    leg = {
        "workload": name, "points": n, "valid_points": nv, "leaf": leaf, "cells": m,
        "key_bits": int(bits), "radix_passes": int(passes),
        "plain_ms_median": round(med * 1e3, 4),
        "plain_ms_p10_p90": [round(float(np.percentile(ts, 10)) * 1e3, 4),
                             round(float(np.percentile(ts, 90)) * 1e3, 4)],
        "mpoints_s": round(n / med / 1e6, 1), "valid_mpoints_s": round(nv / med / 1e6, 1),
        "kernels": kt,
        "radix_roofline_frac": round(sort["gbs"] / HBM_PEAK_GBS, 4) if sort and sort["gbs"] else None,
    }
    if oracle_runs > 0:
        def job(x=x, y=y, z=z, rgb=rgb, leaf=leaf, runs=oracle_runs, n=n):
            import oracle
            ot = []
            for _ in range(runs):
                c0 = time.perf_counter()
                oracle.downsample(x, y, z, rgb, leaf)
                ot.append(time.perf_counter() - c0)
            return {"mpoints_s": round(n / float(np.median(ot)) / 1e6, 3),
                    "sample": f"the whole cloud, median of {runs}"}
        cpu_jobs.append((name, job))
    return leg


def nbd_candidate_checks(x, y, z, leaf):
    """Point pairs the 27-bucket search examines (host-side accounting): for
    every valid point, the points of the 27 cells around its own (itself
    included), on the grid of the voxel filter."""
    v = np.isfinite(x) & np.isfinite(y) & np.isfinite(z)
    if not v.any():
        return 0
    inv = np.float32(1.0) / np.float32(leaf)
    k = [np.floor((a[v] - a[v].min()) * inv).astype(np.int64) for a in (x, y, z)]
    d = [int(kk.max()) + 1 for kk in k]
    key = k[0] + d[0] * (k[1] + d[1] * k[2])
    uniq, cnt = np.unique(key, return_counts=True)
    ux, t = uniq % d[0], uniq // d[0]
    uy, uz = t % d[1], t // d[1]
    s = np.zeros(uniq.size, np.int64)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                nx, ny, nz = ux + dx, uy + dy, uz + dz
                ok = (nx >= 0) & (nx < d[0]) & (ny >= 0) & (ny < d[1]) & (nz >= 0) & (nz < d[2])
                nk = nx + d[0] * (ny + d[1] * nz)
                pos = np.searchsorted(uniq, nk)
                pos = np.minimum(pos, uniq.size - 1)
                hit = ok & (uniq[pos] == nk)
                s += np.where(hit, cnt[pos], 0)
    return int((cnt * s).sum())


def nbd_leg(tuning, dev, reps=5, oracle_runs=1, cpu_jobs=None):
    """The paper's own filter (Alg. 1, neighbour-bucket decimation) on a
    640x480 frame: leaf and radius 0.02 m (the paper's Table I grid),
    umbral 16, 1000 points per round.  Whole synchronous calls are timed; the
    oracle's timing is registered in cpu_jobs for the CPU-baseline leg."""
    import torch

    from paper_2102_11084_amd import datagen as dg
    from paper_2102_11084_amd import vg
    x, y, z, rgb = dg.frame_640x480()
    n = x.size
    leaf, umbral, rs, seed = 0.02, 16, 1000, 7
    d = [torch.from_numpy(a).to(dev) for a in (x, y, z, rgb.reshape(-1))]
    ws = torch.empty(int(vg.lib().vg_nbd_workspace_bytes(n, rs)), dtype=torch.uint8, device=dev)
    r = vg.nbd_decimate(*d, leaf=leaf, umbral=umbral, seed=seed, round_size=rs, workspace=ws,
                        tuning=tuning)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = vg.nbd_decimate(*d, leaf=leaf, umbral=umbral, seed=seed, round_size=rs, workspace=ws,
                            tuning=tuning)
        ts.append(time.perf_counter() - t0)
    med = float(np.median(ts))
    leg = {"workload": "neighbour-bucket decimation (Alg. 1) of a 640x480 RGB-D frame, leaf = radius "
                       "= 0.02 m, umbral 16, 1000 points per round, seed 7",
           "points": n, "valid_points": int(np.isfinite(z).sum()), "survivors": int(r["n_keep"]),
           "rounds": int(r["rounds"]), "marked_first_round": int(r["marked"][0]),
           "ms_median": round(med * 1e3, 3),
           "ms_min_max": [round(min(ts) * 1e3, 3), round(max(ts) * 1e3, 3)],
           "us_per_round": round(med * 1e6 / max(int(r["rounds"]), 1), 2),
           "mpoints_s": round(n / med / 1e6, 2),
           "candidate_pairs": nbd_candidate_checks(x, y, z, leaf)}
    if oracle_runs > 0 and cpu_jobs is not None:
        def job():
            import oracle
            ot = []
            for _ in range(oracle_runs):
                c0 = time.perf_counter()
                oracle.nbd_decimate(x, y, z, leaf, leaf, umbral, seed, rs)
                ot.append(time.perf_counter() - c0)
            return {"ms_per_frame": round(float(np.median(ot)) * 1e3, 1),
                    "sample": f"the same frame, median of {oracle_runs}"}
        cpu_jobs.append((leg["workload"], job))
    return leg


def same_as_ref(h, o_ref):
    """Outputs of a batched call bit-identical to the reference call's."""
    m = int(o_ref["out_offsets"][-1])
    return bool(np.array_equal(h["out_offsets"], o_ref["out_offsets"]) and
                all(np.array_equal(h[k][:m].view(np.uint8), o_ref[k][:m].view(np.uint8))
                    for k in ("x", "y", "z", "rgb", "count", "key")))


def ingest_leg(x, y, z, rgb, offs, leaves, d, plan, outs, o_ref, tuning, dev, steps, use_graph):
    """The batch with its points in pinned host memory instead of HBM: (a) an
    explicit copy to the device then the call; (a') the copy of the next batch
    on a copy stream, overlapped with the call on the current one (two sets of
    device inputs); (b) the call reading the mapped host memory itself, once,
    in its bbox pass (the paper's zero-copy)."""
    import torch

    from paper_2102_11084_amd import vg
    stream = torch.cuda.current_stream(dev)
    N = int(offs[-1])
    B = len(leaves)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    # (a) pinned torch tensors copied in, then the same call as the headline
    pinned = [torch.from_numpy(np.ascontiguousarray(a)).pin_memory() for a in (x, y, z, rgb.reshape(-1))]
    for _ in range(2):
        for t, p in zip(d, pinned):
            t.copy_(p, non_blocking=True)
        plan.run(*d, offs, leaves, out=outs)
    torch.cuda.synchronize()
    e0, e1, e2 = ev(), ev(), ev()
    e0.record(stream)
    for _ in range(steps):
        for t, p in zip(d, pinned):
            t.copy_(p, non_blocking=True)
    e1.record(stream)
    for _ in range(steps):
        for t, p in zip(d, pinned):
            t.copy_(p, non_blocking=True)
        plan.run(*d, offs, leaves, out=outs)
    e2.record(stream)
    torch.cuda.synchronize()
    copy_ms = e0.elapsed_time(e1) / steps
    copy_call_ms = e1.elapsed_time(e2) / steps
    # (a') the same, with the copy of the next batch (on a copy stream, into a
    # second set of device inputs) overlapped with the call on this one
    d2 = [torch.empty_like(t) for t in d]
    bufs = (d, d2)
    cs = torch.cuda.Stream(dev)
    nb = max(steps, 2)
    copied = [ev() for _ in range(nb)]
    computed = [ev() for _ in range(nb)]
    g0, g1 = ev(), ev()
    torch.cuda.synchronize()
    g0.record(cs)
    with torch.cuda.stream(cs):
        for t, p in zip(bufs[0], pinned):
            t.copy_(p, non_blocking=True)
        copied[0].record(cs)
    for k in range(nb):
        if k + 1 < nb:
            if k >= 1:
                cs.wait_event(computed[k - 1])  # the call before last read that buffer
            with torch.cuda.stream(cs):
                for t, p in zip(bufs[(k + 1) % 2], pinned):
                    t.copy_(p, non_blocking=True)
                copied[k + 1].record(cs)
        stream.wait_event(copied[k])
        plan.run(*bufs[k % 2], offs, leaves, out=outs)
        computed[k].record(stream)
    g1.record(stream)
    torch.cuda.synchronize()
    pipe_ms = g0.elapsed_time(g1) / nb
    pipe_same = same_as_ref({k: v.cpu().numpy() for k, v in outs[0].items()}, o_ref)
    del pinned, d2
    # (b) mapped host memory read by the bbox pass
    buf = vg.HostBuffer(15 * N)
    ptrs, off = [], 0
    for a in (x, y, z):
        buf.view(np.float32, N, off)[:] = a
        ptrs.append(buf.device + off)
        off += 4 * N
    buf.view(np.uint8, 3 * N, off)[:] = rgb.reshape(-1)
    ptrs.append(buf.device + off)
    hplan = vg.BatchPlan(B, N, vg.KEY_LINEAR, tuning, use_graph=use_graph)
    hplan.set_host_input(True)
    hout = hplan.alloc_outputs(N, B, dev, outputs=("xyz", "rgb", "count", "key"))
    for _ in range(2):
        hplan.run_host(*ptrs, N, offs, leaves, hout, stream)
    torch.cuda.synchronize()
    f0, f1 = ev(), ev()
    f0.record(stream)
    for _ in range(steps):
        hplan.run_host(*ptrs, N, offs, leaves, hout, stream)
    f1.record(stream)
    torch.cuda.synchronize()
    zc_ms = f0.elapsed_time(f1) / steps
    same = same_as_ref({k: v.cpu().numpy() for k, v in hout[0].items()}, o_ref)
    hplan.close()
    buf.close()
    in_bytes = 15 * N
    return {
        "workload": f"the {B}-frame batch with its {N} points (x, y, z, rgb: {in_bytes} B) in pinned "
                    "host memory",
        "copy_only_ms": round(copy_ms, 3), "copy_gbs": round(in_bytes / (copy_ms * 1e-3) / 1e9, 1),
        "copy_then_call_ms": round(copy_call_ms, 3),
        "copy_then_call_mpoints_s": round(N / (copy_call_ms * 1e-3) / 1e6, 1),
        "copy_overlapped_ms": round(pipe_ms, 3),
        "copy_overlapped_mpoints_s": round(N / (pipe_ms * 1e-3) / 1e6, 1),
        "copy_overlapped_bit_identical": pipe_same,
        "zero_copy_call_ms": round(zc_ms, 3),
        "zero_copy_mpoints_s": round(N / (zc_ms * 1e-3) / 1e6, 1),
        "zero_copy_input_gbs": round(in_bytes / (zc_ms * 1e-3) / 1e9, 1),
        "zero_copy_bit_identical": same,
    }


def map_leg(fout, fo_offsets, offs, leaves, dev, cpu_jobs, res=0.05, capacity=1 << 22, reps=5):
    """The costmap layer's map update over the filtered frames: per frame, the
    voxels inside its camera frustum are cleared, then the frame's cells (in
    the global frame) are marked with the frame's stamp.  The whole 64-frame
    sequence is timed on a fresh map each repetition; the oracle's map runs
    the same sequence in the CPU-baseline leg (cpu_jobs)."""
    import torch

    from paper_2102_11084_amd import datagen as dg
    from paper_2102_11084_amd import vg
    B = len(leaves)
    fr = []
    for b in range(B):
        W, H = int(dg.batch_frame_spec(b)["W"]), int(dg.batch_frame_spec(b)["H"])
        R, t = dg.camera_pose(8000 + b)
        f = 525.0 * W / 640.0
        fr.append((R, t, f, f, (W - 1) / 2.0, (H - 1) / 2.0, W, H, 0.3, 4.0))
    frus = [vg.make_frustum(*a) for a in fr]
    lo = [int(fo_offsets[b]) for b in range(B + 1)]
    cells = [(fout["x"][lo[b]:lo[b + 1]], fout["y"][lo[b]:lo[b + 1]], fout["z"][lo[b]:lo[b + 1]])
             for b in range(B)]
    stream = torch.cuda.current_stream(dev)
    times = []
    for rep in range(reps + 1):
        m = vg.VoxelMap(capacity, res)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for b in range(B):
            m.clear(frus[b])
            m.mark(*cells[b], b + 1)
        e1.record(stream)
        torch.cuda.synchronize()
        if rep > 0:
            times.append(e0.elapsed_time(e1))
        info = m.stats()
        gk, gs = m.export()
        m.close()
    ms = float(np.median(times))
    leg = {"workload": f"{B} filtered frames in order: clear the frame's camera frustum (0.3..4 m), "
                       f"then mark its cells; voxel {res} m, {capacity} slots",
           "ms_sequence": round(ms, 3), "ms_per_frame": round(ms / B, 4),
           "cells_marked": int(lo[B]), "voxels_at_end": int(info.occupied),
           "slots_used": int(info.used_slots)}
    host_cells = [tuple(c.cpu().numpy() for c in cb) for cb in cells]

    def job():
        import oracle
        o = oracle.VoxelMap(res)
        c0 = time.perf_counter()
        for b in range(B):
            o.clear(*fr[b])
            o.mark(*host_cells[b], b + 1)
        ms = (time.perf_counter() - c0) * 1e3
        o.close()
        return {"ms_sequence": round(ms, 1), "sample": "the same 64-frame sequence, once"}
    cpu_jobs.append((leg["workload"], job))
    return leg


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames", type=int, default=64)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--exec-mode", choices=["persistent", "phased", "tuned"], default="tuned",
                    help="launch form; tuned = the one in the tuning file (else the built-in default)")
    ap.add_argument("--tuning", default=os.path.join(ROOT, "paper_2102_11084_amd", "tuning_gfx950.json"))
    ap.add_argument("--set", action="append", default=[], metavar="FIELD=VALUE",
                    help="override a tuning field, e.g. --set sort_items=8")
    ap.add_argument("--point-cell", action="store_true",
                    help="also write every input point's output row (needed for the backward)")
    ap.add_argument("--no-legs", action="store_true", help="skip the plain, backward and config legs")
    ap.add_argument("--no-config-legs", action="store_true",
                    help="skip the single-cloud legs (640x480, 1280x720 sweep, 16M map)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="CPU time of one oracle run over the batch's frames (3 runs, median)")
    ap.add_argument("--kernel-steps", type=int, default=10,
                    help="steps of the per-kernel event timing region")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--leg", choices=["nbd", "room"], default=None,
                    help="only run the named leg (without its oracle timing) and print its JSON; "
                         "for profiling")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: libvg runs on one GPU here (frames would shard across GPUs by frame, "
              "but no multi-GPU path is built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration(max(args.steps, 1))
        return

    import torch

    from paper_2102_11084_amd import datagen as dg
    from paper_2102_11084_amd import vg

    dev = torch.device("cuda:0")
    tuning = vg.load_tuning(args.tuning) if os.path.exists(args.tuning) else vg.default_tuning()
    if args.leg == "nbd":
        print(json.dumps(nbd_leg(tuning, dev, reps=max(args.steps, 1), oracle_runs=0)), flush=True)
        return
    if args.leg == "room":
        leg = single_cloud_leg("16M-point shuffled room map, leaf 0.02, plain path", dg.room_map(),
                               0.02, tuning, dev, max(args.steps, 1), 0, [])
        print(json.dumps(leg), flush=True)
        return
    if args.exec_mode != "tuned":
        tuning.exec_mode = vg.EXEC_PHASED if args.exec_mode == "phased" else vg.EXEC_PERSISTENT
    for kv in args.set:
        k, v = kv.split("=", 1)
        setattr(tuning, k, int(v))
    if not vg.tuning_supported(tuning):
        sys.exit(f"bench.py: tuning {tuning.as_dict()} is not built into libvg")
    log(f"tuning {tuning.as_dict()}")

    t0 = time.time()
    x, y, z, rgb, offs, leaves = dg.batch(args.frames)
    N = int(offs[-1])
    nv_frames = np.array([int(np.isfinite(z[offs[b]:offs[b + 1]]).sum()) for b in range(len(leaves))])
    NV = int(nv_frames.sum())
    log(f"generated {len(leaves)} frames, {N} points ({NV} valid) in {time.time() - t0:.1f}s")
    d = [torch.from_numpy(a).to(dev) for a in (x, y, z, rgb.reshape(-1))]
    plan = vg.BatchPlan(len(leaves), N, vg.KEY_LINEAR, tuning, use_graph=not args.no_graph)
    out_set = ("xyz", "rgb", "count", "key") + (("point_cell",) if args.point_cell else ())
    outs = plan.alloc_outputs(N, len(leaves), dev, outputs=out_set)
    stream = torch.cuda.current_stream(dev)

    for _ in range(args.warmup):
        plan.run(*d, offs, leaves, out=outs)
    torch.cuda.synchronize()
    log("warmup done")

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        plan.run(*d, offs, leaves, out=outs)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    step_ev = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    ev_ms = float(np.mean(step_ev))
    ms_per_step = wall * 1e3 / args.steps
    value = N / (ms_per_step * 1e-3) / 1e6
    log(f"batched: {ms_per_step:.3f} ms/step (events {ev_ms:.3f} ms), {value:.1f} Mpoints/s")

    o = {k: v.cpu().numpy() for k, v in outs[0].items()}
    assert (o["frame_status"] == 0).all(), "a frame failed"
    m_frames = np.diff(o["out_offsets"])
    radix = tuning.radix_bits
    pb = np.array([frame_passes(x[offs[b]:offs[b + 1]], y[offs[b]:offs[b + 1]],
                                z[offs[b]:offs[b + 1]], leaves[b], radix, with_bits=True)
                   for b in range(len(leaves))])
    passes, bits = pb[:, 0], pb[:, 1]
    alg = sum(algorithmic_bytes(int(offs[b + 1] - offs[b]), int(nv_frames[b]), int(passes[b]),
                                int(m_frames[b]), args.point_cell) for b in range(len(leaves)))
    step_achieved = alg / (ev_ms * 1e-3) / 1e9
    floor_bytes = 15 * NV + 27 * int(m_frames.sum())

    # per-kernel timing region: the same step, launched directly with a HIP
    # event pair on the plan's stream around every kernel
    ks = max(args.kernel_steps, 1)
    per_kind, per_launch = plan_kernel_times(plan, ((*d, offs, leaves), {"out": outs}), ks)
    kb = step_bytes_by_kernel(np.diff(offs), nv_frames, passes, m_frames, args.point_cell)
    kbd = kernel_bytes(np.diff(offs), nv_frames, passes, m_frames, bits <= 31, args.point_cell)
    kinds = kernel_table(per_kind, ks, kb)
    for k in kinds:
        kinds[k]["design_bytes_per_step"] = kbd[k]
    dom = max(per_kind, key=lambda k: per_kind[k][0])
    dom_ms = per_kind[dom][0] / per_kind[dom][1]
    dom_launches = per_kind[dom][1] // ks
    dom_bytes = kb[dom] / dom_launches
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    tag = f"batch{len(leaves)}"
    traffic, tsrc = read_traffic(dom, tag)
    log("kernels per step: " + ", ".join(f"{k} {v['ms_per_step']:.3f} ms x{v['launches_per_step']}"
                                         f" ({v['gbs']} GB/s)" for k, v in kinds.items()))
    log(f"dominant kernel: {dom}, {dom_ms:.4f} ms/launch, {achieved:.1f} GB/s; traffic: {tsrc}")
    log("launches of the last timed step (ms): " + " ".join(f"{k}:{v:.3f}" for k, v in per_launch))
    result = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpoints/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded ray-cast RGB-D frames standing in for the paper's corridor data)",
        "config": {
            "workload": f"batched: {len(leaves)} uneven RGB-D frames, 50k-900k valid points each, "
                        "per-frame leaf in {0.02, 0.05, 0.10} m, one call per step, its launch "
                        "sequence (one launch per phase in the tuned form) replayed from a hipGraph",
            "frames": int(len(leaves)), "points": N, "valid_points": NV,
            "cells": int(m_frames.sum()), "radix_passes": [int(p) for p in passes],
            "tuning": tuning.as_dict(), "graph": not args.no_graph, "outputs": list(out_set),
            "launch_form": "persistent" if tuning.exec_mode == vg.EXEC_PERSISTENT else "phased",
        },
        "valid_mpoints_s": round(NV / (ms_per_step * 1e-3) / 1e6, 2),
        "step_ms_events": {"mean": round(ev_ms, 4), "p10": round(float(np.percentile(step_ev, 10)), 4),
                           "p50": round(float(np.percentile(step_ev, 50)), 4),
                           "p90": round(float(np.percentile(step_ev, 90)), 4)},
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": f"vg_pipeline_kernel<{dom}>",
            "byte_basis": "algorithmic bytes of the method per launch (radix: 16 B x passes x "
                          "valid points per step, over the kernel's launches per step)",
            "algorithmic_bytes_per_launch": int(dom_bytes),
            "launches_per_step": int(dom_launches),
            "avg_launch_ms_events": round(dom_ms, 4),
        },
        "step_roofline": {
            "algorithmic_bytes": int(alg), "achieved": round(step_achieved, 1),
            "frac": round(step_achieved / HBM_PEAK_GBS, 4),
            "floor_frac": round(floor_bytes / (ev_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        },
        "kernels": kinds,
    }

    cpu_jobs = []  # oracle timings of the legs' workloads, run in the CPU-baseline leg
    if not args.no_legs:
        # plain per-frame path: one synchronous vg_downsample_ex per frame
        ws = torch.empty(vg.workspace_bytes(int(np.diff(offs).max()), 1, tuning), dtype=torch.uint8,
                         device=dev)
        frames_dev = [[t[int(offs[b]) * (3 if t is d[3] else 1):int(offs[b + 1]) * (3 if t is d[3] else 1)]
                       for t in d] for b in range(len(leaves))]
        for rep in range(2):
            torch.cuda.synchronize()
            p0 = time.perf_counter()
            for b in range(len(leaves)):
                vg.voxel_downsample(*frames_dev[b], leaf=float(leaves[b]), tuning=tuning,
                                    outputs=out_set, workspace=ws)
            torch.cuda.synchronize()
            plain_s = time.perf_counter() - p0
        plain = N / plain_s / 1e6
        log(f"plain per-frame: {plain_s * 1e3:.2f} ms, {plain:.1f} Mpoints/s")
        # outside the timed region: batched rows against the plain rows
        bitwise, worst = True, 0.0
        for b in range(len(leaves)):
            r = vg.voxel_downsample(*frames_dev[b], leaf=float(leaves[b]), tuning=tuning,
                                    outputs=("xyz", "rgb", "count", "key"), workspace=ws)
            lo, hi = int(o["out_offsets"][b]), int(o["out_offsets"][b + 1])
            if r["m"] != hi - lo:
                raise SystemExit(f"bench.py: frame {b}: plain path gave {r['m']} cells, batched {hi - lo}")
            for k in ("count", "key", "rgb"):
                if not np.array_equal(r[k].cpu().numpy(), o[k][lo:hi]):
                    raise SystemExit(f"bench.py: frame {b}: batched {k} differs from the plain path")
            for k in ("x", "y", "z"):
                a, c = r[k].cpu().numpy(), o[k][lo:hi]
                if not np.array_equal(a.view(np.uint32), c.view(np.uint32)):
                    bitwise = False
                    worst = max(worst, float(np.abs(a.astype(np.float64) - c).max()) / float(leaves[b]))
        if worst > 1e-6:
            raise SystemExit(f"bench.py: batched centroids differ from plain by {worst:.3e} leaf")
        # backward leg: 32 clouds of 100k points, leaf 0.05, one batched forward + one backward
        cl = [dg.uniform_cloud(100_000, seed=5000 + c) for c in range(32)]
        bx = [torch.from_numpy(np.concatenate([c[a] for c in cl])).to(dev) for a in range(3)]
        boffs = np.arange(33, dtype=np.int64) * 100_000
        bplan = vg.BatchPlan(32, 3_200_000, vg.KEY_LINEAR, tuning)
        bleaf = np.full(32, 0.05, np.float32)
        bout = bplan.alloc_outputs(3_200_000, 32, dev, outputs=("xyz", "count", "point_cell"),
                                   have_rgb=False)
        bo = bplan.run(bx[0], bx[1], bx[2], None, boffs, bleaf, out=bout)
        torch.cuda.synchronize()
        mt = int(bo["out_offsets"][-1].item())
        G = torch.randn(mt, 3, device=dev)
        gx, gy, gz = (G[:, a].contiguous() for a in range(3))
        cnt = bo["count"][:mt]
        for _ in range(3):
            vg.downsample_backward(gx, gy, gz, cnt, bo["point_cell"])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(20):
            vg.downsample_backward(gx, gy, gz, cnt, bo["point_cell"])
        e1.record(stream)
        torch.cuda.synchronize()
        bwd_ms = e0.elapsed_time(e1) / 20
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        for _ in range(10):
            bplan.run(bx[0], bx[1], bx[2], None, boffs, bleaf, out=bout)
        f1.record(stream)
        torch.cuda.synchronize()
        fwd_ms = f0.elapsed_time(f1) / 10
        bplan.close()
        result["legs"] = {
            "plain_per_frame_mpoints_s": round(plain, 2),
            "batched_over_plain": round(value / plain, 2),
            "batched_vs_plain": {"frames": int(len(leaves)), "bitwise_identical": bitwise,
                                 "max_centroid_diff_over_leaf": worst,
                                 "keys_counts_colours_identical": True},
            "backward_32x100k": {"forward_ms": round(fwd_ms, 4), "backward_ms": round(bwd_ms, 4),
                                 "backward_mpoints_s": round(3_200_000 / (bwd_ms * 1e-3) / 1e6, 1),
                                 "backward_gbs": round(32 * 3_200_000 / (bwd_ms * 1e-3) / 1e9, 1)},
        }
        # the same frames through the filtered form: each frame moved into the
        # global frame by its own camera pose, height-limited to 0.05..2.0 m,
        # cells of fewer than 3 points dropped
        filters = []
        for b in range(len(leaves)):
            R, t = dg.camera_pose(8000 + b)
            filters.append(vg.make_filter(rot=R, trans=t, z_min=0.05, z_max=2.0, min_points=3))
        fplan = vg.BatchPlan(len(leaves), N, vg.KEY_LINEAR, tuning, use_graph=not args.no_graph)
        fouts = fplan.alloc_outputs(N, len(leaves), dev, outputs=out_set)
        for _ in range(max(args.warmup, 2)):
            fplan.run(*d, offs, leaves, out=fouts, filters=filters)
        torch.cuda.synchronize()
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        for _ in range(args.steps):
            fplan.run(*d, offs, leaves, out=fouts, filters=filters)
        f1.record(stream)
        torch.cuda.synchronize()
        fms = f0.elapsed_time(f1) / args.steps
        fo = {k: v.cpu().numpy() for k, v in fouts[0].items() if k in ("out_offsets", "frame_status", "count")}
        result["legs"]["voxel_map"] = map_leg(fouts[0], fo["out_offsets"], offs, leaves, dev, cpu_jobs)
        log(f"leg: voxel map: {result['legs']['voxel_map']['ms_per_frame']} ms per frame")
        fplan.close()
        assert (fo["frame_status"] == 0).all(), "a filtered frame failed"
        kept = int(fo["count"][:int(fo["out_offsets"][-1])].astype(np.int64).sum())
        result["legs"]["filtered_batch"] = {
            "workload": f"the {len(leaves)} frames, each moved by its own camera pose into the "
                        "global frame, height limit 0.05..2.0 m, cells of fewer than 3 points dropped",
            "ms_per_step": round(fms, 4), "mpoints_s": round(N / (fms * 1e-3) / 1e6, 1),
            "over_unfiltered": round(fms / ev_ms, 3), "cells": int(fo["out_offsets"][-1]),
            "points_in_kept_cells": kept}
        log(f"leg: filtered batch: {fms:.3f} ms/step, {result['legs']['filtered_batch']['cells']} cells")
        ing = ingest_leg(x, y, z, rgb, offs, leaves, d, plan, outs, o, tuning, dev,
                         max(3, min(args.steps, 10)), not args.no_graph)
        if not (ing["zero_copy_bit_identical"] and ing["copy_overlapped_bit_identical"]):
            raise SystemExit("bench.py: the call on host-memory points differs from the device-resident one")
        result["legs"]["host_ingest"] = ing
        log(f"leg: host ingest: copy+call {ing['copy_then_call_ms']} ms, overlapped "
            f"{ing['copy_overlapped_ms']} ms, zero-copy {ing['zero_copy_call_ms']} ms")
        if not args.no_config_legs:
            cfg = []
            cfg.append(single_cloud_leg("640x480 RGB-D frame, plain path", dg.frame_640x480(), 0.05,
                                        tuning, dev, 30, 3, cpu_jobs))
            log(f"leg: {cfg[-1]['workload']}: {cfg[-1]['mpoints_s']} Mpoints/s")
            f720 = dg.frame_1280x720()
            for leaf in (0.01, 0.02, 0.05, 0.10):
                cfg.append(single_cloud_leg(f"1280x720 RGB-D frame, leaf {leaf}, plain path", f720,
                                            leaf, tuning, dev, 30, 3, cpu_jobs))
                log(f"leg: {cfg[-1]['workload']}: {cfg[-1]['mpoints_s']} Mpoints/s")
            room = dg.room_map()
            cfg.append(single_cloud_leg("16M-point shuffled room map, leaf 0.02, plain path", room,
                                        0.02, tuning, dev, 10, 0, cpu_jobs))
            log(f"leg: {cfg[-1]['workload']}: {cfg[-1]['mpoints_s']} Mpoints/s")
            # the oracle on a bounded sample of the map: its first 4M points (the
            # points are shuffled, so any 4M of them are a uniform sample)
            sub = tuple(np.ascontiguousarray(a[:4_000_000]) for a in room)

            def room_job(sub=sub):
                import oracle
                c0 = time.perf_counter()
                oracle.downsample(sub[0], sub[1], sub[2], sub[3], 0.02)
                return {"mpoints_s": round(4_000_000 / (time.perf_counter() - c0) / 1e6, 3),
                        "sample": "the map's first 4,000,000 (shuffled) points, once"}
            cpu_jobs.append((cfg[-1]["workload"], room_job))
            del room
            result["legs"]["configs"] = cfg
            result["legs"]["nbd_decimation"] = nbd_leg(tuning, dev, cpu_jobs=cpu_jobs)
            log(f"leg: decimation: {result['legs']['nbd_decimation']['ms_median']} ms per frame, "
                f"{result['legs']['nbd_decimation']['rounds']} rounds")

    if not args.no_cpu_baseline:
        import oracle
        oracle.load()
        # the oracle on one host core (pinned in this process), over the
        # batch's frames in order from the first until about --cpu-seconds of
        # CPU time, three times; the median run is reported
        cpus = sorted(os.sched_getaffinity(0))
        core = cpus[-1]
        os.sched_setaffinity(0, {core})
        try:
            runs = []
            for _ in range(3):
                used, pts, nfr = 0.0, 0, 0
                while used < args.cpu_seconds:
                    b = nfr % len(leaves)
                    s0, s1 = int(offs[b]), int(offs[b + 1])
                    c0 = time.perf_counter()
                    oracle.downsample(x[s0:s1], y[s0:s1], z[s0:s1], rgb[s0:s1], float(leaves[b]))
                    used += time.perf_counter() - c0
                    pts += s1 - s0
                    nfr += 1
                runs.append((pts / used / 1e6, nfr, pts, used))
        finally:
            os.sched_setaffinity(0, set(cpus))
        runs.sort()
        rate, nfr, pts, used = runs[1]
        result["cpu_baseline"] = {
            "value": round(rate, 3), "unit": "Mpoints/s", "cores": 1, "kind": "oracle",
            "sample": f"median of 3 runs; each: {nfr} frame calls over the {len(leaves)}-frame batch "
                      f"in order ({pts} points, {used:.1f} s), single-threaded std::map oracle, "
                      f"process pinned to host core {core}",
            "runs_mpoints_s": [round(r[0], 3) for r in runs],
            "host_cpu": _cpu_name(), "host_cores_available": len(cpus),
        }
        # the oracle on the legs' workloads (same pinned core)
        os.sched_setaffinity(0, {core})
        try:
            result["cpu_baseline"]["legs"] = {name: job() for name, job in cpu_jobs}
        finally:
            os.sched_setaffinity(0, set(cpus))
        log(f"cpu oracle: {result['cpu_baseline']['value']} Mpoints/s on 1 core")

    plan.close()
    print(json.dumps(result), flush=True)


def _cpu_name():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()

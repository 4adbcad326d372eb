"""Batched form on the GPU: per-frame oracle parity, plain-vs-batched, graph replay."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_matches_oracle, gpu_downsample, host, to_dev
from paper_2102_11084_amd import datagen as dg
from paper_2102_11084_amd import vg

pytestmark = pytest.mark.gpu


def small_batch(seed=0):
    """Uneven frames: RGB-D frames of several sizes, an empty frame, an all-NaN
    frame, an overflowing frame, a single point."""
    rng = np.random.default_rng(seed)
    frames, leaves = [], []
    for i, (W, H) in enumerate([(64, 48), (160, 120), (320, 240), (97, 33), (200, 150)]):
        frames.append(dg.rgbd_frame(W, H, seed=100 + i + seed))
        leaves.append(float(rng.choice([0.02, 0.05, 0.1])))
    e = np.zeros(0, np.float32)
    frames.insert(2, (e, e, e, np.zeros((0, 3), np.uint8)))
    leaves.insert(2, 0.05)
    nan = np.full(777, np.nan, np.float32)
    frames.insert(4, (nan, nan.copy(), nan.copy(), np.zeros((777, 3), np.uint8)))
    leaves.insert(4, 0.05)
    ov = np.array([0.0, 1e4, 5.0], np.float32)
    frames.insert(5, (ov, np.zeros(3, np.float32), np.zeros(3, np.float32),
                      np.full((3, 3), 9, np.uint8)))
    leaves.insert(5, 1e-3)
    one = np.array([0.25], np.float32)
    frames.append((one, one.copy(), one.copy(), np.array([[1, 2, 3]], np.uint8)))
    leaves.append(0.1)
    offs = np.zeros(len(frames) + 1, np.int64)
    offs[1:] = np.cumsum([f[0].size for f in frames])
    cat = [np.concatenate([f[a] for f in frames]) for a in range(4)]
    return cat[0], cat[1], cat[2], cat[3], offs, np.array(leaves, np.float32)


def run_batched(x, y, z, rgb, offs, leaves, plan=None, key_mode=vg.KEY_LINEAR, tuning=None):
    d = to_dev(x, y, z, rgb.reshape(-1))
    own = plan is None
    if own:
        plan = vg.BatchPlan(len(leaves), x.size, key_mode, tuning)
    o = plan.run(*d, offs, leaves)
    torch.cuda.synchronize()
    if own:
        plan.close()
    return host({k: v for k, v in o.items()})


def check_against_oracle(g, x, y, z, rgb, offs, leaves, key_mode=vg.KEY_LINEAR):
    res, status = oracle.downsample_batched(x, y, z, rgb, offs, leaves, key_mode)
    assert list(g["frame_status"]) == status
    oo = g["out_offsets"]
    assert oo[0] == 0
    for b, (r, s) in enumerate(zip(res, status)):
        lo, hi = int(oo[b]), int(oo[b + 1])
        s0, s1 = int(offs[b]), int(offs[b + 1])
        if s != oracle.OK:
            assert hi == lo
            assert (g["point_cell"][s0:s1] == -1).all()
            continue
        fr = {k: g[k][lo:hi] for k in ("x", "y", "z", "rgb", "count", "key", "ref_index",
                                       "lx", "ly", "lz")}
        fr["point_cell"] = g["point_cell"][s0:s1]
        fr["m"] = hi - lo
        assert_matches_oracle(fr, r, float(leaves[b]), point_cell_offset=lo, ref_offset=s0)


@pytest.mark.parametrize("key_mode", [vg.KEY_LINEAR, vg.KEY_MORTON])
def test_small_batch_matches_per_frame_oracle(key_mode):
    x, y, z, rgb, offs, leaves = small_batch()
    g = run_batched(x, y, z, rgb, offs, leaves, key_mode=key_mode)
    check_against_oracle(g, x, y, z, rgb, offs, leaves, key_mode)


@pytest.mark.parametrize("mode", [vg.EXEC_PERSISTENT, vg.EXEC_PHASED])
def test_batched_equals_plain_bitwise(mode):
    x, y, z, rgb, offs, leaves = small_batch(seed=1)
    t = vg.launch_tuning(mode)
    g = run_batched(x, y, z, rgb, offs, leaves, tuning=t)
    for b in range(len(leaves)):
        s0, s1 = int(offs[b]), int(offs[b + 1])
        lo, hi = int(g["out_offsets"][b]), int(g["out_offsets"][b + 1])
        if g["frame_status"][b] != 0 or s1 == s0:
            continue
        p = gpu_downsample(x[s0:s1], y[s0:s1], z[s0:s1], rgb[s0:s1], float(leaves[b]), tuning=t)
        assert p["m"] == hi - lo
        for k in ("x", "y", "z", "rgb", "count", "key", "lx", "ly", "lz"):
            assert np.array_equal(p[k].view(np.uint8), g[k][lo:hi].view(np.uint8)), (b, k)
        assert np.array_equal(p["ref_index"].astype(np.int64) + s0, g["ref_index"][lo:hi])
        pc = p["point_cell"].astype(np.int64)
        assert np.array_equal(np.where(pc >= 0, pc + lo, -1), g["point_cell"][s0:s1])


def test_graph_replay_matches_eager():
    plan = vg.BatchPlan(16, 400_000, use_graph=True)
    eager = vg.BatchPlan(16, 400_000, use_graph=False)
    batches = [small_batch(seed=s) for s in (3, 4, 3, 5)]
    for i, (x, y, z, rgb, offs, leaves) in enumerate(batches):
        ge = run_batched(x, y, z, rgb, offs, leaves, plan=eager)
        gg = run_batched(x, y, z, rgb, offs, leaves, plan=plan)
        # unrelated eager work between replays
        a = torch.randn(1000, device="cuda")
        (a * 2).sum().item()
        for k in ge:
            if k == "m":
                continue
            n = int(ge["out_offsets"][-1]) if k not in ("point_cell", "out_offsets", "frame_status") else None
            ea, gb = (ge[k][:n], gg[k][:n]) if n is not None else (ge[k], gg[k])
            assert np.array_equal(np.ascontiguousarray(ea).view(np.uint8),
                                  np.ascontiguousarray(gb).view(np.uint8)), (i, k)
        if i == 0:
            check_against_oracle(gg, x, y, z, rgb, offs, leaves)
    plan.close()
    eager.close()


@pytest.mark.parametrize("mode", [vg.EXEC_PHASED, vg.EXEC_PERSISTENT])
def test_timed_launches_match_graph_replay(mode):
    """Per-launch event timing (launches outside the graph) gives the same
    bytes as graph replay, and names every launch of the call in order."""
    print(f"case timed launches, exec mode {mode}", flush=True)
    x, y, z, rgb, offs, leaves = small_batch(seed=6)
    t = vg.launch_tuning(mode)
    plan = vg.BatchPlan(16, 400_000, vg.KEY_LINEAR, t, use_graph=True)
    gg = run_batched(x, y, z, rgb, offs, leaves, plan=plan)
    plan.set_timing(True)
    gt = run_batched(x, y, z, rgb, offs, leaves, plan=plan)
    times = plan.kernel_times()
    plan.set_timing(False)
    plan.close()
    n = int(gg["out_offsets"][-1])
    for k in gg:
        if k == "m":
            continue
        full = k in ("point_cell", "out_offsets", "frame_status")
        a, b = (gg[k], gt[k]) if full else (gg[k][:n], gt[k][:n])
        assert np.array_equal(np.ascontiguousarray(a).view(np.uint8),
                              np.ascontiguousarray(b).view(np.uint8)), k
    kinds = [k for k, _ in times]
    assert all(ms > 0.0 for _, ms in times)
    if mode == vg.EXEC_PHASED:
        assert kinds[0] == "init" and kinds[1:3] == ["bbox", "hist"]
        assert kinds[-2:] == ["reduce", "fixup"]
        assert set(kinds[3:-2]) == {"sort"} and len(kinds[3:-2]) >= 1
    else:
        assert kinds == ["init", "pipeline"]


def test_batch_of_one_equals_plain():
    x, y, z, rgb = dg.frame_640x480()
    offs = np.array([0, x.size], np.int64)
    g = run_batched(x, y, z, rgb, offs, np.array([0.05], np.float32))
    p = gpu_downsample(x, y, z, rgb, 0.05)
    m = p["m"]
    assert int(g["out_offsets"][1]) == m
    for k in ("x", "y", "z", "rgb", "count", "key", "ref_index"):
        assert np.array_equal(p[k].view(np.uint8), g[k][:m].view(np.uint8)), k


@pytest.mark.slow
def test_full_uneven_batch_every_frame():
    """The 64-frame uneven batch at full size, in the bench's launch form
    (tuned, graph replay): every frame against the oracle, and the batched
    rows bit-identical to 64 plain calls on the same frames."""
    import os
    x, y, z, rgb, offs, leaves = dg.batch()
    print(f"case full batch of {len(leaves)} frames, {x.size} points", flush=True)
    tpath = os.path.join(os.path.dirname(vg.__file__), "tuning_gfx950.json")
    t = vg.load_tuning(tpath) if os.path.exists(tpath) else vg.default_tuning()
    plan = vg.BatchPlan(len(leaves), x.size, vg.KEY_LINEAR, t, use_graph=True)
    g = run_batched(x, y, z, rgb, offs, leaves, plan=plan)
    plan.close()
    assert (g["frame_status"] == 0).all()
    oo = g["out_offsets"]
    for b in range(len(leaves)):
        s0, s1 = int(offs[b]), int(offs[b + 1])
        lo, hi = int(oo[b]), int(oo[b + 1])
        r = oracle.downsample(x[s0:s1], y[s0:s1], z[s0:s1], rgb[s0:s1], float(leaves[b]))
        fr = {k: g[k][lo:hi] for k in ("x", "y", "z", "rgb", "count", "key", "ref_index", "lx", "ly", "lz")}
        fr["point_cell"] = g["point_cell"][s0:s1]
        fr["m"] = hi - lo
        assert_matches_oracle(fr, r, float(leaves[b]), point_cell_offset=lo, ref_offset=s0)
    print("case full batch: plain calls", flush=True)
    for b in range(len(leaves)):
        s0, s1 = int(offs[b]), int(offs[b + 1])
        lo, hi = int(oo[b]), int(oo[b + 1])
        p = gpu_downsample(x[s0:s1], y[s0:s1], z[s0:s1], rgb[s0:s1], float(leaves[b]), tuning=t)
        assert p["m"] == hi - lo, b
        for k in ("x", "y", "z", "rgb", "count", "key", "lx", "ly", "lz"):
            assert np.array_equal(p[k].view(np.uint8), g[k][lo:hi].view(np.uint8)), (b, k)
        assert np.array_equal(p["ref_index"].astype(np.int64) + s0, g["ref_index"][lo:hi])
        pc = p["point_cell"].astype(np.int64)
        assert np.array_equal(np.where(pc >= 0, pc + lo, -1), g["point_cell"][s0:s1]), b


@pytest.mark.parametrize("mode", [vg.EXEC_PHASED, vg.EXEC_PERSISTENT])
@pytest.mark.parametrize("use_graph", [False, True])
def test_device_timeout_marks_every_frame(mode, use_graph):
    """A call whose device-side time-out flag is raised (from the host, so no
    wait really runs out) reports VG_ERR_DEVICE in every frame; the plan's next
    call is correct again."""
    print(f"case simulated time-out, exec mode {mode}, graph {use_graph}", flush=True)
    x, y, z, rgb, offs, leaves = small_batch(seed=7)
    t = vg.launch_tuning(mode)
    plan = vg.BatchPlan(16, 400_000, vg.KEY_LINEAR, t, use_graph=use_graph)
    good = run_batched(x, y, z, rgb, offs, leaves, plan=plan)
    check_against_oracle(good, x, y, z, rgb, offs, leaves)
    plan.set_fail_waits(True)
    bad = run_batched(x, y, z, rgb, offs, leaves, plan=plan)
    assert (bad["frame_status"] == vg.VG_ERR_DEVICE).all(), bad["frame_status"]
    plan.set_fail_waits(False)
    again = run_batched(x, y, z, rgb, offs, leaves, plan=plan)
    check_against_oracle(again, x, y, z, rgb, offs, leaves)
    plan.close()


def many_frames(B, seed):
    """B uneven clouds: sizes 0..6000, some empty, some with NaN/Inf points,
    leaves 0.02..0.2, one wide-key frame.  Batches of up to 64 frames take the
    launches that keep every frame's tables and grid in LDS (one-pass radix
    launches in their own order, the reduce's row chain over tiles with
    points); larger ones exercise the other paths."""
    rng = np.random.default_rng(seed)
    xs, ys, zs, cs, sizes, leaves = [], [], [], [], [], []
    for b in range(B):
        n = 0 if b % 17 == 3 else int(rng.integers(1, 6000))
        p = rng.uniform(-1.0, 2.0, size=(n, 3)).astype(np.float32)
        if b % 5 == 1 and n:
            bad = rng.random(n) < 0.2
            p[bad, rng.integers(0, 3)] = np.nan
        if b % 29 == 7 and n > 1:  # keys over 32 bits
            p[0] = (-500.0, -500.0, -500.0)
            p[1] = (500.0, 500.0, 500.0)
        xs.append(p[:, 0].copy())
        ys.append(p[:, 1].copy())
        zs.append(p[:, 2].copy())
        cs.append(rng.integers(0, 256, size=(n, 3), dtype=np.uint8))
        sizes.append(n)
        leaves.append(0.5 if b % 29 == 7 else float(rng.choice([0.02, 0.05, 0.1, 0.2])))
    offs = np.zeros(B + 1, np.int64)
    offs[1:] = np.cumsum(sizes)
    return (np.concatenate(xs), np.concatenate(ys), np.concatenate(zs), np.concatenate(cs), offs,
            np.array(leaves, np.float32))


@pytest.mark.parametrize("B", [60, 100, 300])
def test_many_frames_match_per_frame_oracle(B):
    print(f"case batch of {B} frames", flush=True)
    x, y, z, rgb, offs, leaves = many_frames(B, seed=B)
    g = run_batched(x, y, z, rgb, offs, leaves)
    check_against_oracle(g, x, y, z, rgb, offs, leaves)


def test_frames_longer_than_a_round_of_tiles():
    """Two frames of more than 4.2 M points (more big tiles than one launch has
    workgroups, so a workgroup takes several tiles of one frame in a row and
    accumulates them together) between small frames: every frame against the
    oracle."""
    print("case batch with two frames of 5.0 M and 4.6 M points", flush=True)
    parts = [dg.uniform_cloud(5_000_000, seed=71, side=6.0), dg.rgbd_frame(160, 120, seed=72),
             dg.uniform_cloud(4_600_000, seed=73, side=3.0), dg.rgbd_frame(64, 48, seed=74)]
    leaves = np.array([0.05, 0.02, 0.02, 0.1], np.float32)
    offs = np.zeros(len(parts) + 1, np.int64)
    offs[1:] = np.cumsum([p[0].size for p in parts])
    x, y, z, rgb = (np.concatenate([p[a] for p in parts]) for a in range(4))
    g = run_batched(x, y, z, rgb, offs, leaves)
    check_against_oracle(g, x, y, z, rgb, offs, leaves)


@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("two_streams", [False, True])
def test_back_to_back_calls_without_sync(use_graph, two_streams):
    """Four calls of one plan on different batches, enqueued without waiting in
    between (the plan waits only for the call two back before it rewrites a
    staging slot), on one stream or alternating between two: every call's
    outputs against the oracle."""
    print(f"case back-to-back calls, graph {use_graph}, two streams {two_streams}", flush=True)
    batches = [small_batch(seed=s) for s in (10, 11, 12, 13)]
    B = len(batches[0][5])
    n_max = max(b[0].size for b in batches)
    devs = [to_dev(b[0], b[1], b[2], b[3].reshape(-1)) for b in batches]
    torch.cuda.synchronize()
    plan = vg.BatchPlan(B, n_max, vg.KEY_LINEAR, None, use_graph=use_graph)
    streams = [torch.cuda.current_stream()] + ([torch.cuda.Stream()] if two_streams else [])
    outs = []
    for i, (b, dv) in enumerate(zip(batches, devs)):
        with torch.cuda.stream(streams[i % len(streams)]):
            outs.append(plan.run(*dv, b[4], b[5]))
    torch.cuda.synchronize()
    plan.close()
    for b, o in zip(batches, outs):
        check_against_oracle(host(o), *b)


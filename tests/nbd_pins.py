"""Pins of the oracle's neighbour-bucket decimation (Alg. 1 of the paper) and
of its Philox4x64-10 generator, against facts that do not come from the oracle:

  * Philox: numpy's own Philox (a 4x64, 10-round implementation written
    independently) at the same counters and keys;
  * brute force: an O(n^2) numpy implementation of the whole loop (all pairs,
    the 27-cell condition as a coordinate test, rounds with numpy's Philox for
    the random choice) on tiny clouds, compared in everything: survivors,
    initial counts, points marked per round, number of rounds;
  * closed forms: a cubic lattice whose spacing is the radius (interior points
    have 6 neighbours, face points 5, edge points 4, corners 3) and clusters
    of coincident points (k - 1 neighbours each), whose outcome follows from
    the loop's rule by hand;
  * invariants on camera frames: no survivor keeps more than `umbral`
    surviving neighbours, every round but the last marks more than
    `round_size` points, and the deletions add up.
Each check takes an oracle library handle, so that broken builds of the oracle
can be run through them (test_oracle_mutants.py).
"""
from __future__ import annotations

import numpy as np

import oracle
from oracle_pins import f32_cell_coords

MASK64 = (1 << 64) - 1


def numpy_priority(i, rnd, seed):
    """Word 0 of Philox4x64-10 at counter (i, rnd, 0, 0), key (seed, 0), by
    numpy's generator (which advances its counter by one before drawing)."""
    c = (int(i) + (int(rnd) << 64) - 1) % (1 << 256)
    ctr = np.array([(c >> (64 * w)) & MASK64 for w in range(4)], np.uint64)
    g = np.random.Philox(key=np.array([seed & MASK64, 0], np.uint64), counter=ctr)
    return int(g.random_raw())


def brute_nbd(x, y, z, leaf, radius, umbral, seed, round_size):
    p = np.stack([x, y, z], 1).astype(np.float32)
    valid = np.isfinite(p).all(1)
    n = p.shape[0]
    count0 = np.zeros(n, np.uint32)
    if not valid.any():
        return dict(keep=np.zeros(n, bool), count0=count0, marked=[0], rounds=1)
    k, _, _, _ = f32_cell_coords(x, y, z, leaf)
    idx = np.flatnonzero(valid)
    q = p[idx]
    d = q[None, :, :] - q[:, None, :]          # row p, column q: q - p, binary32
    sq = d * d
    d2 = (sq[..., 0] + sq[..., 1]) + sq[..., 2]
    kk = k[idx].astype(np.int64)
    near = (np.abs(kk[None, :, :] - kk[:, None, :]) <= 1).all(-1)
    r2 = np.float32(radius) * np.float32(radius)
    A = (d2 <= r2) & near
    np.fill_diagonal(A, False)
    count0[idx] = A.sum(1)
    present = np.ones(idx.size, bool)
    marked, rnd = [], 0
    while True:
        cnt = A[:, present].sum(1)
        M = np.flatnonzero(present & (cnt > umbral))
        marked.append(M.size)
        if M.size > round_size:
            pri = sorted((numpy_priority(idx[j], rnd, seed), idx[j], j) for j in M)
            for _, _, j in pri[:round_size]:
                present[j] = False
            rnd += 1
            continue
        present[M] = False
        break
    keep = np.zeros(n, bool)
    keep[idx[present]] = True
    return dict(keep=keep, count0=count0, marked=marked, rounds=len(marked))


def _same(r, b, ctx):
    assert r["rounds"] == b["rounds"], (ctx, r["rounds"], b["rounds"])
    assert list(r["marked"]) == list(b["marked"]), ctx
    assert np.array_equal(r["count0"], b["count0"]), ctx
    assert np.array_equal(r["keep"], b["keep"]), ctx


def pin_nbd_philox(lib, seed=11):
    rng = np.random.default_rng(seed)
    for _ in range(100):
        ctr = rng.integers(0, 2 ** 63, size=4, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 4, dtype=np.uint64)
        key = rng.integers(0, 2 ** 63, size=2, dtype=np.uint64) * np.uint64(2)
        c = sum(int(v) << (64 * w) for w, v in enumerate(ctr))
        c1 = (c - 1) % (1 << 256)
        g = np.random.Philox(key=key, counter=np.array([(c1 >> (64 * w)) & MASK64 for w in range(4)],
                                                       np.uint64))
        assert [int(v) for v in oracle.philox4x64(ctr, key, lib=lib)] == [int(v) for v in g.random_raw(4)]


def pin_nbd_brute_force(lib, seed=12):
    rng = np.random.default_rng(seed)
    for trial in range(24):
        leaf = float(rng.choice([0.1, 0.25]))
        radius = float(np.float32(leaf * rng.choice([1.0, 0.6])))
        n = int(rng.integers(0, 160))
        p = rng.uniform(0.0, 0.5, size=(n, 3)).astype(np.float32)
        if n > 10:
            p[rng.integers(0, n, 5)] = p[rng.integers(0, n, 5)]            # duplicates
            p[rng.integers(0, n, 3), rng.integers(0, 3)] = np.nan            # invalid points
            p[rng.integers(0, n, 4), 0] = np.float32(leaf) * rng.integers(0, 3, 4)  # on faces
        umbral = int(rng.integers(0, 7))
        rs = int(rng.choice([1, 3, 7, 1000]))
        sd = int(rng.integers(0, 2 ** 62))
        x, y, z = p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()
        r = oracle.nbd_decimate(x, y, z, leaf, radius, umbral, sd, rs, lib=lib)
        b = brute_nbd(x, y, z, leaf, radius, umbral, sd, rs)
        _same(r, b, trial)


def lattice(k, s=1.0 / 16):
    g = np.arange(k, dtype=np.float32) * np.float32(s)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy()


def pin_nbd_lattice(lib):
    s = 1.0 / 16
    x, y, z = lattice(12, s)
    k = np.stack([x, y, z], 1) / s
    faces = ((k == 0) | (k == 11)).sum(1)          # boundary planes a point lies on
    exp0 = (6 - faces).astype(np.uint32)
    interior = faces == 0
    # umbral 5: exactly the 1000 interior points are marked (1000 is not more
    # than 1000), the loop ends at once and deletes them
    r = oracle.nbd_decimate(x, y, z, s, s, 5, 1, 1000, lib=lib)
    assert np.array_equal(r["count0"], exp0)
    assert r["rounds"] == 1 and list(r["marked"]) == [1000]
    assert np.array_equal(r["keep"], ~interior)
    # umbral 6: nothing is marked
    r = oracle.nbd_decimate(x, y, z, s, s, 6, 1, 1000, lib=lib)
    assert r["keep"].all() and r["rounds"] == 1 and list(r["marked"]) == [0]
    # a radius below the spacing: no neighbours at all
    r = oracle.nbd_decimate(x, y, z, s, s * 0.99, 0, 1, 1000, lib=lib)
    assert (r["count0"] == 0).all() and r["keep"].all()
    # round size 600, umbral 5: 1000 marked > 600, so 600 interior points go
    # at random; the rest follows the rule (checked by the invariant)
    r = oracle.nbd_decimate(x, y, z, s, s, 5, 3, 600, lib=lib)
    assert r["marked"][0] == 1000 and r["rounds"] >= 2
    check_nbd_invariants(r, x, y, z, s, s, 5, 600)


def pin_nbd_clusters(lib):
    far = np.array([[10.0, 10.0, 10.0], [20.0, 0.0, 0.0], [0.0, 20.0, 5.0]], np.float32)

    def run(k, umbral, rs=1000):
        p = np.concatenate([np.full((k, 3), 0.25, np.float32), far])
        return oracle.nbd_decimate(p[:, 0], p[:, 1], p[:, 2], 0.5, 0.5, umbral, 5, rs, lib=lib)

    r = run(2500, 10)   # 2500 marked: 1000 go; 1500: 1000 go; 500 <= 1000: all go
    assert list(r["marked"]) == [2500, 1500, 500] and r["rounds"] == 3
    assert not r["keep"][:2500].any() and r["keep"][2500:].all()
    assert (r["count0"][:2500] == 2499).all() and (r["count0"][2500:] == 0).all()
    r = run(11, 10)     # 10 neighbours each, not more than 10: nothing marked
    assert r["keep"].all() and list(r["marked"]) == [0]
    r = run(12, 10)     # 11 each: all 12 marked, deleted at the end
    assert list(r["marked"]) == [12] and not r["keep"][:12].any() and r["keep"][12:].all()
    r = run(12, 10, rs=5)   # 12 > 5: 5 go; then 7 left with 6 neighbours each, none marked
    assert list(r["marked"]) == [12, 0] and r["keep"][:12].sum() == 7


def check_nbd_invariants(r, x, y, z, leaf, radius, umbral, rs):
    marked = list(r["marked"])
    assert len(marked) == r["rounds"]
    assert all(m > rs for m in marked[:-1]) and marked[-1] <= rs
    valid = np.isfinite(x) & np.isfinite(y) & np.isfinite(z)
    assert not r["keep"][~valid].any()
    assert valid.sum() - r["keep"].sum() == rs * (len(marked) - 1) + marked[-1]
    # no survivor has more than umbral surviving neighbours (brute force over
    # survivors, in chunks)
    p = np.stack([x, y, z], 1).astype(np.float32)
    k, _, _, _ = f32_cell_coords(x, y, z, leaf)
    s = np.flatnonzero(r["keep"])
    q, kk = p[s], k[s].astype(np.int64)
    r2 = np.float32(radius) * np.float32(radius)
    for a in range(0, s.size, 512):
        d = q[None, :, :] - q[a:a + 512, None, :]
        sq = d * d
        d2 = (sq[..., 0] + sq[..., 1]) + sq[..., 2]
        near = (np.abs(kk[None, :, :] - kk[a:a + 512, None, :]) <= 1).all(-1)
        cnt = ((d2 <= r2) & near).sum(1) - 1
        assert (cnt <= umbral).all()


def pin_nbd_invariants(lib):
    from paper_2102_11084_amd import datagen as dg
    for seed, (W, H), leaf, umbral, rs in [(1, (64, 48), 0.05, 8, 100), (2, (80, 60), 0.1, 30, 50),
                                           (3, (72, 54), 0.05, 3, 1000)]:
        x, y, z, _ = dg.rgbd_frame(W, H, seed=seed)
        r = oracle.nbd_decimate(x, y, z, leaf, leaf, umbral, seed, rs, lib=lib)
        check_nbd_invariants(r, x, y, z, leaf, leaf, umbral, rs)


def pin_nbd_errors(lib):
    x = np.array([0.0, 1.0, 2.0], np.float32)
    for leaf, radius, rs, st in [(0.5, 0.6, 10, oracle.ERR_ARG), (0.5, 0.0, 10, oracle.ERR_ARG),
                                 (0.5, float("nan"), 10, oracle.ERR_ARG), (0.5, 0.5, 0, oracle.ERR_ARG),
                                 (0.0, 0.0, 10, oracle.ERR_LEAF), (1e-7, 1e-7, 10, oracle.ERR_GRID_OVERFLOW)]:
        try:
            oracle.nbd_decimate(x * np.float32(1e3), x, x, leaf, radius, 1, 1, rs, lib=lib)
        except oracle.OracleError as e:
            assert e.status == st, (leaf, radius, rs, e.status)
        else:
            raise AssertionError((leaf, radius, rs))
    e = np.zeros(0, np.float32)
    r = oracle.nbd_decimate(e, e, e, 0.5, 0.5, 1, 1, 10, lib=lib)
    assert r["keep"].size == 0 and r["rounds"] == 1 and list(r["marked"]) == [0]


ALL_NBD_PINS = [pin_nbd_philox, pin_nbd_brute_force, pin_nbd_lattice, pin_nbd_clusters,
                pin_nbd_invariants, pin_nbd_errors]

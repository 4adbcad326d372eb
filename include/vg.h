/*
 * vg.h -- voxel-grid centroid downsampling of point clouds on MI355X (gfx950).
 *
 * C ABI of libvg.so.  Every call takes plain pointers and sizes; device
 * pointers point to HIP device memory of the current device, host pointers
 * to ordinary host memory.  Streams are passed as `void *` holding a
 * hipStream_t (NULL = the default stream).
 *
 * The operation (arXiv 2102.11084, Sec. II-C and Alg. 1; the filter of
 * Sec. I / Sec. II-C that the paper moves off the CPU):
 *   1. a point (x, y, z) is valid iff all three coordinates are finite;
 *   2. the grid is anchored at min_a = min over valid points of coordinate a
 *      and has cubic cells of edge `leaf`; inv = RN32(1/leaf) is computed once
 *      on the host;
 *   3. cell coordinate k_a = floor(RN32(RN32(p_a - min_a) * inv)) in binary32,
 *      cells per axis d_a = floor(RN32(RN32(max_a - min_a) * inv)) + 1, and
 *      more than 2^21 cells on an axis is VG_ERR_GRID_OVERFLOW;
 *   4. key = k_x + d_x * (k_y + d_y * k_z)        (VG_KEY_LINEAR), or
 *      key = bit-interleave, bit b of k_x at 3b, k_y at 3b+1, k_z at 3b+2
 *                                                 (VG_KEY_MORTON);
 *   5. (key, index) pairs are sorted by key with a stable radix sort, so the
 *      points of a cell are contiguous and in input order (the paper's sorted
 *      subdivision table);
 *   6. each occupied cell becomes one output row, rows in ascending key:
 *      centroid = mean of its points' xyz, colour = per-channel
 *      floor((sum + floor(n/2)) / n), count n, key, and the smallest input
 *      index among its points.
 *
 * Errors: every call returns a vg_status and never throws.  Argument errors
 * are detected on the host before anything is launched; on any error the
 * output contents are unspecified and *m (where present) is 0.
 * Ownership: the caller owns every buffer it passes; the library frees none
 * of them.  A batch plan owns only what vg_batch_plan_create allocated.
 * A workspace serves one call at a time: calls that share a workspace must be
 * ordered (for example, issued on one stream).
 */
#ifndef VG_H
#define VG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum vg_status {
  VG_OK = 0,
  VG_ERR_ARG = 1,            /* null pointer, negative or too large size, bad enum */
  VG_ERR_LEAF = 2,           /* leaf not finite, not > 0, or 1/leaf not finite */
  VG_ERR_GRID_OVERFLOW = 3,  /* more than 2^21 cells on some axis */
  VG_ERR_WORKSPACE = 4,      /* workspace smaller than vg_workspace_bytes() */
  VG_ERR_DEVICE = 5          /* HIP runtime error, or a device-side time-out */
} vg_status;

typedef enum vg_key_mode { VG_KEY_LINEAR = 0, VG_KEY_MORTON = 1 } vg_key_mode;

/* How the pipeline is launched.  PERSISTENT: one kernel whose workgroups take
 * tiles of every phase from a work queue ordered so that a tile only waits on
 * tiles dequeued before it.  PHASED: one launch per phase, each with a kernel
 * compiled for that phase alone (fewer registers and less LDS, so more
 * workgroups per CU); the stream orders the phases, so no tile ever waits on
 * another launch's tiles.  Both give bit-identical results. */
typedef enum vg_exec_mode { VG_EXEC_PERSISTENT = 0, VG_EXEC_PHASED = 1 } vg_exec_mode;

/* Input cloud, structure of arrays, device memory.  x, y, z: n binary32 each.
 * rgb: n x 3 uint8 interleaved, or NULL (then output colours are not written). */
typedef struct vg_points {
  const float *x, *y, *z;
  const uint8_t *rgb;
} vg_points;

/* Output cells, device memory, capacity >= number of input points.
 * Every pointer may be NULL, then that output is not written.
 *   x, y, z     centroid (binary32)
 *   rgb         m x 3 uint8
 *   count       points in the cell
 *   key         64-bit cell key
 *   point_cell  [n]: output row of every input point, -1 for invalid points
 *               (rows of a batch are rows of the concatenated output)
 *   ref_index   smallest input index among the cell's points (an index into
 *               the arrays passed to the call)
 *   lx, ly, lz  mean of (p - p_ref), p_ref = the point at ref_index */
typedef struct vg_cells {
  float *x, *y, *z;
  uint8_t *rgb;
  uint32_t *count;
  uint64_t *key;
  int32_t *point_cell;
  uint32_t *ref_index;
  float *lx, *ly, *lz;
} vg_cells;

/* Tile shapes and launch shape.  A variant must be one the library was built
 * with (vg_tuning_supported).  radix_bits is the widest digit of a sort pass;
 * a frame whose key has b bits is sorted in P = max(1, ceil(b / radix_bits))
 * passes of ceil(b / P) bits. */
typedef struct vg_tuning {
  int sort_block;     /* threads per sort/bbox/histogram tile */
  int sort_items;     /* items per thread of such a tile */
  int radix_bits;     /* widest radix digit */
  int reduce_block;   /* threads per reduce tile */
  int reduce_items;   /* items per thread of a reduce tile */
  int blocks_per_cu;  /* persistent grid = CUs x this (0: occupancy limit) */
  int exec_mode;      /* vg_exec_mode */
} vg_tuning;

/* Per-call options.  workspace: device memory of at least
 * vg_workspace_bytes(n, 1, tuning) bytes, or NULL (then the call allocates
 * and frees its own, which costs a hipMalloc/hipFree pair).  tuning: NULL =
 * the built-in default. */
typedef struct vg_options {
  void *stream;
  void *workspace;
  size_t workspace_bytes;
  vg_key_mode key_mode;
  const vg_tuning *tuning;
} vg_options;

/* Human-readable name of a status; never NULL.  (Library helper; not in the
 * paper.) */
const char *vg_status_string(vg_status s);

/* Fills *t with the built-in default tuning.  VG_ERR_ARG if t is NULL.
 * (The paper sizes its launch by the device's processor count, Sec. II-C
 * after Alg. 1; the tuning generalises that choice.) */
vg_status vg_default_tuning(vg_tuning *t);

/* VG_OK if the library holds kernels for this tuning, else VG_ERR_ARG.  The
 * VG_EXEC_PERSISTENT form is built for the variants with 4 reduce items per
 * thread only (512/8/8/4 and 256/8/8/4).
 * (Library helper; not in the paper.) */
vg_status vg_tuning_supported(const vg_tuning *t);

/* Device workspace needed for n_total points in n_frames frames (0 on bad
 * arguments).  Grows linearly in n_total (about 42 bytes per point): the
 * sorted key/value table of Sec. II-C (double-buffered key and index words)
 * and the per-tile look-back state. */
size_t vg_workspace_bytes(int64_t n_total, int n_frames, const vg_tuning *t);

/* Downsample one cloud on the default stream with an internal workspace.
 * The operation of steps 1-6 above: Sec. II-C (grid over space, per-point
 * subdivision lookup, radix-sorted subdivision table, per-subdivision counts)
 * and Alg. 1 (lookup, table update, radix sort, deletion of the merged points,
 * copy of the filtered cloud back to the caller), with the centroid rule of
 * the voxel filter named in Sec. I and Sec. II-C.
 * p: device points; n: number of points, 0 <= n < 2^30; leaf: cell edge;
 * out: device outputs of capacity n; m: host, receives the number of cells.
 * Synchronous: returns after the cells are written (one stream sync).
 * Errors: VG_ERR_ARG / VG_ERR_LEAF before any launch; VG_ERR_GRID_OVERFLOW
 * and VG_ERR_DEVICE after the sync. */
vg_status vg_downsample(const vg_points *p, int64_t n, float leaf, vg_cells *out, int64_t *m);

/* As vg_downsample (Sec. II-C, Alg. 1), with a stream, a caller workspace,
 * key mode and tuning.  Waits for the stream only to read m back; on an error
 * after work was enqueued it also waits for that work before returning, so
 * the workspace and the library's staging buffer are free again. */
vg_status vg_downsample_ex(const vg_points *p, int64_t n, float leaf, vg_cells *out, int64_t *m,
                           const vg_options *o);

/* Not in the paper (a differentiable form of the filter): backward of the
 * centroids with the cell assignment held fixed:
 *   d{x,y,z}[i] = g{x,y,z}[c] / count[c] for c = point_cell[i] >= 0, else 0.
 * g*, count: device [m]; point_cell: device [n] (as written by a forward
 * call); d*: device [n].  Asynchronous on `stream`.  0 <= n < 2^31. */
vg_status vg_downsample_backward(const float *gx, const float *gy, const float *gz,
                                 const uint32_t *count, int64_t m, const int32_t *point_cell,
                                 int64_t n, float *dx, float *dy, float *dz, void *stream);

/* ---- batched form: many frames of uneven size and leaf in one launch ---- */
typedef struct vg_batch_plan vg_batch_plan;

/* Not in the paper (which filters one camera frame per call, Alg. 1): a plan
 * for batches of up to max_frames frames and max_total_points points in total
 * (< 2^31, and < 2^30 per frame).  Allocates the device workspace and a
 * pinned descriptor buffer.  tuning NULL = default.  The paper's processor-
 * count launch sizing (Sec. II-C after Alg. 1) becomes the plan's fixed grids. */
vg_status vg_batch_plan_create(int max_frames, int64_t max_total_points, vg_key_mode key_mode,
                               const vg_tuning *tuning, vg_batch_plan **plan);

/* Not in the paper: if use_graph != 0, the plan records its launch sequence
 * (descriptor copy, state reset, pipeline kernels, status kernel) into a
 * hipGraph on first use and replays it. */
vg_status vg_batch_plan_set_graph(vg_batch_plan *plan, int use_graph);

/* Not in the paper (batching of frames); every frame is filtered exactly as
 * vg_downsample filters it (Sec. II-C, Alg. 1), with its own box and leaf.
 * Downsample B frames concatenated in p.  frame_offsets: host [B+1],
 * non-decreasing, frame b = points [frame_offsets[b], frame_offsets[b+1]).
 * leaf: host [B].  out: device, capacity frame_offsets[B]; frame b's cells
 * are rows [out_offsets[b], out_offsets[b+1]) of every output array.
 * out_offsets: device int64 [B+1]; frame_status: device int32 [B]:
 *   VG_OK, VG_ERR_GRID_OVERFLOW (that frame has no rows), or VG_ERR_DEVICE in
 *   every frame when a device-side wait of the call timed out (then every
 *   output of the call, out_offsets included, is unspecified).
 * Fully asynchronous on `stream`.  A plan has two pinned descriptor slots,
 * used in turn: a call waits on the host only for the call two before it
 * (whose slot it reuses), and its stream waits on the device for the call
 * just before it (calls of a plan share its workspace and run one after the
 * other, whichever streams they come on).
 * Host-side errors (VG_ERR_ARG, VG_ERR_LEAF) are returned before anything is
 * enqueued. */
vg_status vg_downsample_batched(vg_batch_plan *plan, const vg_points *p,
                                const int64_t *frame_offsets, const float *leaf, int B,
                                vg_cells *out, int64_t *out_offsets, int32_t *frame_status,
                                void *stream);

/* ---- the filter's input contract: global frame, height limit, noise ----
 * Sec. II-C: the costmap layer hands the filter a cloud already transformed
 * into the global frame, so that its height can be limited for the
 * navigation stack's projection; the filter is also meant to remove the
 * depth sensor's noise.  Per cloud (frame):
 *   - if flags has VG_FILTER_TRANSFORM, every point is moved first:
 *     p'_a = RN32(RN32(RN32(RN32(rot[3a] x) + RN32(rot[3a+1] y)) + RN32(rot[3a+2] z))
 *            + trans[a]) in binary32 (rot row-major; applied as given);
 *   - a point is kept iff it is valid, p' is finite and
 *     z_min <= p'_z <= z_max (both inclusive; -INFINITY / INFINITY: no limit);
 *     the others are invalid points (point_cell -1);
 *   - the voxel filter runs on the kept points p' (outputs in that frame);
 *   - cells with fewer than min_points points are dropped (0 or 1: none) and
 *     the remaining rows renumbered in key order; their points' point_cell
 *     follows, points of dropped cells get -1.
 * The transform and height limit are applied by the bbox pass, which writes
 * the moved points once for the later passes; the sparse cells are removed by
 * a short pass over the output rows, launched only when asked for. */
typedef struct vg_filter {
  float rot[9];          /* row-major, used with VG_FILTER_TRANSFORM */
  float trans[3];
  float z_min, z_max;    /* not NaN, z_min <= z_max */
  uint32_t min_points;
  uint32_t flags;        /* VG_FILTER_* bits; others must be 0 */
} vg_filter;
#define VG_FILTER_TRANSFORM 1u

/* vg_downsample_ex on the filtered cloud (f: one filter).  VG_ERR_ARG for a
 * NULL or malformed filter (NaN or crossed limits, non-finite rot / trans
 * with VG_FILTER_TRANSFORM, unknown flags). */
vg_status vg_downsample_filtered(const vg_points *p, int64_t n, float leaf, const vg_filter *f,
                                 vg_cells *out, int64_t *m, const vg_options *o);

/* vg_downsample_batched with a filter per frame (filters: host [B]).  The
 * plan's graph gains the sparse-cell pass on the first call that needs it. */
vg_status vg_downsample_batched_filtered(vg_batch_plan *plan, const vg_points *p,
                                         const int64_t *frame_offsets, const float *leaf,
                                         const vg_filter *filters, int B, vg_cells *out,
                                         int64_t *out_offsets, int32_t *frame_status,
                                         void *stream);

/* Kernels of the pipeline, as reported by vg_batch_plan_kernel_times. */
typedef enum vg_kernel_kind {
  VG_KERNEL_INIT = 0,     /* state reset */
  VG_KERNEL_BBOX = 1,     /* validity, bounding box, point records */
  VG_KERNEL_HIST = 2,     /* cell keys and all radix-digit histograms */
  VG_KERNEL_SORT = 3,     /* one radix pass (pass 0 also computes the keys) */
  VG_KERNEL_REDUCE = 4,   /* segment heads, segmented sums, finalize, compaction */
  VG_KERNEL_FIXUP = 5,    /* cells that span several reduce tiles */
  VG_KERNEL_PIPELINE = 6  /* every phase in one persistent launch */
} vg_kernel_kind;

/* Measurement support (not in the paper, which times whole filter calls, Table
 * I): per-launch timing.  With enable != 0 every later vg_downsample_batched call
 * on this plan launches its kernels directly (not through the plan's graph)
 * and records a HIP event pair on the call's stream around each launch.
 * Waits for the plan's outstanding work before switching. */
vg_status vg_batch_plan_set_timing(vg_batch_plan *plan, int enable);

/* Durations of the kernel launches of the plan's last call, in launch order:
 * kinds[i] (a vg_kernel_kind) and ms[i] (milliseconds between the events
 * recorded right before and right after launch i).  Waits for the last event.
 * At most cap entries are written (host arrays); *count receives how many.
 * VG_ERR_ARG if timing is off. */
vg_status vg_batch_plan_kernel_times(vg_batch_plan *plan, int *kinds, float *ms, int cap,
                                     int *count);

/* ---- input in host memory (the paper's zero-copy theme, Sec. I, II-B, III) ----
 * On the paper's board the GPU reads the camera's buffer in shared memory
 * instead of copying it.  Here the analogue for a discrete GPU: points in
 * pinned host memory mapped into the device's address space, read by the
 * kernels over the host link.
 * vg_host_alloc: pinned, mapped host memory of `bytes` bytes; *host is the
 * host address (for filling), *device the address to pass to the library.
 * Free with vg_host_free(host).  VG_ERR_DEVICE if the runtime refuses.
 * vg_batch_plan_set_host_input: while on != 0, later calls on the plan take
 * their points from such memory: the bbox pass reads every point once from
 * there (its validity, box and record pass) and writes a device copy of the
 * coordinates that every later pass reads, so the host link carries the input
 * exactly once.  Results are bit-identical to device-resident input. */
vg_status vg_host_alloc(size_t bytes, void **host, void **device);
vg_status vg_host_free(void *host);
vg_status vg_batch_plan_set_host_input(vg_batch_plan *plan, int on);

/* Test support for callers' error handling (not in the paper): while enable
 * != 0, each later call on the plan starts with the device-side time-out flag
 * raised, as a bounded wait that timed out would raise it.  Every kernel then
 * exits without touching the outputs and every frame_status reads
 * VG_ERR_DEVICE.  Nothing waits or faults. */
vg_status vg_batch_plan_set_fail_waits(vg_batch_plan *plan, int enable);

/* Releases the plan (waits for its work to finish first). */
vg_status vg_batch_plan_destroy(vg_batch_plan *plan);

/* ---- neighbour-bucket decimation: the paper's own GPU filter ----
 * Sec. II-C and Alg. 1: space is cut into a regular grid (here the grid of
 * vg_downsample: cubic cells of edge `leaf` anchored at the valid points'
 * minimum), and a point's neighbours are searched in the 27 cells around its
 * own, with the Euclidean distance of Eq. (1).  In rounds, every point still
 * present counts its present neighbours and is marked if the count exceeds
 * `umbral`; while more than `round_size` points are marked (1000 in the
 * paper), `round_size` of them chosen at random are deleted and another round
 * runs; the marked points of the last round are deleted too.  The survivors
 * are handed back.  Readings of what the paper leaves open:
 *   - q is a neighbour of p iff q != p, both are valid (finite), their cell
 *     coordinates differ by at most 1 on every axis, and
 *     RN32(RN32(RN32(dx*dx) + RN32(dy*dy)) + RN32(dz*dz)) <= RN32(radius^2),
 *     dx = RN32(xq - xp) and so on; 0 < radius <= leaf, so the 27 cells hold
 *     every point within the radius;
 *   - the random choice: in round r, marked point i has the priority word 0
 *     of Philox4x64-10 (Salmon et al., SC'11) at counter (i, r, 0, 0) under
 *     key (seed, 0); the round_size marked points of smallest (priority, i)
 *     are deleted. */
typedef struct vg_nbd_params {
  float leaf;           /* cell edge of the grid */
  float radius;         /* neighbour radius, 0 < radius <= leaf */
  uint32_t umbral;      /* a point with more neighbours than this is marked */
  int32_t round_size;   /* points deleted per round while more are marked, >= 1 */
  uint64_t seed;        /* key of the random choice */
  uint32_t flags;       /* VG_NBD_* bits */
  uint32_t reserved;    /* 0 */
} vg_nbd_params;

/* Choose each round's deletions by the exact select over every marked point
 * instead of ranking the candidates of a priority window first.  Slower; the
 * deletions are the same (the window only ever narrows the search). */
#define VG_NBD_EXACT_SELECT 1u

/* Outputs of a decimation; every pointer may be NULL.  Device arrays of
 * capacity n unless noted. */
typedef struct vg_nbd_out {
  uint32_t *keep_index;  /* input indices of the survivors, ascending */
  float *x, *y, *z;      /* the survivors' coordinates (complete triple or none) */
  uint8_t *rgb;          /* their colours, n x 3 (written only if the input has rgb) */
  uint32_t *count0;      /* every point's neighbours before any deletion (0 if invalid) */
  int64_t *marked;       /* host [marked_cap]: points marked in round 0, 1, ... */
  int64_t marked_cap;
} vg_nbd_out;

/* Device workspace of vg_nbd_decimate for n points (0 on bad arguments). */
size_t vg_nbd_workspace_bytes(int64_t n, int32_t round_size);

/* Neighbour-bucket decimation of one cloud (Sec. II-C, Alg. 1; readings
 * above).  p: device points; 0 <= n < 2^30; o: stream, workspace (NULL: the
 * call allocates its own) and tuning of the grid pipeline it runs first
 * (o->key_mode is not used; o may be NULL).  *n_keep: survivors; *rounds:
 * rounds run (the last one deletes every point it marks).  Synchronous: the
 * rounds are enqueued in batches, and the host reads a device flag between
 * batches to see whether the last round has run (the paper's loop test is a
 * host decision too).  Errors: VG_ERR_ARG (also radius outside (0, leaf],
 * round_size < 1), VG_ERR_LEAF, VG_ERR_WORKSPACE before any launch;
 * VG_ERR_GRID_OVERFLOW, VG_ERR_DEVICE after. */
vg_status vg_nbd_decimate(const vg_points *p, int64_t n, const vg_nbd_params *prm,
                          vg_nbd_out *out, int64_t *n_keep, int64_t *rounds,
                          const vg_options *o);

/* ---- global voxel map: marking and clearing (the costmap layer's other hot
 * operation) ----
 * Sec. II-C: the layer marks the cells of each new cloud as occupied and
 * clears, as free, the cells inside the sensor's view, on a sparse map of the
 * whole space (OpenVDB on the CPU in the paper; a GPU map is its future work,
 * Sec. IV).  Readings:
 *   - voxels of edge `res` on a grid fixed in the global frame:
 *     k_a = floor(RN32(p_a * RN32(1/res))), -2^20 <= k_a < 2^20 (points outside,
 *     or not finite, are skipped); key = (k_x + 2^20) | (k_y + 2^20) << 21 |
 *     (k_z + 2^20) << 42;
 *   - mark: every voxel holding a point gets the (non-zero) time stamp;
 *   - clear: every occupied voxel whose centre lies in the camera frustum is
 *     freed.  With c_a = RN32(RN32(k_a + 0.5) * res), d_a = RN32(c_a - trans[a])
 *     and q_j = RN32(RN32(RN32(rot[j] d_0) + RN32(rot[3+j] d_1)) + RN32(rot[6+j] d_2))
 *     (the centre in the camera frame), inside iff z_near <= q_2 <= z_far,
 *     -0.5 <= RN32(RN32(fx * RN32(q_0 / q_2)) + cx) <= width - 0.5 and the same
 *     for v with fy, cy, height;
 *   - expire: voxels stamped before min_stamp are freed (temporal decay).
 * Storage: an open-addressing hash table of `capacity` slots (rounded up to a
 * power of two) in device memory; a freed voxel keeps its slot until
 * vg_map_compact.  Keep the used slots under about half the capacity: a mark
 * whose probe runs too long is dropped and reported (vg_map_stats().full,
 * and VG_ERR_WORKSPACE from vg_map_export).  mark, clear, expire and compact
 * are asynchronous on `stream`; export and stats wait for it.  The operations
 * on one map must run in order (one stream, or streams ordered by the caller):
 * each counting operation clears the counter that the next one of its kind
 * uses, and the table itself is shared. */
typedef struct vg_map vg_map;

typedef struct vg_frustum {
  float rot[9];          /* camera-to-global rotation, row-major */
  float trans[3];        /* camera position in the global frame */
  float fx, fy, cx, cy;  /* pinhole intrinsics, pixels */
  int32_t width, height; /* image size, >= 1 */
  float z_near, z_far;   /* depth range along the optical axis, z_near <= z_far */
} vg_frustum;

typedef struct vg_map_info {
  int64_t capacity, occupied, used_slots;
  int64_t last_skipped, last_cleared, last_expired;  /* of the last mark / clear / expire */
  int32_t full;          /* a mark or compaction ran out of probe length */
} vg_map_info;

vg_status vg_map_create(int64_t capacity, float res, vg_map **map);
vg_status vg_map_destroy(vg_map *map);
/* x, y, z: device [n], global frame; stamp >= 1. */
vg_status vg_map_mark(vg_map *map, const float *x, const float *y, const float *z, int64_t n,
                      uint32_t stamp, void *stream);
vg_status vg_map_clear_frustum(vg_map *map, const vg_frustum *f, void *stream);
vg_status vg_map_expire(vg_map *map, uint32_t min_stamp, void *stream);
/* Occupied voxels into device arrays keys, stamps (at most cap written, in no
 * particular order); *n = their number (host). */
vg_status vg_map_export(vg_map *map, uint64_t *keys, uint32_t *stamps, int64_t cap, int64_t *n,
                        void *stream);
/* Rebuilds the table with its occupied voxels only (freed slots reclaimed). */
vg_status vg_map_compact(vg_map *map, void *stream);
vg_status vg_map_stats(vg_map *map, vg_map_info *info, void *stream);

/* ---- a call that allocates nothing ----
 * For callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  The operation of
 * vg_downsample_ex with the default tuning, but every scratch buffer (the
 * sorted key/value table, look-back state, staged call header) lives in one
 * fixed device array of VG_NOALLOC_SCRATCH_BYTES that the library holds on
 * each GPU it runs on until the process ends; the call header goes to the
 * device as kernel arguments, so no host buffer is used either.
 * p, out: as vg_downsample_ex (device, capacity n); 0 <= n <=
 * VG_NOALLOC_MAX_POINTS, else VG_ERR_WORKSPACE before anything is enqueued.
 * d_m: device int64 [1], receives the number of cells (0 unless d_status is
 * VG_OK); d_status: device int32 [1], receives VG_OK, VG_ERR_GRID_OVERFLOW or
 * VG_ERR_DEVICE.  Fully asynchronous on `stream`: nothing is read back.
 * Every call on one GPU shares that GPU's array, and each call clears the
 * state it needs at its start: calls must be ordered (one stream, or
 * synchronised); calls that overlap on one GPU race and give wrong results. */
#define VG_NOALLOC_MAX_POINTS 1048576
#define VG_NOALLOC_SCRATCH_BYTES (64u << 20)
vg_status vg_downsample_noalloc(const vg_points *p, int64_t n, float leaf, vg_key_mode key_mode,
                                vg_cells *out, int64_t *d_m, int32_t *d_status, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* VG_H */

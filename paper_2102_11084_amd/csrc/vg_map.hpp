// A global voxel map on the GPU: the costmap layer's other hot operation
// (Sec. II-C: cells of each new cloud are marked occupied, cells inside the
// sensor's view are cleared as free; the paper names a GPU map as future
// work, Sec. IV).  Voxels of edge `res` on a grid fixed in the global frame,
// key (k_x + 2^20) | (k_y + 2^20) << 21 | (k_z + 2^20) << 42 with
// k_a = floor(RN32(p_a * inv_res)), -2^20 <= k_a < 2^20.
//
// Storage: one open-addressing hash table of 64-bit keys (empty = all ones)
// with a 32-bit time stamp per slot; stamp 0 is a free voxel (cleared or
// expired), whose slot keeps its key until the map is compacted.  Slots are
// found by linear probing from a SplitMix64-finalizer hash (Steele, Lea and
// Flood, OOPSLA 2014) of the key; a key is inserted by a compare-and-swap on
// an empty slot, never on a free one, so a key has at most one slot.
//   mark     per point: its voxel's slot gets the stamp (inserted if new)
//   clear    per slot: a voxel whose centre projects inside the camera
//            frustum is freed
//   expire   per slot: a voxel stamped before a given stamp is freed
//   export   per slot: occupied voxels appended to the caller's arrays
//   compact  occupied voxels re-inserted into an emptied table
#pragma once

#include "vg_pipeline.hpp"

namespace vg {

constexpr uint64_t kMapEmpty = ~0ull;
constexpr int32_t kMapHalfRange = 1 << 20;
constexpr uint32_t kMapMaxProbe = 4096;  // longer probes report the table as full
constexpr int kMapBlock = 256;

// Counters of an operation come in pairs: the k-th operation of a kind counts
// into slot k & 1 and clears slot (k + 1) & 1 for the next one (operations on
// a map run in stream order), so no launch is spent clearing counters.
struct MapCtl {
  uint32_t error;       // non-zero: a probe ran past kMapMaxProbe (table too full)
  uint32_t skipped[2];  // points of a mark outside the key range or not finite
  uint32_t cleared[2];  // voxels freed by a clear
  uint32_t expired[2];  // voxels freed by an expire
  uint32_t live[2];     // voxels appended by an export / compact
  uint32_t count[2];    // occupied voxels, used slots (stats)
  uint32_t pad[5];
};

// The counter pair of an operation: this one's slot, and the next one's
// cleared by the first thread of the launch.
__device__ __forceinline__ uint32_t* map_slot(uint32_t* pair, uint32_t slot) {
  if (blockIdx.x == 0 && threadIdx.x == 0) pair[slot ^ 1u] = 0u;
  return pair + slot;
}

struct MapWs {
  uint64_t* keys;      // [cap]
  uint32_t* stamps;    // [cap]
  uint64_t* tkeys;     // [cap] compaction scratch
  uint32_t* tstamps;   // [cap]
  MapCtl* ctl;
  uint64_t mask;       // cap - 1 (cap a power of two)
  float res, inv;
};

struct MapFrustum {
  float r[9];          // camera -> global rotation, row-major
  float t[3];          // camera position
  float fx, fy, cx, cy;
  int32_t width, height;
  float z_near, z_far;
};

__device__ __forceinline__ uint64_t map_hash(uint64_t z) {
  z ^= z >> 30;
  z *= 0xbf58476d1ce4e5b9ull;
  z ^= z >> 27;
  z *= 0x94d049bb133111ebull;
  z ^= z >> 31;
  return z;
}

__device__ __forceinline__ bool map_key(const MapWs& m, float x, float y, float z, uint64_t* key) {
  if (!finite3(x, y, z)) return false;
  const float p[3] = {x, y, z};
  uint64_t k = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float f = floorf(__fmul_rn(p[a], m.inv));
    if (!(f >= -(float)kMapHalfRange && f < (float)kMapHalfRange)) return false;
    k |= (uint64_t)((int64_t)f + kMapHalfRange) << (21 * a);
  }
  *key = k;
  return true;
}

// Wave-aggregated add of a per-lane flag to a counter.
__device__ __forceinline__ void map_count(uint32_t* ctr, bool flag) {
  const uint64_t b = __ballot(flag);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(ctr, (uint32_t)__popcll(b));
}

// Slot of `key`, inserting it into an empty slot if absent; -1 when the probe
// runs too long.
__device__ __forceinline__ int64_t map_find_or_insert(const MapWs& m, uint64_t key) {
  uint64_t h = map_hash(key) & m.mask;
  for (uint32_t step = 0; step < kMapMaxProbe; ++step, h = (h + 1) & m.mask) {
    const uint64_t s = __hip_atomic_load(&m.keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (s == key) return (int64_t)h;
    if (s == kMapEmpty) {
      const uint64_t old = atomicCAS((unsigned long long*)&m.keys[h], (unsigned long long)kMapEmpty,
                                     (unsigned long long)key);
      if (old == kMapEmpty || old == key) return (int64_t)h;
    }
  }
  return -1;
}

__global__ __launch_bounds__(kMapBlock) void vg_map_mark_kernel(MapWs m, const float* x,
                                                                 const float* y, const float* z,
                                                                 int64_t n, uint32_t stamp,
                                                                 uint32_t slot) {
  uint32_t* skipped = map_slot(m.ctl->skipped, slot);
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n; i0 += nth) {
    const int64_t i = i0 + threadIdx.x;
    bool skip = false;
    if (i < n) {
      uint64_t key;
      if (map_key(m, x[i], y[i], z[i], &key)) {
        const int64_t h = map_find_or_insert(m, key);
        if (h >= 0) m.stamps[h] = stamp;  // every writer of a slot writes the same stamp
        else atomicOr(&m.ctl->error, 1u);
      } else {
        skip = true;
      }
    }
    map_count(skipped, skip);
  }
}

// Centre of a voxel in the camera frame, and whether it lies in the frustum:
// c_a = RN32(RN32(k_a + 0.5) * res), d_a = RN32(c_a - t_a),
// q_j = RN32(RN32(RN32(r[0][j] d_0) + RN32(r[1][j] d_1)) + RN32(r[2][j] d_2)),
// z_near <= q_2 <= z_far, u = RN32(RN32(fx * RN32(q_0 / q_2)) + cx) in
// [-0.5, width - 0.5], v likewise with fy, cy, height.
__device__ __forceinline__ bool map_in_frustum(const MapWs& m, const MapFrustum& f, uint64_t key) {
  float d[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int64_t k = (int64_t)((key >> (21 * a)) & ((1ull << 21) - 1ull)) - kMapHalfRange;
    const float c = __fmul_rn(__fadd_rn((float)k, 0.5f), m.res);
    d[a] = __fsub_rn(c, f.t[a]);
  }
  float q[3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
    q[j] = __fadd_rn(__fadd_rn(__fmul_rn(f.r[j], d[0]), __fmul_rn(f.r[3 + j], d[1])),
                     __fmul_rn(f.r[6 + j], d[2]));
  if (!(q[2] >= f.z_near && q[2] <= f.z_far)) return false;
  const float u = __fadd_rn(__fmul_rn(f.fx, __fdiv_rn(q[0], q[2])), f.cx);
  const float v = __fadd_rn(__fmul_rn(f.fy, __fdiv_rn(q[1], q[2])), f.cy);
  return u >= -0.5f && u <= __fsub_rn((float)f.width, 0.5f) && v >= -0.5f &&
         v <= __fsub_rn((float)f.height, 0.5f);
}

__global__ __launch_bounds__(kMapBlock) void vg_map_clear_kernel(MapWs m, MapFrustum f,
                                                                  uint32_t slot) {
  uint32_t* cleared = map_slot(m.ctl->cleared, slot);
  const uint64_t cap = m.mask + 1;
  const uint64_t nth = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t h0 = (uint64_t)blockIdx.x * blockDim.x; h0 < cap; h0 += nth) {
    const uint64_t h = h0 + threadIdx.x;
    bool hit = false;
    if (h < cap && m.stamps[h] != 0u) {
      const uint64_t key = m.keys[h];
      if (key != kMapEmpty && map_in_frustum(m, f, key)) {
        m.stamps[h] = 0u;
        hit = true;
      }
    }
    map_count(cleared, hit);
  }
}

__global__ __launch_bounds__(kMapBlock) void vg_map_expire_kernel(MapWs m, uint32_t min_stamp,
                                                                   uint32_t slot) {
  uint32_t* expired = map_slot(m.ctl->expired, slot);
  const uint64_t cap = m.mask + 1;
  const uint64_t nth = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t h0 = (uint64_t)blockIdx.x * blockDim.x; h0 < cap; h0 += nth) {
    const uint64_t h = h0 + threadIdx.x;
    bool hit = false;
    if (h < cap) {
      const uint32_t s = m.stamps[h];
      if (s != 0u && s < min_stamp) {
        m.stamps[h] = 0u;
        hit = true;
      }
    }
    map_count(expired, hit);
  }
}

// Occupied voxels appended to (okeys, ostamps) (at most cap_out written; the
// count goes to ctl->live[slot]).  Appends are gathered per workgroup.
__global__ __launch_bounds__(kMapBlock) void vg_map_export_kernel(MapWs m, uint64_t* okeys,
                                                                   uint32_t* ostamps,
                                                                   uint64_t cap_out,
                                                                   uint32_t slot) {
  __shared__ uint32_t ws[kMapBlock / 64];
  __shared__ uint32_t base_s;
  uint32_t* live_ctr = map_slot(m.ctl->live, slot);
  const uint64_t cap = m.mask + 1;
  const uint64_t nth = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t h0 = (uint64_t)blockIdx.x * blockDim.x; h0 < cap; h0 += nth) {
    const uint64_t h = h0 + threadIdx.x;
    uint32_t s = 0u;
    uint64_t key = kMapEmpty;
    if (h < cap) {
      s = m.stamps[h];
      key = m.keys[h];
    }
    const bool live = s != 0u && key != kMapEmpty;
    uint32_t tot;
    const uint32_t off = block_excl_scan<kMapBlock>(live ? 1u : 0u, ws, tot);
    if (tot == 0) continue;
    if (threadIdx.x == 0) base_s = atomicAdd(live_ctr, tot);
    __syncthreads();
    const uint64_t at = (uint64_t)base_s + off;
    if (live && at < cap_out) {
      okeys[at] = key;
      ostamps[at] = s;
    }
    __syncthreads();  // base_s is reused
  }
}

// The stats counters are zeroed by their own launch before the count (a reset
// inside it could land after other workgroups counted).
__global__ void vg_map_zero2_kernel(uint32_t* p) {
  if (threadIdx.x < 2) p[threadIdx.x] = 0u;
}

// Occupied voxels and used slots (stats).
__global__ __launch_bounds__(kMapBlock) void vg_map_count_kernel(MapWs m, uint32_t* out2) {
  const uint64_t cap = m.mask + 1;
  const uint64_t nth = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t h0 = (uint64_t)blockIdx.x * blockDim.x; h0 < cap; h0 += nth) {
    const uint64_t h = h0 + threadIdx.x;
    bool used = false, live = false;
    if (h < cap) {
      used = m.keys[h] != kMapEmpty;
      live = used && m.stamps[h] != 0u;
    }
    map_count(&out2[0], live);
    map_count(&out2[1], used);
  }
}

__global__ __launch_bounds__(kMapBlock) void vg_map_reset_kernel(MapWs m) {
  const uint64_t cap = m.mask + 1;
  const uint64_t nth = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; h < cap; h += nth) {
    m.keys[h] = kMapEmpty;
    m.stamps[h] = 0u;
  }
}

// Re-inserts the exported voxels (tkeys, tstamps; ctl->live[slot] of them).
__global__ __launch_bounds__(kMapBlock) void vg_map_reinsert_kernel(MapWs m, uint32_t slot) {
  const uint64_t n = m.ctl->live[slot];
  const uint64_t nth = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nth) {
    const int64_t h = map_find_or_insert(m, m.tkeys[i]);
    if (h >= 0) m.stamps[h] = m.tstamps[i];
    else atomicOr(&m.ctl->error, 1u);
  }
}

}  // namespace vg

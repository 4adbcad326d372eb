// Device side of the voxel-grid pipeline for gfx950 (wave64).
//
// One call runs these phases over tiles of every frame (arXiv 2102.11084,
// Sec. II-C and Alg. 1):
//   BBOX   per-frame bounding box of the valid points, valid count
//   HIST   per-frame digit histograms of every radix pass (cell keys are
//          recomputed from xyz: the per-point subdivision lookup)
//   SORT p stable LSD radix pass p of (key, index) pairs: ballot-based
//          ranking in a wave, tile staging in LDS, decoupled look-back for the
//          tile's global offsets; pass 0 computes keys from xyz and drops
//          invalid points while keeping input order (the sorted subdivision
//          table)
//   RED    head flags over the sorted keys, global look-back of head counts
//          (dense output rows over all frames), compensated FP32 segmented
//          reduction of (p - cell corner) and integer colour sums, output of
//          one row per occupied cell (the final deletion/compaction step)
// Every tile is a work-queue item; queue order is phase-major, and a tile
// only ever waits for tiles that were dequeued before it, so the pipeline
// cannot deadlock however many workgroups are resident.
#pragma once

#include "vg_common.hpp"

namespace vg {

constexpr uint32_t kSpinLimit = 1u << 21;

// ------------------------------------------------------------- helpers ----
__device__ __forceinline__ uint32_t f2ord(float v) {
  uint32_t b = __float_as_uint(v);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
  uint32_t b = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
  return __uint_as_float(b);
}
__device__ __forceinline__ bool finite3(float x, float y, float z) {
  const uint32_t e = 0x7f800000u;
  return ((__float_as_uint(x) & e) != e) && ((__float_as_uint(y) & e) != e) &&
         ((__float_as_uint(z) & e) != e);
}
__device__ __forceinline__ uint32_t ld_rlx(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_rlx64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fence_acq() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void fence_rel() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

// Spin (one thread) until *p >= target; on time-out flag an error and give up.
__device__ __noinline__ bool wait_geq(const uint32_t* p, uint32_t target, Ctl* ctl) {
  uint32_t spins = 0;
  while (ld_rlx(p) < target) {
    if (++spins > kSpinLimit || ld_rlx(&ctl->error) != 0) {
      atomicOr(&ctl->error, 1u);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return true;
}

// Count of set bits of `mask` in lanes below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Exclusive block scan of one u32 per thread; `wsum` holds NW words of LDS.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* wsum, uint32_t& total) {
  constexpr int NW = BLOCK / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    uint32_t s = wsum[i];
    before += (i < w) ? s : 0u;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return before + incl - v;
}

// ------------------------------------------------------- frame params ----
struct FrameParams {
  int64_t off, n;
  float mn[3];
  float inv, leaf;
  uint32_t d[3];
  uint32_t n_valid;
  int bits, passes, w;
  bool wide;
  int status;
};

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__device__ __forceinline__ uint32_t cell_coord(float p, float mn, float inv) {
  float diff = __fsub_rn(p, mn);
  float t = __fmul_rn(diff, inv);
  return (uint32_t)floorf(t);
}

// Grid of frame b from its (complete) bounding box.  Identical in every tile.
__device__ FrameParams frame_params(const Ws& ws, int b, int key_mode, int radix_bits) {
  FrameParams f;
  const FrameDesc fd = ws.fd[b];
  const FrameState& s = ws.fs[b];
  f.off = fd.off;
  f.n = fd.n;
  f.inv = fd.inv;
  f.leaf = fd.leaf;
  f.n_valid = s.n_valid;
  f.status = kFrameOk;
  f.bits = 0;
  f.passes = 0;
  f.w = 0;
  f.wide = false;
  for (int a = 0; a < 3; ++a) { f.mn[a] = 0.f; f.d[a] = 0; }
  if (f.n_valid == 0) return f;
  for (int a = 0; a < 3; ++a) {
    float mn = ord2f(~s.mn_neg[a]);
    float mx = ord2f(s.mx[a]);
    f.mn[a] = mn;
    float t = __fmul_rn(__fsub_rn(mx, mn), f.inv);
    if (!(t < kMaxCellsPerAxis)) {
      f.status = kFrameOverflow;
      return f;
    }
    f.d[a] = (uint32_t)floorf(t) + 1u;
  }
  uint64_t top;
  if (key_mode == 1) {
    top = spread3(f.d[0] - 1) | (spread3(f.d[1] - 1) << 1) | (spread3(f.d[2] - 1) << 2);
  } else {
    top = (uint64_t)f.d[0] * (uint64_t)f.d[1] * (uint64_t)f.d[2] - 1ull;
  }
  f.bits = top ? 64 - __clzll(top) : 0;
  f.wide = f.bits > 32;
  f.passes = f.bits == 0 ? 1 : (f.bits + radix_bits - 1) / radix_bits;
  f.w = (f.bits + f.passes - 1) / f.passes;
  return f;
}

__device__ __forceinline__ uint64_t point_key(const FrameParams& f, int key_mode, uint32_t kx,
                                              uint32_t ky, uint32_t kz) {
  if (key_mode == 1) return spread3(kx) | (spread3(ky) << 1) | (spread3(kz) << 2);
  if (!f.wide) return (uint64_t)(kx + f.d[0] * (ky + f.d[1] * kz));
  return (uint64_t)kx + (uint64_t)f.d[0] * ((uint64_t)ky + (uint64_t)f.d[1] * (uint64_t)kz);
}

// ------------------------------------------------- compensated sums ----
// Sum of binary32 values kept as an unevaluated pair (s, c); each addition
// uses the error-free TwoSum transformation (Knuth; Neumaier-style carry).
struct Acc {
  uint32_t n;
  float s[3], c[3];
  uint32_t rgb[3];
};

__device__ __forceinline__ void two_sum_into(float& s, float& c, float v) {
  float t = __fadd_rn(s, v);
  float bp = __fsub_rn(t, s);
  float e = __fadd_rn(__fsub_rn(s, __fsub_rn(t, bp)), __fsub_rn(v, bp));
  s = t;
  c = __fadd_rn(c, e);
}

__device__ __forceinline__ void acc_zero(Acc& a) {
  a.n = 0;
  for (int i = 0; i < 3; ++i) { a.s[i] = 0.f; a.c[i] = 0.f; a.rgb[i] = 0u; }
}

__device__ __forceinline__ void acc_add(Acc& a, const float d[3], const uint32_t rgb[3]) {
  a.n += 1;
  for (int i = 0; i < 3; ++i) {
    two_sum_into(a.s[i], a.c[i], d[i]);
    a.rgb[i] += rgb[i];
  }
}

// a <- a (+) b, a on the left.
__device__ __forceinline__ void acc_merge(Acc& a, const Acc& b) {
  a.n += b.n;
  for (int i = 0; i < 3; ++i) {
    two_sum_into(a.s[i], a.c[i], b.s[i]);
    a.c[i] = __fadd_rn(a.c[i], b.c[i]);
    a.rgb[i] += b.rgb[i];
  }
}

// Segmented-scan element: f = a head lies in the covered range, hp = frame
// position of the last such head, a = sums since that head (or since the start).
struct Seg {
  uint32_t f, hp;
  Acc a;
};

__device__ __forceinline__ Seg seg_combine(const Seg& x, const Seg& y) {
  if (y.f) return y;
  Seg r = x;
  acc_merge(r.a, y.a);
  return r;
}

__device__ __forceinline__ Seg seg_shfl_up(const Seg& v, int off) {
  Seg r;
  r.f = __shfl_up(v.f, off);
  r.hp = __shfl_up(v.hp, off);
  r.a.n = __shfl_up(v.a.n, off);
  for (int i = 0; i < 3; ++i) {
    r.a.s[i] = __shfl_up(v.a.s[i], off);
    r.a.c[i] = __shfl_up(v.a.c[i], off);
    r.a.rgb[i] = __shfl_up(v.a.rgb[i], off);
  }
  return r;
}

// ---------------------------------------------------------- configs ----
template <int BLOCK_, int SORT_ITEMS_, int RADIX_, int RED_ITEMS_>
struct Cfg {
  static constexpr int BLOCK = BLOCK_;
  static constexpr int NW = BLOCK / 64;
  static constexpr int SI = SORT_ITEMS_;
  static constexpr int TS = BLOCK * SI;
  static constexpr int W = RADIX_;
  static constexpr int R = 1 << W;
  static constexpr int MAXP = (63 + W - 1) / W;
  static constexpr int RI = RED_ITEMS_;
  static constexpr int TR = BLOCK * RI;
  static constexpr int PH_BBOX = 0, PH_HIST = 1, PH_SORT0 = 2, PH_RED = 2 + MAXP, NPH = 3 + MAXP;
  static_assert(R <= BLOCK, "one digit per thread in the look-back");
  static_assert(MAXP <= kMaxPassSlots, "pass slots");
  static_assert(SI <= 32 && RI <= 32, "item masks are 32-bit");

  struct SortSmem {
    uint32_t lo[TS];
    uint32_t hi[TS];
    uint32_t idx[TS];
    uint32_t wcnt[NW][R];
    uint32_t tstart[R];
    uint32_t gbase[R];
    uint32_t dstart[R];
    uint32_t wsum[NW];
  };
  struct HistSmem {
    uint32_t h[MAXP][R];
    uint32_t wsum[NW];
  };
  struct BboxSmem {
    uint32_t mn[NW][3];
    uint32_t mx[NW][3];
    uint32_t nv[NW];
  };
  struct RedSmem {
    uint32_t wsum[NW];
    Seg wtot[NW];
    Acc part[BLOCK];
    Acc span_acc;
    float span_r[3];
    uint32_t span_lo, span_hi;
    uint32_t span_pending;
    uint32_t span_start;
    uint64_t excl;
  };
  union Smem {
    SortSmem sort;
    HistSmem hist;
    BboxSmem bbox;
    RedSmem red;
  };
};

// ---------------------------------------------------------- BBOX tile ----
template <class C>
__device__ void bbox_tile(const Ws& ws, const Io& io, typename C::Smem& sm, int b, int j,
                          uint32_t want) {
  const FrameDesc fd = ws.fd[b];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t t0 = (int64_t)j * C::TS;
  uint32_t mn[3] = {0u, 0u, 0u}, mx[3] = {0u, 0u, 0u}, nv = 0;
#pragma unroll 4
  for (int it = 0; it < C::SI; ++it) {
    int64_t pos = t0 + (int64_t)w * 64 * C::SI + it * 64 + lane;
    if (pos < fd.n) {
      int64_t g = fd.off + pos;
      float x = io.x[g], y = io.y[g], z = io.z[g];
      if (finite3(x, y, z)) {
        uint32_t ex = f2ord(x), ey = f2ord(y), ez = f2ord(z);
        mn[0] = max(mn[0], ~ex); mn[1] = max(mn[1], ~ey); mn[2] = max(mn[2], ~ez);
        mx[0] = max(mx[0], ex); mx[1] = max(mx[1], ey); mx[2] = max(mx[2], ez);
        nv += 1;
      } else if (want & kOutPointCell) {
        io.point_cell[g] = -1;
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    for (int a = 0; a < 3; ++a) {
      mn[a] = max(mn[a], (uint32_t)__shfl_xor(mn[a], off));
      mx[a] = max(mx[a], (uint32_t)__shfl_xor(mx[a], off));
    }
    nv += __shfl_xor(nv, off);
  }
  if (lane == 0) {
    for (int a = 0; a < 3; ++a) { sm.bbox.mn[w][a] = mn[a]; sm.bbox.mx[w][a] = mx[a]; }
    sm.bbox.nv[w] = nv;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tn = 0;
    for (int i = 0; i < C::NW; ++i) {
      tn += sm.bbox.nv[i];
      for (int a = 0; a < 3; ++a) {
        mn[a] = max(mn[a], sm.bbox.mn[i][a]);
        mx[a] = max(mx[a], sm.bbox.mx[i][a]);
      }
    }
    FrameState* fs = ws.fs + b;
    if (tn) {
      for (int a = 0; a < 3; ++a) {
        atomicMax(&fs->mn_neg[a], mn[a]);
        atomicMax(&fs->mx[a], mx[a]);
      }
      atomicAdd(&fs->n_valid, tn);
    }
    fence_rel();
    atomicAdd(&fs->bbox_done, 1u);
  }
}

// Load pass-0 items of a tile: keys from xyz, invalid points masked out.
template <class C>
__device__ __forceinline__ uint32_t load_points_keys(const Io& io, const FrameParams& f,
                                                     int key_mode, int64_t t0, uint32_t* klo,
                                                     uint32_t* khi, uint32_t* kid) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t vmask = 0;
#pragma unroll
  for (int it = 0; it < C::SI; ++it) {
    int64_t pos = t0 + (int64_t)w * 64 * C::SI + it * 64 + lane;
    klo[it] = 0u;
    khi[it] = 0u;
    kid[it] = 0u;
    if (pos < f.n) {
      int64_t g = f.off + pos;
      float x = io.x[g], y = io.y[g], z = io.z[g];
      if (finite3(x, y, z)) {
        uint64_t k = point_key(f, key_mode, cell_coord(x, f.mn[0], f.inv),
                               cell_coord(y, f.mn[1], f.inv), cell_coord(z, f.mn[2], f.inv));
        klo[it] = (uint32_t)k;
        khi[it] = (uint32_t)(k >> 32);
        kid[it] = (uint32_t)g;
        vmask |= 1u << it;
      }
    }
  }
  return vmask;
}

__device__ __forceinline__ uint32_t digit_of(uint32_t lo, uint32_t hi, int shift, uint32_t mask) {
  uint64_t k = ((uint64_t)hi << 32) | lo;
  return (uint32_t)(k >> shift) & mask;
}

// ---------------------------------------------------------- HIST tile ----
template <class C>
__device__ void hist_tile(const Ws& ws, const Io& io, typename C::Smem& sm, int b, int j, int t,
                          const FrameParams& f, int key_mode, uint32_t want) {
  const int P = f.passes;
  const int Rb = 1 << f.w;
  const uint32_t mask = (uint32_t)Rb - 1u;
  if (f.status == kFrameOverflow) {
    if (want & kOutPointCell) {
      const int64_t t0 = (int64_t)j * C::TS;
      for (int i = threadIdx.x; i < C::TS; i += C::BLOCK) {
        int64_t pos = t0 + i;
        if (pos < f.n) io.point_cell[f.off + pos] = -1;
      }
    }
  } else if (P > 0) {
    // this tile's look-back descriptors of every pass start cleared
    for (int p = 0; p < P; ++p) {
      uint32_t* row = ws.sdesc + ((size_t)p * ws.capNTs + t) * C::R;
      for (int d = threadIdx.x; d < C::R; d += C::BLOCK) row[d] = 0u;
    }
    for (int i = threadIdx.x; i < C::MAXP * C::R; i += C::BLOCK) (&sm.hist.h[0][0])[i] = 0u;
    __syncthreads();
    uint32_t klo[C::SI], khi[C::SI], kid[C::SI];
    uint32_t vm = load_points_keys<C>(io, f, key_mode, (int64_t)j * C::TS, klo, khi, kid);
#pragma unroll
    for (int it = 0; it < C::SI; ++it) {
      if (vm & (1u << it)) {
        for (int p = 0; p < P; ++p)
          atomicAdd(&sm.hist.h[p][digit_of(klo[it], khi[it], p * f.w, mask)], 1u);
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < P * C::R; i += C::BLOCK) {
      int p = i / C::R, d = i % C::R;
      uint32_t v = sm.hist.h[p][d];
      if (v) atomicAdd(&ws.hist[((size_t)b * ws.slots + p) * C::R + d], v);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    fence_rel();
    atomicAdd(&ws.fs[b].hist_done, 1u);
  }
}

// ---------------------------------------------------------- SORT tile ----
template <class C>
__device__ void sort_tile(const Ws& ws, const Io& io, typename C::Smem& sm, int b, int j, int t,
                          int p, const FrameParams& f, int key_mode) {
  auto& S = sm.sort;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int Rb = 1 << f.w;
  const uint32_t mask = (uint32_t)Rb - 1u;
  const int shift = p * f.w;
  const int64_t t0 = (int64_t)j * C::TS;

  // frame-wide digit offsets of this pass
  {
    uint32_t hv = 0;
    if ((int)threadIdx.x < Rb) hv = ws.hist[((size_t)b * ws.slots + p) * C::R + threadIdx.x];
    uint32_t tot;
    uint32_t ex = block_excl_scan<C::BLOCK>(hv, S.wsum, tot);
    if ((int)threadIdx.x < C::R) S.dstart[threadIdx.x] = ex;
  }
  for (int i = threadIdx.x; i < C::NW * C::R; i += C::BLOCK) (&S.wcnt[0][0])[i] = 0u;

  uint32_t klo[C::SI], khi[C::SI], kid[C::SI];
  uint32_t vm;
  if (p == 0) {
    vm = load_points_keys<C>(io, f, key_mode, t0, klo, khi, kid);
  } else {
    const int src = p & 1;
    const uint32_t* slo = ws.lo[src] + f.off;
    const uint32_t* shi = ws.hi[src] + f.off;
    const uint32_t* sid = ws.idx[src] + f.off;
    vm = 0;
#pragma unroll
    for (int it = 0; it < C::SI; ++it) {
      int64_t pos = t0 + (int64_t)w * 64 * C::SI + it * 64 + lane;
      klo[it] = 0u;
      khi[it] = 0u;
      kid[it] = 0u;
      if (pos < (int64_t)f.n_valid) {
        klo[it] = slo[pos];
        if (f.wide) khi[it] = shi[pos];
        kid[it] = sid[pos];
        vm |= 1u << it;
      }
    }
  }
  __syncthreads();

  // rank every item among equal digits of its wave, in input order
  uint32_t rank[C::SI], dg[C::SI];
#pragma unroll
  for (int it = 0; it < C::SI; ++it) {
    const bool valid = (vm >> it) & 1u;
    const uint32_t d = digit_of(klo[it], khi[it], shift, mask);
    dg[it] = d;
    uint64_t match = __ballot(valid);
    for (int bit = 0; bit < f.w; ++bit) {
      const bool set = (d >> bit) & 1u;
      const uint64_t bal = __ballot(set);
      match &= set ? bal : ~bal;
    }
    const uint32_t below = lanes_below(match);
    const uint32_t cnt = (uint32_t)__popcll(match);
    uint32_t pre = 0;
    if (valid) pre = S.wcnt[w][d];
    if (valid && below == 0) S.wcnt[w][d] = pre + cnt;
    rank[it] = pre + below;
  }
  __syncthreads();

  // per digit: offsets of the waves, tile count
  uint32_t tcnt = 0;
  if ((int)threadIdx.x < Rb) {
    const int d = threadIdx.x;
    for (int i = 0; i < C::NW; ++i) {
      uint32_t v = S.wcnt[i][d];
      S.wcnt[i][d] = tcnt;
      tcnt += v;
    }
  }
  uint32_t tile_total;
  const uint32_t tex = block_excl_scan<C::BLOCK>(tcnt, S.wsum, tile_total);
  if ((int)threadIdx.x < C::R) S.tstart[threadIdx.x] = tex;

  // decoupled look-back over the frame's earlier tiles of this pass
  if ((int)threadIdx.x < Rb) {
    const int d = threadIdx.x;
    uint32_t* mine = ws.sdesc + ((size_t)p * ws.capNTs + t) * C::R + d;
    uint32_t excl = 0;
    if (j == 0) {
      st_rlx(mine, kFlagP32 | tcnt);
    } else {
      st_rlx(mine, kFlagA32 | tcnt);
      int k = t - 1;
      uint32_t spins = 0;
      for (;;) {
        uint32_t v = ld_rlx(ws.sdesc + ((size_t)p * ws.capNTs + k) * C::R + d);
        uint32_t fl = v & 0xc0000000u;
        if (fl == 0u) {
          if (++spins > kSpinLimit || ((spins & 255u) == 0u && ld_rlx(&ws.ctl->error))) {
            atomicOr(&ws.ctl->error, 1u);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += v & kVal32;
        if (fl == kFlagP32) break;
        if (--k < t - j) {  // the frame's first tile always holds a prefix
          atomicOr(&ws.ctl->error, 1u);
          break;
        }
      }
      st_rlx(mine, kFlagP32 | ((excl + tcnt) & kVal32));
    }
    S.gbase[d] = S.dstart[d] + excl;
  }
  __syncthreads();

  // stage the tile in LDS in digit order
#pragma unroll
  for (int it = 0; it < C::SI; ++it) {
    if ((vm >> it) & 1u) {
      const uint32_t d = dg[it];
      const uint32_t lp = S.tstart[d] + S.wcnt[w][d] + rank[it];
      S.lo[lp] = klo[it];
      S.hi[lp] = khi[it];
      S.idx[lp] = kid[it];
    }
  }
  __syncthreads();

  // write runs of equal digits to their global places
  const int dst = (p + 1) & 1;
  uint32_t* dlo = ws.lo[dst] + f.off;
  uint32_t* dhi = ws.hi[dst] + f.off;
  uint32_t* did = ws.idx[dst] + f.off;
  for (uint32_t i = threadIdx.x; i < tile_total; i += C::BLOCK) {
    const uint32_t lo = S.lo[i], hi = S.hi[i];
    const uint32_t d = digit_of(lo, hi, shift, mask);
    const uint32_t gp = S.gbase[d] + (i - S.tstart[d]);
    if (gp < (uint32_t)f.n) {
      dlo[gp] = lo;
      if (f.wide) dhi[gp] = hi;
      did[gp] = S.idx[i];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    fence_rel();
    atomicAdd(&ws.fs[b].pass_done[p], 1u);
  }
}

// ------------------------------------------------------------ RED tile ----
struct CellOut {
  uint32_t lo, hi, ref;
  float r[3];
};

// Writes one output row from a segment's sums.
__device__ __forceinline__ void finalize_row(const Io& io, uint32_t want, int64_t row, int64_t N,
                                             const Acc& a, uint64_t rgb_wide[3], const CellOut& c) {
  if (row < 0 || row >= N || a.n == 0 || c.ref >= N) return;
  const float fn = (float)a.n;
  float mean[3];
  for (int i = 0; i < 3; ++i) mean[i] = __fdiv_rn(__fadd_rn(a.s[i], a.c[i]), fn);
  if (want & kOutXYZ) {
    io.cx[row] = __fadd_rn(c.r[0], mean[0]);
    io.cy[row] = __fadd_rn(c.r[1], mean[1]);
    io.cz[row] = __fadd_rn(c.r[2], mean[2]);
  }
  if (want & kOutLocal) {
    const float px = io.x[c.ref], py = io.y[c.ref], pz = io.z[c.ref];
    io.lx[row] = __fadd_rn(__fsub_rn(c.r[0], px), mean[0]);
    io.ly[row] = __fadd_rn(__fsub_rn(c.r[1], py), mean[1]);
    io.lz[row] = __fadd_rn(__fsub_rn(c.r[2], pz), mean[2]);
  }
  if (want & kOutRGB) {
    for (int i = 0; i < 3; ++i) {
      uint64_t s = rgb_wide ? rgb_wide[i] : (uint64_t)a.rgb[i];
      io.crgb[3 * row + i] = (uint8_t)((s + a.n / 2) / a.n);
    }
  }
  if (want & kOutCount) io.count[row] = a.n;
  if (want & kOutKey) io.key[row] = ((uint64_t)c.hi << 32) | c.lo;
  if (want & kOutRef) io.ref_index[row] = c.ref;
}

template <class C>
__device__ void red_tile(const Ws& ws, const Io& io, typename C::Smem& sm, int b, int j, int t,
                         const FrameParams& f, uint32_t want, int B, int NTr, int64_t N) {
  auto& S = sm.red;
  constexpr int K = C::RI;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t nv = (f.status == kFrameOk) ? (int64_t)f.n_valid : 0;
  const int64_t s0 = (int64_t)j * C::TR;
  const int64_t e0 = min(s0 + (int64_t)C::TR, nv);
  const int cnt = e0 > s0 ? (int)(e0 - s0) : 0;
  const int fb = f.passes & 1;
  const uint32_t* klo = ws.lo[fb] + f.off;
  const uint32_t* khi = ws.hi[fb] + f.off;
  const uint32_t* kid = ws.idx[fb] + f.off;
  const int base = threadIdx.x * K;

  // ---- keys and head flags (blocked: thread i owns items i*K .. i*K+K-1)
  uint32_t lo_[K], hi_[K], id_[K];
  uint32_t vmask = 0, hmask = 0;
  {
    uint32_t plo = 0, phi = 0;
    bool have_prev = false;
    if (base < cnt && s0 + base > 0) {
      plo = klo[s0 + base - 1];
      phi = f.wide ? khi[s0 + base - 1] : 0u;
      have_prev = true;
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
      lo_[i] = 0u;
      hi_[i] = 0u;
      id_[i] = 0u;
      if (base + i < cnt) {
        const int64_t pos = s0 + base + i;
        lo_[i] = klo[pos];
        hi_[i] = f.wide ? khi[pos] : 0u;
        id_[i] = kid[pos];
        if (id_[i] >= (uint64_t)N) id_[i] = 0;  // never for a consistent sort
        vmask |= 1u << i;
        const bool head = !have_prev || lo_[i] != plo || hi_[i] != phi;
        if (head) hmask |= 1u << i;
        plo = lo_[i];
        phi = hi_[i];
        have_prev = true;
      }
    }
  }
  uint32_t H;
  const uint32_t hb = block_excl_scan<C::BLOCK>((uint32_t)__popc(hmask), S.wsum, H);

  // ---- global look-back over head counts: dense rows across frames
  if (threadIdx.x == 0) {
    uint64_t excl = 0;
    if (t == 0) {
      st_rlx64(&ws.rdesc[0], kFlagP64 | H);
    } else {
      st_rlx64(&ws.rdesc[t], kFlagA64 | H);
      int k = t - 1;
      uint32_t spins = 0;
      for (;;) {
        uint64_t v = ld_rlx64(&ws.rdesc[k]);
        uint64_t fl = v & (3ull << 62);
        if (fl == 0) {
          if (++spins > kSpinLimit || ((spins & 255u) == 0u && ld_rlx(&ws.ctl->error))) {
            atomicOr(&ws.ctl->error, 1u);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += v & kVal64;
        if (fl == kFlagP64) break;
        if (--k < 0) {
          atomicOr(&ws.ctl->error, 1u);
          break;
        }
      }
      st_rlx64(&ws.rdesc[t], kFlagP64 | (excl + H));
    }
    S.excl = excl;
    S.span_pending = 0;
    if (j == 0) {
      io.out_offsets[b] = (int64_t)excl;
      io.frame_status[b] = ld_rlx(&ws.ctl->error) ? 5 : f.status;
    }
    if (t == NTr - 1) io.out_offsets[B] = (int64_t)(excl + H);
  }
  __syncthreads();
  const int64_t excl_t = (int64_t)S.excl;

  // ---- gather points, per-item values, thread-sequential segmented sums
  Acc pre, cur;
  acc_zero(pre);
  acc_zero(cur);
  bool seen_head = false;
  uint32_t cur_hp = 0, lh = 0;
  CellOut cur_c, pre_c;
  cur_c.lo = cur_c.hi = cur_c.ref = 0;
  pre_c = cur_c;
  for (int i = 0; i < 3; ++i) cur_c.r[i] = pre_c.r[i] = 0.f;
  for (int i = 0; i < K; ++i) {
    if (!((vmask >> i) & 1u)) continue;
    const uint32_t g = id_[i];
    const float p[3] = {io.x[g], io.y[g], io.z[g]};
    uint32_t rgb[3] = {0u, 0u, 0u};
    if (want & kOutRGB) {
      rgb[0] = io.rgb[3 * (size_t)g];
      rgb[1] = io.rgb[3 * (size_t)g + 1];
      rgb[2] = io.rgb[3 * (size_t)g + 2];
    }
    float r[3], dv[3];
    for (int a = 0; a < 3; ++a) {
      const uint32_t k = cell_coord(p[a], f.mn[a], f.inv);
      r[a] = __fadd_rn(f.mn[a], __fmul_rn((float)k, f.leaf));
      dv[a] = __fsub_rn(p[a], r[a]);
    }
    const bool head = (hmask >> i) & 1u;
    if (head) {
      if (!seen_head) {
        pre = cur;
        seen_head = true;
      } else {
        // a segment that opened and closed inside this thread
        finalize_row(io, want, excl_t + hb + lh - 1, N, cur, nullptr, cur_c);
      }
      acc_zero(cur);
      ++lh;
      cur_hp = (uint32_t)(s0 + base + i);
      cur_c.lo = lo_[i];
      cur_c.hi = hi_[i];
      cur_c.ref = g;
      for (int a = 0; a < 3; ++a) cur_c.r[a] = r[a];
    } else if (!seen_head && cur.n == 0) {
      pre_c.lo = lo_[i];
      pre_c.hi = hi_[i];
      for (int a = 0; a < 3; ++a) pre_c.r[a] = r[a];
    }
    acc_add(cur, dv, rgb);
    if (want & kOutPointCell) io.point_cell[g] = (int32_t)(excl_t + hb + lh - 1);
  }
  if (!seen_head) pre = cur;

  // ---- block segmented scan of the threads' open ends
  Seg mine;
  mine.f = seen_head ? 1u : 0u;
  mine.hp = seen_head ? cur_hp : 0u;
  mine.a = seen_head ? cur : pre;
  Seg incl = mine;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    Seg o = seg_shfl_up(incl, off);
    if (lane >= off) incl = seg_combine(o, incl);
  }
  if (lane == 63) S.wtot[w] = incl;
  __syncthreads();
  Seg wp;
  wp.f = 0;
  wp.hp = 0;
  acc_zero(wp.a);
  for (int i = 0; i < w; ++i) wp = seg_combine(wp, S.wtot[i]);
  Seg ex = seg_shfl_up(incl, 1);
  if (lane == 0) {
    ex.f = 0;
    ex.hp = 0;
    acc_zero(ex.a);
  }
  ex = seg_combine(wp, ex);

  // (i) the segment open at this thread's start closes at its first head
  if (seen_head) {
    Acc tot = ex.a;
    acc_merge(tot, pre);
    if (tot.n > 0) {
      if (ex.f) {
        CellOut c = pre.n ? pre_c : cur_c;  // key/corner from any member
        if (pre.n == 0) {
          // all of its members sit in earlier threads: read them back
          const uint32_t pos = ex.hp;
          c.lo = klo[pos];
          c.hi = f.wide ? khi[pos] : 0u;
          const uint32_t g = min(kid[pos], (uint32_t)(N - 1));
          const float p[3] = {io.x[g], io.y[g], io.z[g]};
          for (int a = 0; a < 3; ++a)
            c.r[a] = __fadd_rn(f.mn[a], __fmul_rn((float)cell_coord(p[a], f.mn[a], f.inv), f.leaf));
        }
        c.ref = kid[ex.hp];
        finalize_row(io, want, excl_t + hb - 1, N, tot, nullptr, c);
      } else {
        // opened in an earlier tile: combined below with the earlier tiles' parts
        CellOut c = pre.n ? pre_c : cur_c;
        if (pre.n == 0) {
          const int64_t pos = s0;  // the tile's first item belongs to it
          c.lo = klo[pos];
          c.hi = f.wide ? khi[pos] : 0u;
          const uint32_t g = min(kid[pos], (uint32_t)(N - 1));
          const float p[3] = {io.x[g], io.y[g], io.z[g]};
          for (int a = 0; a < 3; ++a)
            c.r[a] = __fadd_rn(f.mn[a], __fmul_rn((float)cell_coord(p[a], f.mn[a], f.inv), f.leaf));
        }
        S.span_acc = tot;
        S.span_lo = c.lo;
        S.span_hi = c.hi;
        for (int a = 0; a < 3; ++a) S.span_r[a] = c.r[a];
        S.span_pending = 1;
      }
    }
  }
  // (ii) the thread holding the tile's last item closes or hands on the last segment
  if (cnt > 0 && base < cnt && base + K >= cnt) {
    Seg last = seg_combine(ex, mine);
    const int64_t e = s0 + cnt;
    bool cont = false;
    if (e < nv) {
      cont = klo[e] == lo_[cnt - 1 - base] && (!f.wide || khi[e] == hi_[cnt - 1 - base]);
    }
    CellOut c;
    c.lo = lo_[cnt - 1 - base];
    c.hi = hi_[cnt - 1 - base];
    {
      const uint32_t g = id_[cnt - 1 - base];
      const float p[3] = {io.x[g], io.y[g], io.z[g]};
      for (int a = 0; a < 3; ++a)
        c.r[a] = __fadd_rn(f.mn[a], __fmul_rn((float)cell_coord(p[a], f.mn[a], f.inv), f.leaf));
    }
    if (cont) {
      Frag fr;
      fr.n = last.a.n;
      for (int a = 0; a < 3; ++a) {
        fr.s[a] = last.a.s[a];
        fr.c[a] = last.a.c[a];
        fr.rgb[a] = last.a.rgb[a];
      }
      fr.pad[0] = fr.pad[1] = 0;
      ws.frag[t] = fr;
      fence_rel();
      st_rlx(&ws.fflag[t], 1u);
    } else if (last.f) {
      c.ref = kid[last.hp];
      finalize_row(io, want, excl_t + (int64_t)H - 1, N, last.a, nullptr, c);
    } else {
      S.span_acc = last.a;
      S.span_lo = c.lo;
      S.span_hi = c.hi;
      for (int a = 0; a < 3; ++a) S.span_r[a] = c.r[a];
      S.span_pending = 1;
    }
  }
  __syncthreads();

  // ---- a segment that began in an earlier tile and ends in this one
  if (S.span_pending) {
    if (threadIdx.x == 0) {
      // first position of this key in the frame's sorted keys
      uint32_t lo = 0, hi = (uint32_t)s0;
      const uint64_t key = ((uint64_t)S.span_hi << 32) | S.span_lo;
      while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        uint64_t km = ((uint64_t)(f.wide ? khi[mid] : 0u) << 32) | klo[mid];
        if (km < key) lo = mid + 1;
        else hi = mid;
      }
      S.span_start = lo;
    }
    __syncthreads();
    const uint32_t start = S.span_start;
    const int th = (int)(start / (uint32_t)C::TR);
    const int nf = j - th;
    const int tbase = (int)ws.tpr[b] + th;
    Acc part;
    acc_zero(part);
    uint64_t wide_rgb[3] = {0, 0, 0};
    for (int k = threadIdx.x; k < nf; k += C::BLOCK) {
      if (wait_geq(&ws.fflag[tbase + k], 1u, ws.ctl)) fence_acq();
      const Frag fr = ws.frag[tbase + k];
      Acc a;
      a.n = fr.n;
      for (int q = 0; q < 3; ++q) {
        a.s[q] = fr.s[q];
        a.c[q] = fr.c[q];
        a.rgb[q] = 0u;
        wide_rgb[q] += fr.rgb[q];
      }
      acc_merge(part, a);
    }
    S.part[threadIdx.x] = part;
    __syncthreads();
    for (int stride = C::BLOCK / 2; stride > 0; stride >>= 1) {
      if ((int)threadIdx.x < stride) {
        Acc a = S.part[threadIdx.x];
        acc_merge(a, S.part[threadIdx.x + stride]);
        S.part[threadIdx.x] = a;
      }
      __syncthreads();
    }
    // colour sums of the parts, 64-bit: reuse the part slots thread by thread
    for (int q = 0; q < 3; ++q) {
      S.part[threadIdx.x].rgb[0] = (uint32_t)wide_rgb[q];
      S.part[threadIdx.x].rgb[1] = (uint32_t)(wide_rgb[q] >> 32);
      __syncthreads();
      if (threadIdx.x == 0) {
        uint64_t sum = 0;
        for (int i = 0; i < C::BLOCK; ++i)
          sum += ((uint64_t)S.part[i].rgb[1] << 32) | S.part[i].rgb[0];
        wide_rgb[q] = sum;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      Acc tot = S.part[0];
      acc_merge(tot, S.span_acc);
      uint64_t rgbw[3];
      for (int q = 0; q < 3; ++q) rgbw[q] = wide_rgb[q] + S.span_acc.rgb[q];
      CellOut c;
      c.lo = S.span_lo;
      c.hi = S.span_hi;
      c.ref = kid[start];
      for (int a = 0; a < 3; ++a) c.r[a] = S.span_r[a];
      finalize_row(io, want, excl_t - 1, N, tot, rgbw, c);
    }
  }
}

// ---------------------------------------------------------- pipeline ----
template <class C>
__device__ __forceinline__ int find_frame(const uint32_t* tp, int B, int t) {
  int lo = 0, hi = B;  // largest b with tp[b] <= t
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if ((int)tp[mid] <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <class C>
__global__ __launch_bounds__(C::BLOCK) void vg_pipeline_kernel(Ws ws, int ph_lo, int ph_hi) {
  __shared__ typename C::Smem sm;
  __shared__ uint32_t s_item;
  const CallHdr hdr = *ws.hdr;
  const Io io = *ws.io;
  const int B = hdr.B, NTs = hdr.NTs, NTr = hdr.NTr;
  const bool persistent = (ph_lo == 0 && ph_hi == C::NPH);
  uint32_t* counter = persistent ? &ws.ctl->queue[0] : &ws.ctl->queue[1 + ph_lo];
  const uint32_t total = persistent ? (uint32_t)(C::PH_RED * NTs + NTr)
                                    : (uint32_t)(ph_lo == C::PH_RED ? NTr : NTs);
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t item = s_item;
    __syncthreads();
    if (item >= total) break;
    int ph, t;
    uint32_t phase_base;
    if (persistent) {
      ph = min((int)(item / (uint32_t)NTs), C::PH_RED);
      phase_base = (uint32_t)ph * (uint32_t)NTs;
      t = (int)(item - phase_base);
    } else {
      ph = ph_lo;
      phase_base = 0;
      t = (int)item;
    }
    const bool red = ph == C::PH_RED;
    const uint32_t* tp = red ? ws.tpr : ws.tps;
    const int b = find_frame<C>(tp, B, t);
    const int j = t - (int)tp[b];
    const int ntb = (int)(ws.tps[b + 1] - ws.tps[b]);
    if (ph == C::PH_BBOX) {
      bbox_tile<C>(ws, io, sm, b, j, hdr.want);
    } else {
      // wait for what this tile depends on
      if (threadIdx.x == 0) {
        wait_geq(&ws.fs[b].bbox_done, (uint32_t)ntb, ws.ctl);
        if (ph >= C::PH_SORT0) wait_geq(&ws.fs[b].hist_done, (uint32_t)ntb, ws.ctl);
        fence_acq();
      }
      __syncthreads();
      fence_acq();
      const FrameParams f = frame_params(ws, b, hdr.key_mode, C::W);
      if (ph == C::PH_HIST) {
        hist_tile<C>(ws, io, sm, b, j, t, f, hdr.key_mode, hdr.want);
      } else if (ph < C::PH_RED) {
        const int p = ph - C::PH_SORT0;
        if (p >= f.passes) {
          // nothing of this frame in this pass: let the queue jump past it
          if (threadIdx.x == 0)
            atomicMax(counter, phase_base + ws.tps[b + 1]);
        } else {
          if (p > 0) {
            if (threadIdx.x == 0) {
              wait_geq(&ws.fs[b].pass_done[p - 1], (uint32_t)ntb, ws.ctl);
              fence_acq();
            }
            __syncthreads();
            fence_acq();
          }
          sort_tile<C>(ws, io, sm, b, j, t, p, f, hdr.key_mode);
        }
      } else {
        if (f.passes > 0 && f.status == kFrameOk) {
          if (threadIdx.x == 0) {
            wait_geq(&ws.fs[b].pass_done[f.passes - 1], (uint32_t)ntb, ws.ctl);
            fence_acq();
          }
          __syncthreads();
          fence_acq();
        }
        red_tile<C>(ws, io, sm, b, j, t, f, hdr.want, B, NTr, hdr.N);
      }
    }
    __syncthreads();
  }
}

// Clears the per-call state (a fill kernel: graph-safe, no memset nodes).
__global__ void vg_init_kernel(Ws ws) {
  const CallHdr hdr = *ws.hdr;
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nth = (size_t)gridDim.x * blockDim.x;
  uint32_t* ctl = reinterpret_cast<uint32_t*>(ws.ctl);
  for (size_t i = tid; i < sizeof(Ctl) / 4; i += nth) ctl[i] = 0u;
  uint32_t* fs = reinterpret_cast<uint32_t*>(ws.fs);
  for (size_t i = tid; i < (size_t)hdr.B * (sizeof(FrameState) / 4); i += nth) fs[i] = 0u;
  for (size_t i = tid; i < (size_t)hdr.B * ws.slots * ws.R; i += nth) ws.hist[i] = 0u;
  for (size_t i = tid; i < (size_t)hdr.NTr; i += nth) {
    ws.rdesc[i] = 0ull;
    ws.fflag[i] = 0u;
  }
}

// dL/dp_i = G[c] / count[c], c = point_cell[i]; zero where c < 0.
__global__ void vg_backward_kernel(const float* gx, const float* gy, const float* gz,
                                   const uint32_t* count, int64_t m, const int32_t* pc, int64_t n,
                                   float* dx, float* dy, float* dz) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nth) {
    const int32_t c = pc[i];
    float vx = 0.f, vy = 0.f, vz = 0.f;
    if (c >= 0 && c < m) {
      const float fn = (float)count[c];
      vx = __fdiv_rn(gx[c], fn);
      vy = __fdiv_rn(gy[c], fn);
      vz = __fdiv_rn(gz[c], fn);
    }
    dx[i] = vx;
    dy[i] = vy;
    dz[i] = vz;
  }
}

}  // namespace vg

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
__device__ __forceinline__ bool wait_geq(const uint32_t* p, uint32_t target, Ctl* ctl) {
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

// Lane moves within a wave by DPP (data-parallel primitives: a VALU operand
// read from another lane, no LDS).  A row is 16 lanes.  row_shr:k (0x110+k)
// reads the lane k below in the same row, 0 past the row start; row_bcast:15
// (0x142) and row_bcast:31 (0x143) read lane 15 / 31 of the row block before,
// into the rows that ROWS selects (the others read 0); wave_shr:1 (0x138)
// reads the lane below across the whole wave, 0 for lane 0.
template <int CTRL, int ROWS, bool BOUND>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, BOUND);
}

// Inclusive prefix sum over the lanes of a wave: within each row by shifts of
// 1, 2, 4, 8, then across rows with the two broadcasts.
__device__ __forceinline__ uint32_t wave_incl_add(uint32_t x) {
  x += dpp_u32<0x111, 0xf, true>(x);
  x += dpp_u32<0x112, 0xf, true>(x);
  x += dpp_u32<0x114, 0xf, true>(x);
  x += dpp_u32<0x118, 0xf, true>(x);
  x += dpp_u32<0x142, 0xa, false>(x);
  x += dpp_u32<0x143, 0xc, false>(x);
  return x;
}

// Exclusive block scan of one u32 per thread; `wsum` holds NW words of LDS.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* wsum, uint32_t& total) {
  constexpr int NW = BLOCK / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_add(v);
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

// Two exclusive block scans at once (one pair of barriers); `wsum` holds 2*NW
// words of LDS.
template <int BLOCK>
__device__ __forceinline__ void block_excl_scan2(uint32_t va, uint32_t vb, uint32_t* wsum,
                                                 uint32_t& ea, uint32_t& eb, uint32_t& ta,
                                                 uint32_t& tb) {
  constexpr int NW = BLOCK / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t ia = wave_incl_add(va), ib = wave_incl_add(vb);
  if (lane == 63) {
    wsum[w] = ia;
    wsum[NW + w] = ib;
  }
  __syncthreads();
  uint32_t ba = 0, bb = 0, sa = 0, sb = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const uint32_t xa = wsum[k], xb = wsum[NW + k];
    ba += (k < w) ? xa : 0u;
    bb += (k < w) ? xb : 0u;
    sa += xa;
    sb += xb;
  }
  __syncthreads();
  ea = ba + ia - va;
  eb = bb + ib - vb;
  ta = sa;
  tb = sb;
}

// Decoupled look-back: sum the published values of tiles k0, k0-1, ... down
// to the first inclusive prefix.  LB descriptors are read per round trip.
constexpr int kLookBatchSort = 2;   // per digit, per round trip

__device__ __forceinline__ uint32_t look_back32(const uint32_t* desc, size_t stride, int k0,
                                                int lo, Ctl* ctl) {
  constexpr int LB = kLookBatchSort;
  uint32_t excl = 0;
  int k = k0;
  uint32_t spins = 0;
  for (;;) {
    uint32_t v[LB];
#pragma unroll
    for (int i = 0; i < LB; ++i)
      v[i] = (k - i >= lo) ? ld_rlx(desc + (size_t)(k - i) * stride) : kFlagP32;
    int used = 0;
    bool done = false;
    for (int i = 0; i < LB; ++i) {
      if (done || used < i) break;
      const uint32_t fl = v[i] & 0xc0000000u;
      if (fl == 0u) break;
      excl += v[i] & kVal32;
      ++used;
      if (fl == kFlagP32) done = true;
    }
    if (done) return excl;
    k -= used;
    if (k < lo) {  // the first tile always holds a prefix
      atomicOr(&ctl->error, 1u);
      return excl;
    }
    if (used == 0) {
      if (++spins > kSpinLimit || ((spins & 255u) == 0u && ld_rlx(&ctl->error))) {
        atomicOr(&ctl->error, 1u);
        return excl;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
}

// The same chain read by a whole wave: lane i reads descriptor k - i, so one
// round trip covers 64 predecessors.  The values of the lanes up to the
// nearest inclusive prefix are summed if every lane before it has published;
// otherwise the published run before the first unpublished lane is summed and
// the wave reads on from there.  Every lane returns the prefix.
__device__ __forceinline__ uint64_t look_back64_wave(const uint64_t* desc, int k0, Ctl* ctl) {
  const int lane = threadIdx.x & 63;
  uint64_t excl = 0;
  int k = k0;
  uint32_t spins = 0;
  for (;;) {
    const int idx = k - lane;
    const uint64_t v = idx >= 0 ? ld_rlx64(desc + idx) : kFlagP64;  // before tile 0: prefix 0
    const uint64_t fl = v & (3ull << 62);
    const uint64_t unready = __ballot(fl == 0);
    const int first_un = unready ? __ffsll((unsigned long long)unready) - 1 : 64;
    const uint64_t below = first_un == 64 ? ~0ull : ((1ull << first_un) - 1ull);
    const uint64_t pre = __ballot(fl == kFlagP64) & below;
    const int last = pre ? __ffsll((unsigned long long)pre) - 1 : first_un - 1;
    uint64_t part = lane <= last ? (v & kVal64) : 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const uint32_t lo = __shfl_xor((uint32_t)part, off);
      const uint32_t hi = __shfl_xor((uint32_t)(part >> 32), off);
      part += ((uint64_t)hi << 32) | lo;
    }
    excl += part;
    if (pre) return excl;
    k -= first_un;
    if (first_un == 0) {
      if (++spins > kSpinLimit || ((spins & 255u) == 0u && ld_rlx(&ctl->error))) {
        if (lane == 0) atomicOr(&ctl->error, 1u);
        return excl;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
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
  bool narrow;  // keys fit 31 bits: the histogram pass stores them for radix pass 0
  int status;
};

// Stored key of an invalid point (never a key of a narrow frame).
constexpr uint32_t kNoKey = 0xffffffffu;

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__device__ __forceinline__ uint32_t compact3(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
  x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
  x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
  x = (x ^ (x >> 32)) & 0x1fffffull;
  return (uint32_t)x;
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
  f.narrow = false;
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
  f.narrow = f.bits <= 31;
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
// Colour sums of a tile-local part are packed in one 64-bit word, 21 bits per
// channel (a reduce tile holds at most 8192 points, 8192 * 255 < 2^21).
struct Acc {
  uint32_t n;
  float s[3], c[3];
  uint64_t rgb;
};

constexpr int kRgbShift = 21;
constexpr uint64_t kRgbMask = (1ull << kRgbShift) - 1;

__device__ __forceinline__ uint64_t rgb_pack(uint32_t rgb24) {
  return (uint64_t)(rgb24 & 0xffu) | ((uint64_t)((rgb24 >> 8) & 0xffu) << kRgbShift) |
         ((uint64_t)((rgb24 >> 16) & 0xffu) << (2 * kRgbShift));
}
__device__ __forceinline__ uint64_t rgb_channel(uint64_t packed, int c) {
  return (packed >> (c * kRgbShift)) & kRgbMask;
}

__device__ __forceinline__ void two_sum_into(float& s, float& c, float v) {
  float t = __fadd_rn(s, v);
  float bp = __fsub_rn(t, s);
  float e = __fadd_rn(__fsub_rn(s, __fsub_rn(t, bp)), __fsub_rn(v, bp));
  s = t;
  c = __fadd_rn(c, e);
}

__device__ __forceinline__ void acc_zero(Acc& a) {
  a.n = 0;
  for (int i = 0; i < 3; ++i) { a.s[i] = 0.f; a.c[i] = 0.f; }
  a.rgb = 0ull;
}

__device__ __forceinline__ void acc_add(Acc& a, const float d[3], uint32_t rgb24) {
  a.n += 1;
  for (int i = 0; i < 3; ++i) two_sum_into(a.s[i], a.c[i], d[i]);
  a.rgb += rgb_pack(rgb24);
}

// a <- a (+) b, a on the left.
__device__ __forceinline__ void acc_merge(Acc& a, const Acc& b) {
  a.n += b.n;
  for (int i = 0; i < 3; ++i) {
    two_sum_into(a.s[i], a.c[i], b.s[i]);
    a.c[i] = __fadd_rn(a.c[i], b.c[i]);
  }
  a.rgb += b.rgb;
}

// Segmented-scan element: f = a head lies in the covered range, a = sums since
// the last such head (or since the start).
struct Seg {
  uint32_t f;
  Acc a;
};

__device__ __forceinline__ Seg seg_combine(const Seg& x, const Seg& y) {
  if (y.f) return y;
  Seg r = x;
  acc_merge(r.a, y.a);
  return r;
}

// A Seg moved between lanes by one DPP control (see dpp_u32); lanes with no
// source read the all-zero Seg, which seg_combine treats as an identity.
template <int CTRL, int ROWS, bool BOUND>
__device__ __forceinline__ Seg seg_dpp(const Seg& v) {
  Seg r;
  r.f = dpp_u32<CTRL, ROWS, BOUND>(v.f);
  r.a.n = dpp_u32<CTRL, ROWS, BOUND>(v.a.n);
  for (int i = 0; i < 3; ++i) {
    r.a.s[i] = __uint_as_float(dpp_u32<CTRL, ROWS, BOUND>(__float_as_uint(v.a.s[i])));
    r.a.c[i] = __uint_as_float(dpp_u32<CTRL, ROWS, BOUND>(__float_as_uint(v.a.c[i])));
  }
  r.a.rgb = ((uint64_t)dpp_u32<CTRL, ROWS, BOUND>((uint32_t)(v.a.rgb >> 32)) << 32) |
            dpp_u32<CTRL, ROWS, BOUND>((uint32_t)v.a.rgb);
  return r;
}

// Inclusive segmented scan over the lanes of a wave (same steps as
// wave_incl_add; the earlier lanes' Seg is always the left operand).
__device__ __forceinline__ Seg wave_incl_seg(Seg x) {
  x = seg_combine(seg_dpp<0x111, 0xf, true>(x), x);
  x = seg_combine(seg_dpp<0x112, 0xf, true>(x), x);
  x = seg_combine(seg_dpp<0x114, 0xf, true>(x), x);
  x = seg_combine(seg_dpp<0x118, 0xf, true>(x), x);
  x = seg_combine(seg_dpp<0x142, 0xa, false>(x), x);
  x = seg_combine(seg_dpp<0x143, 0xc, false>(x), x);
  return x;
}

// ---------------------------------------------------------- configs ----
template <int BLOCK_, int SORT_ITEMS_, int RADIX_, int RED_ITEMS_>
struct Cfg {
  static constexpr int BLOCK = BLOCK_;
  static constexpr int NW = BLOCK / 64;
  static constexpr int SI = SORT_ITEMS_;
  static constexpr int TS = BLOCK * SI;      // sort tile
  static constexpr int KB = 2;
  static constexpr int TB = TS * KB;         // big tile (bbox, histogram)
  static constexpr int W = RADIX_;
  static constexpr int R = 1 << W;
  static constexpr int MAXP = (63 + W - 1) / W;
  static constexpr int RI = RED_ITEMS_;
  static constexpr int TR = BLOCK * RI;      // reduce tile
  static constexpr int PH_BBOX = 0, PH_HIST = 1, PH_SORT0 = 2, PH_RED = 2 + MAXP,
                       PH_FIX = 3 + MAXP, NPH = 4 + MAXP;
  static_assert(R <= BLOCK, "one digit per thread in the look-back");
  static_assert(MAXP <= kMaxPassSlots, "pass slots");
  static_assert(SI <= 32 && RI <= 32, "item masks are 32-bit");
  static_assert(TR <= 8192, "reduce tile: 16-bit item positions, 21-bit colour sums");

  struct SortSmem {
    uint32_t lo[TS];
    uint32_t hi[TS];
    uint32_t idx[TS];
    uint32_t wcnt[NW][R];
    uint32_t gbase[R];
    uint32_t wsum[2 * NW];
  };
  struct HistSmem {
    uint32_t h[MAXP][R];
  };
  struct BboxSmem {
    uint32_t mn[NW][3];
    uint32_t mx[NW][3];
    uint32_t nv[NW];
  };
  struct RedSmem {
    uint32_t klo[TR];
    uint32_t khi[TR];
    uint32_t kid[TR];
    uint16_t hpos[TR];   // tile item of the r-th head of the tile
    uint32_t has_prev, prev_lo, prev_hi, has_next, next_lo, next_hi;
    uint32_t wsum[NW];
    Seg wtot[NW];
    uint64_t excl;
  };
  union Smem {
    SortSmem sort;
    HistSmem hist;
    BboxSmem bbox;
    RedSmem red;
  };
};

// LDS of a kernel entry: every phase's layout for the persistent kernel,
// only its own phase's for a one-phase kernel.
// Phase kinds a kernel can hold (see vg_pipeline_kernel).
enum Kind : int { kAll = 0, kBbox = 1, kHist = 2, kSort = 3, kRed = 4, kFix = 5 };

template <class C, int KIND>
struct SmemOf {
  union type {
    typename C::SortSmem sort;
    typename C::HistSmem hist;
    typename C::BboxSmem bbox;
    typename C::RedSmem red;
  };
};

// Control state of a workgroup, written by thread 0 and read by all.
constexpr int kLdsFrames = 256;  // calls with at most this many frames keep tile prefixes in LDS
constexpr int kFpCache = 64;     // ... and this many, every frame's grid parameters

struct BlockCtl {
  uint32_t item;
  int32_t ph, t, b, j;
  int32_t skip;          // the item needs no work
  int32_t fp_b;          // frame whose parameters are in fp
  int32_t fd_b;          // frame whose description is in fd
  int32_t dep_b[kMaxPassSlots + 3];  // per phase: last frame whose inputs were seen complete
  FrameParams fp;
  FrameDesc fd;
  uint32_t tp[3][kLdsFrames + 1];    // big / sort / reduce tile prefixes over frames
  uint32_t ilv_s[kIlvMaxRounds + 1];
  uint32_t ilv_perm[kIlvMaxFrames];
  int32_t ilv_rounds;                // rounds of the round-robin sort order (0: frame order)
  uint32_t ilv_total;                // items of a one-pass launch's own order
  uint32_t scan_w[32];               // block scan scratch
  int32_t cached;                    // one-phase launches after the bbox: every frame below
  FrameParams fpa[kFpCache];
  FrameDesc fda[kFpCache];
  uint32_t vt0[kFpCache + 1];        // one-phase reduce: first row-count descriptor per frame
};

template <class C>
struct SmemOf<C, 1> {
  union type { typename C::BboxSmem bbox; };
};
template <class C>
struct SmemOf<C, 2> {
  union type { typename C::HistSmem hist; };
};
template <class C>
struct SmemOf<C, 3> {
  union type { typename C::SortSmem sort; };
};
template <class C>
struct SmemOf<C, 4> {
  union type { typename C::RedSmem red; };
};
template <class C>
struct SmemOf<C, 5> {
  union type { typename C::BboxSmem bbox; };
};

// The call's input and output pointers reach the kernels through memory, so
// the compiler cannot tell that they point to global memory and would access
// them with flat instructions, which every LDS wait then also waits for.  The
// kernels use them through this view, whose pointers are global ones.
template <class T>
using gptr = __attribute__((address_space(1))) T*;

struct GIo {
  gptr<const float> x, y, z;
  gptr<const float> vx, vy, vz;  // the point view of the phases after the bbox pass
  gptr<const uint8_t> rgb;
  gptr<float> cx, cy, cz;
  gptr<uint8_t> crgb;
  gptr<uint32_t> count;
  gptr<uint64_t> key;
  gptr<int32_t> point_cell;
  gptr<uint32_t> ref_index;
  gptr<float> lx, ly, lz;
  gptr<int64_t> out_offsets;
  gptr<int32_t> frame_status;
};

__device__ __forceinline__ GIo global_view(const Io& o) {
  GIo g;
  g.x = (gptr<const float>)o.x;
  g.y = (gptr<const float>)o.y;
  g.z = (gptr<const float>)o.z;
  g.vx = (gptr<const float>)o.vx;
  g.vy = (gptr<const float>)o.vy;
  g.vz = (gptr<const float>)o.vz;
  g.rgb = (gptr<const uint8_t>)o.rgb;
  g.cx = (gptr<float>)o.cx;
  g.cy = (gptr<float>)o.cy;
  g.cz = (gptr<float>)o.cz;
  g.crgb = (gptr<uint8_t>)o.crgb;
  g.count = (gptr<uint32_t>)o.count;
  g.key = (gptr<uint64_t>)o.key;
  g.point_cell = (gptr<int32_t>)o.point_cell;
  g.ref_index = (gptr<uint32_t>)o.ref_index;
  g.lx = (gptr<float>)o.lx;
  g.ly = (gptr<float>)o.ly;
  g.lz = (gptr<float>)o.lz;
  g.out_offsets = (gptr<int64_t>)o.out_offsets;
  g.frame_status = (gptr<int32_t>)o.frame_status;
  return g;
}

// Points of a big tile (bbox and histogram tiles) are read in batches of HB
// per thread, lane-consecutive: point i of a batch goes to lane i mod BLOCK.
template <int HB>
struct Pts {
  float x[HB], y[HB], z[HB];
  uint32_t c[HB];  // packed rgb (bbox tiles only)
};

// VIEW: read the point view (the phases after the bbox pass) instead of the
// input as given (the bbox pass).
template <class C, int HB, bool RGB = true, bool VIEW = false>
__device__ __forceinline__ void load_pts(const GIo& io, Pts<HB>& p, int64_t g0, int64_t last,
                                         bool with_rgb) {
#pragma unroll
  for (int u = 0; u < HB; ++u) {
    const int64_t g = min(g0 + u * C::BLOCK + (int)threadIdx.x, last);
    p.x[u] = VIEW ? io.vx[g] : io.x[g];
    p.y[u] = VIEW ? io.vy[g] : io.y[g];
    p.z[u] = VIEW ? io.vz[g] : io.z[g];
    p.c[u] = 0u;
    if (RGB && with_rgb) {
      const gptr<const uint8_t> q = io.rgb + 3 * (size_t)g;
      p.c[u] = (uint32_t)q[0] | ((uint32_t)q[1] << 8) | ((uint32_t)q[2] << 16);
    }
  }
}

// Points per thread of one batch: 4 in tiles taken from the work queue (the
// persistent kernel holds every phase's registers); in one-phase launches,
// which stream with the next batch in flight, 4 for bbox tiles (which also
// carry colours and write records) and 8 for histogram tiles.
constexpr int kBigBatch = 4;
template <int KIND>
constexpr int kStreamBatch = KIND == kBbox ? 4 : 8;

// A value every lane of the wave holds alike (read from LDS at a uniform
// address), moved to scalar registers.
// One word per lane from global memory straight into LDS: lane l of the wave
// writes dst[l] (dst is the same for the whole wave).  The data is in LDS once
// the wave's vector memory loads have completed (lds_load_wait).
__device__ __forceinline__ void lds_load_word(const uint32_t* src, uint32_t* dst) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                   (__attribute__((address_space(3))) void*)dst, 4, 0, 0);
}
__device__ __forceinline__ void lds_load_wait() { __builtin_amdgcn_s_waitcnt(0); }

template <class T>
__device__ __forceinline__ T wave_uniform(const T& v) {
  static_assert(sizeof(T) % 4 == 0, "whole dwords");
  uint32_t w[sizeof(T) / 4];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

// ---------------------------------------------------------- BBOX tile ----
struct BboxAcc {
  uint32_t mn[3], mx[3], nv;  // order-preserving encodings: max of ~enc (min) and of enc (max)
};

__device__ __forceinline__ void bbox_zero(BboxAcc& a) {
  for (int q = 0; q < 3; ++q) a.mn[q] = a.mx[q] = 0u;
  a.nv = 0u;
}

// One batch: the 16 B record of every point, the valid points' box and count,
// row -1 for invalid points.  `g0` is the batch's first point, `rem` the points
// of the tile from there on.
// A point of a frame with a filter, as every later phase sees it: rotated and
// translated when asked for, p'_a = RN32(RN32(RN32(RN32(r[a][0] x) + RN32(r[a][1] y))
// + RN32(r[a][2] z)) + t[a]); NaN when the point or p' is not finite or p'_z is
// outside the height limit (an invalid point from then on).
__device__ __forceinline__ void apply_xf(const FrameXf& f, float& x, float& y, float& z) {
  const float X = x, Y = y, Z = z;
  if (f.on & kXfRotate) {
    x = __fadd_rn(__fadd_rn(__fadd_rn(__fmul_rn(f.r[0], X), __fmul_rn(f.r[1], Y)),
                            __fmul_rn(f.r[2], Z)), f.t[0]);
    y = __fadd_rn(__fadd_rn(__fadd_rn(__fmul_rn(f.r[3], X), __fmul_rn(f.r[4], Y)),
                            __fmul_rn(f.r[5], Z)), f.t[1]);
    z = __fadd_rn(__fadd_rn(__fadd_rn(__fmul_rn(f.r[6], X), __fmul_rn(f.r[7], Y)),
                            __fmul_rn(f.r[8], Z)), f.t[2]);
  }
  const bool keep = finite3(X, Y, Z) && finite3(x, y, z) && z >= f.zlo && z <= f.zhi;
  if (!keep) {
    x = __builtin_nanf("");
    y = x;
    z = x;
  }
}

// XF: the call has filters; the frame's (f) is applied first and the point
// view written.
template <class C, int HB, bool XF = false>
__device__ __forceinline__ void bbox_batch(const Ws& ws, const GIo& io, BboxAcc& a,
                                           Pts<HB>& p, int64_t g0, int64_t rem, uint32_t want,
                                           const FrameXf* xf = nullptr) {
#pragma unroll
  for (int u = 0; u < HB; ++u) {
    const int64_t i = u * C::BLOCK + (int)threadIdx.x;
    if (i < rem) {
      const int64_t g = g0 + i;
      if constexpr (XF) {
        if (xf->on) apply_xf(*xf, p.x[u], p.y[u], p.z[u]);
        ws.tx[g] = p.x[u];
        ws.ty[g] = p.y[u];
        ws.tz[g] = p.z[u];
      }
      ws.rec[g] = make_float4(p.x[u], p.y[u], p.z[u], __uint_as_float(p.c[u]));
      if (finite3(p.x[u], p.y[u], p.z[u])) {
        const uint32_t ex = f2ord(p.x[u]), ey = f2ord(p.y[u]), ez = f2ord(p.z[u]);
        a.mn[0] = max(a.mn[0], ~ex); a.mn[1] = max(a.mn[1], ~ey); a.mn[2] = max(a.mn[2], ~ez);
        a.mx[0] = max(a.mx[0], ex); a.mx[1] = max(a.mx[1], ey); a.mx[2] = max(a.mx[2], ez);
        a.nv += 1;
      } else if (want & kOutPointCell) {
        io.point_cell[g] = -1;
      }
    }
  }
}

// End of a bbox tile: block reduction, frame atomics, done counter.
template <class C>
__device__ __forceinline__ void bbox_finish(const Ws& ws, typename C::BboxSmem& bs, BboxAcc& a,
                                            int b, bool persistent, uint32_t tiles = 1u) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    for (int q = 0; q < 3; ++q) {
      a.mn[q] = max(a.mn[q], (uint32_t)__shfl_xor(a.mn[q], off));
      a.mx[q] = max(a.mx[q], (uint32_t)__shfl_xor(a.mx[q], off));
    }
    a.nv += __shfl_xor(a.nv, off);
  }
  if (lane == 0) {
    for (int q = 0; q < 3; ++q) { bs.mn[w][q] = a.mn[q]; bs.mx[w][q] = a.mx[q]; }
    bs.nv[w] = a.nv;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tn = 0;
    for (int i = 0; i < C::NW; ++i) {
      tn += bs.nv[i];
      for (int q = 0; q < 3; ++q) {
        a.mn[q] = max(a.mn[q], bs.mn[i][q]);
        a.mx[q] = max(a.mx[q], bs.mx[i][q]);
      }
    }
    FrameState* fs = ws.fs + b;
    if (tn) {
      for (int q = 0; q < 3; ++q) {
        atomicMax(&fs->mn_neg[q], a.mn[q]);
        atomicMax(&fs->mx[q], a.mx[q]);
      }
      atomicAdd(&fs->n_valid, tn);
    }
    if (persistent) fence_rel();
    atomicAdd(&fs->bbox_done, tiles);
  }
  __syncthreads();  // bs is reused by the next tile
}

template <class C>
__device__ void bbox_tile(const Ws& ws, const GIo& io, typename C::BboxSmem& bs, const FrameDesc& fd,
                          int b, int j, uint32_t want, bool persistent) {
  constexpr int HB = kBigBatch;
  static_assert(C::TB % (C::BLOCK * HB) == 0, "big tile = whole load batches");
  const int64_t t0 = (int64_t)j * C::TB;
  const int64_t cnt = min((int64_t)C::TB, fd.n - t0);
  BboxAcc a;
  bbox_zero(a);
  const bool xf = (ws.hdr->filt & kFiltView) != 0;
  FrameXf fx;
  if (xf) fx = ws.xf[b];
  for (int64_t c = 0; c < cnt; c += C::BLOCK * HB) {
    Pts<HB> p;
    load_pts<C, HB>(io, p, fd.off + t0 + c, fd.off + fd.n - 1, io.rgb != nullptr);
    if (xf) bbox_batch<C, HB, true>(ws, io, a, p, fd.off + t0 + c, cnt - c, want, &fx);
    else bbox_batch<C, HB>(ws, io, a, p, fd.off + t0 + c, cnt - c, want);
  }
  bbox_finish<C>(ws, bs, a, b, persistent);
}

__device__ __forceinline__ uint32_t digit_of(uint32_t lo, uint32_t hi, int shift, uint32_t mask) {
  const uint64_t k = ((uint64_t)hi << 32) | lo;
  return (uint32_t)(k >> shift) & mask;
}

__device__ __forceinline__ uint64_t key_of_point(const FrameParams& f, int key_mode, float x,
                                                 float y, float z) {
  return point_key(f, key_mode, cell_coord(x, f.mn[0], f.inv), cell_coord(y, f.mn[1], f.inv),
                   cell_coord(z, f.mn[2], f.inv));
}

// ---------------------------------------------------------- HIST tile ----
// Start of a histogram tile: the look-back descriptors of the radix tiles
// under it start cleared.
template <class C>
__device__ __forceinline__ void hist_start(const Ws& ws, const FrameDesc& fd, int j,
                                           const FrameParams& f) {
  if (f.status == kFrameOverflow) return;
  const int s_lo = j * C::KB, s_hi = min((j + 1) * C::KB, fd.nts);
  for (int p = 0; p < f.passes; ++p) {
    for (int st = s_lo; st < s_hi; ++st) {
      uint32_t* row = ws.sdesc + ((size_t)p * ws.capNTs + fd.ts0 + st) * C::R;
      for (int d = threadIdx.x; d < C::R; d += C::BLOCK) row[d] = 0u;
    }
  }
}

// The key of point_key with the key mode and key width fixed at compile time.
template <int KM, bool WIDE>
__device__ __forceinline__ uint64_t key_fixed(const FrameParams& f, float x, float y, float z) {
  const uint32_t kx = cell_coord(x, f.mn[0], f.inv);
  const uint32_t ky = cell_coord(y, f.mn[1], f.inv);
  const uint32_t kz = cell_coord(z, f.mn[2], f.inv);
  if constexpr (KM == 1) return spread3(kx) | (spread3(ky) << 1) | (spread3(kz) << 2);
  else if constexpr (!WIDE) return (uint64_t)(kx + f.d[0] * (ky + f.d[1] * kz));
  else return (uint64_t)kx + (uint64_t)f.d[0] * ((uint64_t)ky + (uint64_t)f.d[1] * (uint64_t)kz);
}

template <class C, int HB, int KM, bool WIDE>
__device__ __forceinline__ void hist_batch_fixed(const Ws& ws, typename C::HistSmem& hs,
                                                 const FrameParams& f, const Pts<HB>& p,
                                                 int64_t g0, int64_t rem) {
  const int lane = threadIdx.x & 63;
  const int P = f.passes;
  const uint32_t mask = (1u << f.w) - 1u;
#pragma unroll
  for (int u = 0; u < HB; ++u) {
    const bool inr = u * C::BLOCK + (int)threadIdx.x < rem;
    const bool valid = inr && finite3(p.x[u], p.y[u], p.z[u]);
    // an invalid point's key is formed from the grid minimum and dropped
    const uint64_t k = key_fixed<KM, WIDE>(f, valid ? p.x[u] : f.mn[0], valid ? p.y[u] : f.mn[1],
                                           valid ? p.z[u] : f.mn[2]);
    const uint32_t lo = valid ? (uint32_t)k : 0u;
    const uint32_t hi = WIDE && valid ? (uint32_t)(k >> 32) : 0u;
    if (!WIDE && f.narrow && inr) ws.lo[0][g0 + u * C::BLOCK + (int)threadIdx.x] = valid ? lo : kNoKey;
    const uint64_t vb = __ballot(valid);
    const uint32_t plo = dpp_u32<0x138, 0xf, true>(lo);  // the lane below's key
    const uint32_t phi = WIDE ? dpp_u32<0x138, 0xf, true>(hi) : 0u;
    const bool prev_same = lane > 0 && ((vb >> (lane - 1)) & 1ull) && plo == lo && phi == hi;
    const bool head = valid && !prev_same;
    const uint64_t brk = __ballot(head) | ~vb;  // a run ends before a head or an invalid lane
    if (head) {
      const uint64_t after = lane == 63 ? 0ull : brk & (~0ull << (lane + 1));
      const uint32_t len = (uint32_t)((after ? __ffsll((unsigned long long)after) - 1 : 64) - lane);
      for (int q = 0; q < P; ++q) atomicAdd(&hs.h[q][digit_of(lo, hi, q * f.w, mask)], len);
    }
  }
}

// One batch: every pass's digit counted in the LDS histogram.  Neighbouring
// lanes hold neighbouring points, which mostly fall in one cell: every run of
// equal keys over consecutive valid lanes adds its length to each pass's digit
// once, from its first lane.  Keys of frames that fit 31 bits are stored for
// radix pass 0.  An overflowing frame's points get row -1.
template <class C, int HB>
__device__ __forceinline__ void hist_batch(const Ws& ws, const GIo& io, typename C::HistSmem& hs,
                                           const FrameParams& f, int key_mode, const Pts<HB>& p,
                                           int64_t g0, int64_t rem, uint32_t want) {
  if (f.status == kFrameOverflow) {
    if (want & kOutPointCell) {
#pragma unroll
      for (int u = 0; u < HB; ++u) {
        const int64_t i = u * C::BLOCK + (int)threadIdx.x;
        if (i < rem) io.point_cell[g0 + i] = -1;
      }
    }
    return;
  }
  if (f.passes == 0) return;
  if (key_mode == 1) {
    if (f.wide) hist_batch_fixed<C, HB, 1, true>(ws, hs, f, p, g0, rem);
    else hist_batch_fixed<C, HB, 1, false>(ws, hs, f, p, g0, rem);
  } else {
    if (f.wide) hist_batch_fixed<C, HB, 0, true>(ws, hs, f, p, g0, rem);
    else hist_batch_fixed<C, HB, 0, false>(ws, hs, f, p, g0, rem);
  }
}

// End of a histogram tile: the LDS counts go to the frame's histograms (and
// are cleared for the next tile), then the done counters.
// `call_counters`: also the call-wide counters (a streaming launch adds its
// workgroup's totals to them once, at its end).
template <class C>
__device__ __forceinline__ void hist_finish(const Ws& ws, typename C::HistSmem& hs, int b,
                                            const FrameParams& f, bool persistent,
                                            uint32_t tiles = 1u, bool call_counters = true) {
  const int P = f.status == kFrameOverflow ? 0 : f.passes;
  __syncthreads();
  for (int i = threadIdx.x; i < P * C::R; i += C::BLOCK) {
    const int q = i / C::R, d = i % C::R;
    const uint32_t v = hs.h[q][d];
    if (v) {
      atomicAdd(&ws.hist[((size_t)b * ws.slots + q) * C::R + d], v);
      hs.h[q][d] = 0u;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (P > 0 && call_counters) atomicMax(&ws.ctl->max_passes, (uint32_t)P);
    if (persistent) fence_rel();
    atomicAdd(&ws.fs[b].hist_done, tiles);
    if (call_counters) atomicAdd(&ws.ctl->hist_tiles_done, tiles);
  }
}

template <class C>
__device__ void hist_tile(const Ws& ws, const GIo& io, typename C::HistSmem& hs, const FrameDesc& fd,
                          int b, int j, const FrameParams& f, int key_mode, uint32_t want,
                          bool persistent) {
  constexpr int HB = kBigBatch;
  static_assert(C::TB % (C::BLOCK * HB) == 0, "big tile = whole load batches");
  const int64_t t0 = (int64_t)j * C::TB;
  const int64_t cnt = min((int64_t)C::TB, fd.n - t0);
  // the LDS histogram shares its memory with other phases' tiles
  for (int i = threadIdx.x; i < C::MAXP * C::R; i += C::BLOCK) (&hs.h[0][0])[i] = 0u;
  hist_start<C>(ws, fd, j, f);
  __syncthreads();
  for (int64_t c = 0; c < cnt; c += C::BLOCK * HB) {
    Pts<HB> p;
    load_pts<C, HB, false, true>(io, p, fd.off + t0 + c, fd.off + fd.n - 1, false);
    hist_batch<C, HB>(ws, io, hs, f, key_mode, p, fd.off + t0 + c, cnt - c, want);
  }
  hist_finish<C>(ws, hs, b, f, persistent);
}

// Big tiles of a one-phase bbox or histogram launch (frames cached in LDS,
// at least one point in the call).  These tiles wait on nothing, so tile t
// goes to workgroup t mod G without a queue (the workgroups read neighbouring
// tiles at any one time; runs of consecutive tiles per workgroup measured
// slower), and each workgroup streams its tiles' points: the next batch (of
// this tile or of the workgroup's next tile) is requested before the current
// one is processed.  That request is made on every iteration (of point 0 when
// there is no next batch), so the number of loads in flight is the same on
// every path and the wait for the current batch does not drain the next one.
// A workgroup's successive tiles of one frame (a cloud of more than G tiles)
// share one accumulation (box, LDS histogram), handed to the frame's totals
// when the frame changes or the tiles run out: one set of frame atomics per
// frame and workgroup, not per tile, which a single large cloud would
// otherwise queue by the thousand on one line.
template <class C, int KIND, bool RGB, bool XF = false>
__device__ void stream_big_tiles(const Ws& ws, const GIo& io, const CallHdr& hdr, BlockCtl& bc,
                                 typename SmemOf<C, KIND>::type& sm) {
  constexpr bool VIEW = KIND == kHist;  // the histogram reads the point view
  constexpr int HB = kStreamBatch<KIND>;
  constexpr int64_t BS = (int64_t)C::BLOCK * HB;
  static_assert(C::TB % (C::BLOCK * HB) == 0, "big tile = whole load batches");
  const int G = gridDim.x, NT = hdr.NTb;
  if constexpr (KIND == kHist) {
    for (int i = threadIdx.x; i < C::MAXP * C::R; i += C::BLOCK) (&sm.hist.h[0][0])[i] = 0u;
  }
  // tile t -> frame b (largest b with tp[b] <= t), tile j in it
  auto frame_of = [&](int t) {
    int lo = 0, hi = hdr.B;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if ((int)bc.tp[0][mid] <= t) lo = mid;
      else hi = mid;
    }
    return __builtin_amdgcn_readfirstlane(lo);
  };
  int t = blockIdx.x;
  if (t >= NT) return;
  uint32_t ntl = 0;  // tiles accumulated since the last hand-over
  uint32_t nall = 0, pmax = 0;  // the workgroup's tiles and largest pass count (histogram)
  int b = frame_of(t);
  int64_t t0 = (int64_t)(t - (int)__builtin_amdgcn_readfirstlane(bc.tp[0][b])) * C::TB;
  int64_t off = wave_uniform(bc.fda[b].off), fn = wave_uniform(bc.fda[b].n);
  int64_t cnt = min((int64_t)C::TB, fn - t0);
  int64_t c = 0;  // batch start within the tile
  Pts<HB> cur, nxt;
  if (cnt > 0) load_pts<C, HB, RGB, VIEW>(io, cur, off + t0, off + fn - 1, true);
  else load_pts<C, HB, RGB, VIEW>(io, cur, 0, 0, true);
  BboxAcc acc;
  bbox_zero(acc);
  FrameXf fx;
  if constexpr (XF) fx = wave_uniform(ws.xf[b]);
  FrameParams f;
  if constexpr (KIND == kHist) {
    f = wave_uniform(bc.fpa[b]);
    hist_start<C>(ws, bc.fda[b], (int)(t0 / C::TB), f);
  }
  __syncthreads();
  for (;;) {
    // the batch after this one
    int t2 = t, b2 = b;
    int64_t t02 = t0, off2 = off, fn2 = fn, cnt2 = cnt, c2 = c + BS;
    if (c2 >= cnt) {
      t2 = t + G;
      c2 = 0;
      if (t2 < NT) {
        b2 = frame_of(t2);
        t02 = (int64_t)(t2 - (int)__builtin_amdgcn_readfirstlane(bc.tp[0][b2])) * C::TB;
        off2 = wave_uniform(bc.fda[b2].off);
        fn2 = wave_uniform(bc.fda[b2].n);
        cnt2 = min((int64_t)C::TB, fn2 - t02);
      }
    }
    const bool more = t2 < NT && cnt2 > 0;
    load_pts<C, HB, RGB, VIEW>(io, nxt, more ? off2 + t02 + c2 : 0, more ? off2 + fn2 - 1 : 0, true);
    if (cnt > 0) {
      if constexpr (KIND == kBbox)
        bbox_batch<C, HB, XF>(ws, io, acc, cur, off + t0 + c, cnt - c, hdr.want, &fx);
      else hist_batch<C, HB>(ws, io, sm.hist, f, hdr.key_mode, cur, off + t0 + c, cnt - c, hdr.want);
    }
    if (t2 != t) {
      ++ntl;
      const bool hand_over = t2 >= NT || b2 != b;
      if constexpr (KIND == kBbox) {
        if (hand_over) {
          bbox_finish<C>(ws, sm.bbox, acc, b, false, ntl);
          bbox_zero(acc);
          ntl = 0;
          if constexpr (XF) {
            if (t2 < NT) fx = wave_uniform(ws.xf[b2]);
          }
        }
      } else {
        if (hand_over) {
          hist_finish<C>(ws, sm.hist, b, f, false, ntl, false);
          nall += ntl;
          if (f.status != kFrameOverflow) pmax = max(pmax, (uint32_t)f.passes);
          ntl = 0;
        }
        if (t2 < NT) {
          if (hand_over) f = wave_uniform(bc.fpa[b2]);
          hist_start<C>(ws, bc.fda[b2], (int)(t02 / C::TB), f);
        }
      }
      if (t2 >= NT) {
        if constexpr (KIND == kHist) {
          if (threadIdx.x == 0) {
            if (pmax > 0) atomicMax(&ws.ctl->max_passes, pmax);
            atomicAdd(&ws.ctl->hist_tiles_done, nall);
          }
        }
        break;
      }
    }
    cur = nxt;
    t = t2;
    b = b2;
    t0 = t02;
    off = off2;
    fn = fn2;
    cnt = cnt2;
    c = c2;
  }
}

// ---------------------------------------------------------- SORT tile ----
template <class C>
__device__ void sort_tile(const Ws& ws, const GIo& io, typename C::SortSmem& S, const FrameDesc& fd,
                          int b, int j, int p, const FrameParams& f, int key_mode,
                          bool persistent) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int Rb = 1 << f.w;
  const uint32_t mask = (uint32_t)Rb - 1u;
  const int shift = p * f.w;
  const int64_t t0 = (int64_t)j * C::TS;
  const int t = fd.ts0 + j;
  if (p > 0 && t0 >= (int64_t)f.n_valid) {
    // past the frame's valid points (only later tiles of the frame, which no
    // tile looks back at)
    if (threadIdx.x == 0) {
      if (persistent) fence_rel();
      atomicAdd(&ws.fs[b].pass_done[p], 1u);
    }
    return;
  }

  // this pass's digit counts of the frame (scanned with the tile's counts)
  uint32_t hv = 0;
  if ((int)threadIdx.x < Rb) hv = ws.hist[((size_t)b * ws.slots + p) * C::R + threadIdx.x];
  // this wave's digit counters (no other wave touches them before the
  // barrier that ends the ranking)
  for (int k = lane; k < C::R; k += 64) S.wcnt[w][k] = 0u;

  // items in wave-striped order: wave w owns 64*SI consecutive positions
  uint32_t klo[C::SI], khi[C::SI], kid[C::SI];
  uint32_t vm = 0;
  const int64_t wbase = t0 + (int64_t)w * 64 * C::SI + lane;
  if (p == 0 && f.narrow) {
    // keys stored by the histogram pass, in input order
    const int64_t last = fd.off + max(fd.n - 1, (int64_t)0);
#pragma unroll
    for (int it = 0; it < C::SI; ++it) klo[it] = ws.lo[0][min(fd.off + wbase + it * 64, last)];
#pragma unroll
    for (int it = 0; it < C::SI; ++it) {
      const int64_t pos = wbase + it * 64;
      khi[it] = 0u;
      kid[it] = (uint32_t)(fd.off + pos);
      if (pos < fd.n && klo[it] != kNoKey) vm |= 1u << it;
    }
  } else if (p == 0) {
    const int64_t last = fd.off + max(fd.n - 1, (int64_t)0);
    float xs[C::SI], ys[C::SI], zs[C::SI];
#pragma unroll
    for (int it = 0; it < C::SI; ++it) {
      const int64_t g = min(fd.off + wbase + it * 64, last);
      xs[it] = io.vx[g];
      ys[it] = io.vy[g];
      zs[it] = io.vz[g];
    }
#pragma unroll
    for (int it = 0; it < C::SI; ++it) {
      const int64_t pos = wbase + it * 64;
      klo[it] = 0u;
      khi[it] = 0u;
      kid[it] = (uint32_t)(fd.off + pos);
      if (pos < fd.n && finite3(xs[it], ys[it], zs[it])) {
        const uint64_t k = key_of_point(f, key_mode, xs[it], ys[it], zs[it]);
        klo[it] = (uint32_t)k;
        khi[it] = (uint32_t)(k >> 32);
        vm |= 1u << it;
      }
    }
  } else {
    const int src = p & 1;
    const uint32_t* slo = ws.lo[src] + fd.off;
    const uint32_t* shi = ws.hi[src] + fd.off;
    const uint32_t* sid = ws.idx[src] + fd.off;
    const int64_t last = max((int64_t)f.n_valid - 1, (int64_t)0);
#pragma unroll
    for (int it = 0; it < C::SI; ++it) {
      const int64_t pos = min(wbase + it * 64, last);
      klo[it] = slo[pos];
      khi[it] = f.wide ? shi[pos] : 0u;
      kid[it] = sid[pos];
    }
#pragma unroll
    for (int it = 0; it < C::SI; ++it)
      if (wbase + it * 64 < (int64_t)f.n_valid) vm |= 1u << it;
  }
  // rank every item among equal digits of its wave, in input order: the
  // lanes with an equal digit (one ballot per digit bit), then one LDS add per
  // distinct digit, by the group's lowest lane.  A wave's LDS operations take
  // effect in issue order, so the count each add returns is the number of
  // equal digits in the wave's earlier items; the other lanes of the group read
  // it from the lowest lane.
  uint32_t rank[C::SI], dg[C::SI];
  static_assert(C::SI % 2 == 0, "items ranked in pairs");
#pragma unroll
  for (int it = 0; it < C::SI; it += 2) {
    // two items at a time: their ballot chains are independent
    const bool v0 = (vm >> it) & 1u, v1 = (vm >> (it + 1)) & 1u;
    const uint32_t d0 = digit_of(klo[it], khi[it], shift, mask);
    const uint32_t d1 = digit_of(klo[it + 1], khi[it + 1], shift, mask);
    const uint64_t vb0 = __ballot(v0), vb1 = __ballot(v1);
    uint32_t m0lo = (uint32_t)vb0, m0hi = (uint32_t)(vb0 >> 32);
    uint32_t m1lo = (uint32_t)vb1, m1hi = (uint32_t)(vb1 >> 32);
    const uint32_t nd0 = ~d0, nd1 = ~d1;
    for (int bit = 0; bit < f.w; ++bit) {
      const uint32_t c0 = (uint32_t)(((int32_t)(nd0 << (31 - bit))) >> 31);  // ~0 where the bit is 0
      const uint32_t c1 = (uint32_t)(((int32_t)(nd1 << (31 - bit))) >> 31);
      const uint64_t b0 = __ballot(c0 == 0u), b1 = __ballot(c1 == 0u);
      m0lo &= (uint32_t)b0 ^ c0;
      m0hi &= (uint32_t)(b0 >> 32) ^ c0;
      m1lo &= (uint32_t)b1 ^ c1;
      m1hi &= (uint32_t)(b1 >> 32) ^ c1;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint32_t mlo = q ? m1lo : m0lo, mhi = q ? m1hi : m0hi, d = q ? d1 : d0;
      const bool valid = q ? v1 : v0;
      const uint32_t below = __builtin_amdgcn_mbcnt_hi(mhi, __builtin_amdgcn_mbcnt_lo(mlo, 0u));
      uint32_t pre = 0;
      if (valid && below == 0)
        pre = atomicAdd(&S.wcnt[w][d], (uint32_t)(__popc(mlo) + __popc(mhi)));
      // lowest lane of the group, and this lane's place after it
      const uint32_t lead =
          mlo ? (uint32_t)__builtin_ctz(mlo) : 32u + (uint32_t)__builtin_ctz(mhi | 0x80000000u);
      rank[it + q] = pre;
      dg[it + q] = d | (lead << 16) | (below << 24);
    }
  }
#pragma unroll
  for (int it = 0; it < C::SI; ++it) {
    const uint32_t lead = (dg[it] >> 16) & 0xffu;
    rank[it] = (uint32_t)__shfl((int)rank[it], (int)lead) + (dg[it] >> 24);
    dg[it] &= 0xffffu;
  }
  __syncthreads();

  // per digit: offsets of the waves, tile count
  uint32_t tcnt = 0;
  if ((int)threadIdx.x < Rb) {
    const int d = threadIdx.x;
    for (int i = 0; i < C::NW; ++i) {
      const uint32_t v = S.wcnt[i][d];
      S.wcnt[i][d] = tcnt;
      tcnt += v;
    }
  }
  // the digit's place among this tile's items, and among the frame's items of
  // this pass (from the frame's digit counts)
  uint32_t tex, dex, tile_total, frame_total;
  block_excl_scan2<C::BLOCK>(tcnt, hv, S.wsum, tex, dex, tile_total, frame_total);
  if ((int)threadIdx.x < Rb) {
    // S.wcnt[w][d] becomes the tile place of wave w's first item of digit d
    const int d = threadIdx.x;
    for (int i = 0; i < C::NW; ++i) S.wcnt[i][d] += tex;
  }
  const int t_mine = t;
  // publish this tile's digit counts before anything else
  if ((int)threadIdx.x < Rb)
    st_rlx(ws.sdesc + ((size_t)p * ws.capNTs + t_mine) * C::R + threadIdx.x,
           (j == 0 ? kFlagP32 : kFlagA32) | tcnt);
  __syncthreads();

  // stage the tile in LDS in digit order
  {
    uint32_t lp[C::SI];
#pragma unroll
    for (int it = 0; it < C::SI; ++it) lp[it] = S.wcnt[w][dg[it]] + rank[it];
    if (f.wide) {
#pragma unroll
      for (int it = 0; it < C::SI; ++it)
        if ((vm >> it) & 1u) {
          S.lo[lp[it]] = klo[it];
          S.hi[lp[it]] = khi[it];
          S.idx[lp[it]] = kid[it];
        }
    } else {
#pragma unroll
      for (int it = 0; it < C::SI; ++it)
        if ((vm >> it) & 1u) {
          S.lo[lp[it]] = klo[it];
          S.idx[lp[it]] = kid[it];
        }
    }
  }

  // decoupled look-back over the frame's earlier tiles of this pass; gbase[d]
  // becomes the global place of digit d's run minus its place in the tile
  if ((int)threadIdx.x < Rb) {
    const int d = threadIdx.x;
    uint32_t excl = 0;
    if (j > 0) {
      uint32_t* mine = ws.sdesc + ((size_t)p * ws.capNTs + t_mine) * C::R + d;
      excl = look_back32(ws.sdesc + (size_t)p * ws.capNTs * C::R + d, C::R, t_mine - 1, fd.ts0,
                         ws.ctl);
      st_rlx(mine, kFlagP32 | ((excl + tcnt) & kVal32));
    }
    S.gbase[d] = dex + excl - tex;
  }
  __syncthreads();

  // write runs of equal digits to their global places
  const int dst = (p + 1) & 1;
  uint32_t* dlo = ws.lo[dst] + fd.off;
  uint32_t* dhi = ws.hi[dst] + fd.off;
  uint32_t* did = ws.idx[dst] + fd.off;
  const uint32_t nlim = (uint32_t)fd.n;
  if (f.wide) {
    uint32_t lo[C::SI], hi[C::SI], id[C::SI], gp[C::SI];
#pragma unroll
    for (int k = 0; k < C::SI; ++k) {
      const uint32_t i = threadIdx.x + k * C::BLOCK;
      lo[k] = S.lo[i];
      hi[k] = S.hi[i];
      id[k] = S.idx[i];
    }
#pragma unroll
    for (int k = 0; k < C::SI; ++k)
      gp[k] = S.gbase[digit_of(lo[k], hi[k], shift, mask)] + threadIdx.x + k * C::BLOCK;
#pragma unroll
    for (int k = 0; k < C::SI; ++k)
      if (threadIdx.x + k * C::BLOCK < tile_total && gp[k] < nlim) {
        dlo[gp[k]] = lo[k];
        dhi[gp[k]] = hi[k];
        did[gp[k]] = id[k];
      }
  } else {
    uint32_t lo[C::SI], id[C::SI], gp[C::SI];
#pragma unroll
    for (int k = 0; k < C::SI; ++k) {
      const uint32_t i = threadIdx.x + k * C::BLOCK;
      lo[k] = S.lo[i];
      id[k] = S.idx[i];
    }
#pragma unroll
    for (int k = 0; k < C::SI; ++k)
      gp[k] = S.gbase[(lo[k] >> shift) & mask] + threadIdx.x + k * C::BLOCK;
#pragma unroll
    for (int k = 0; k < C::SI; ++k)
      if (threadIdx.x + k * C::BLOCK < tile_total && gp[k] < nlim) {
        dlo[gp[k]] = lo[k];
        did[gp[k]] = id[k];
      }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (persistent) fence_rel();
    atomicAdd(&ws.fs[b].pass_done[p], 1u);
  }
}

// ------------------------------------------------------------ RED tile ----
struct CellOut {
  uint32_t lo, hi, ref;
  float r[3];
};

__device__ __forceinline__ void corner_of(const FrameParams& f, const float p[3], float r[3]) {
  for (int a = 0; a < 3; ++a)
    r[a] = __fadd_rn(f.mn[a], __fmul_rn((float)cell_coord(p[a], f.mn[a], f.inv), f.leaf));
}

// Cell corner from a cell key (the inverse of point_key), so that a segment's
// corner is known without reading one of its points back.
__device__ __forceinline__ void corner_of_key(const FrameParams& f, int key_mode, uint32_t lo,
                                              uint32_t hi, float r[3]) {
  uint32_t k[3];
  if (key_mode == 1) {
    const uint64_t key = ((uint64_t)hi << 32) | lo;
    k[0] = compact3(key);
    k[1] = compact3(key >> 1);
    k[2] = compact3(key >> 2);
  } else if (!f.wide) {
    const uint32_t q = lo / f.d[0];
    k[0] = lo - q * f.d[0];
    k[2] = q / f.d[1];
    k[1] = q - k[2] * f.d[1];
  } else {
    const uint64_t key = ((uint64_t)hi << 32) | lo;
    const uint64_t q = key / f.d[0];
    k[0] = (uint32_t)(key - q * f.d[0]);
    k[2] = (uint32_t)(q / f.d[1]);
    k[1] = (uint32_t)(q - (uint64_t)k[2] * f.d[1]);
  }
  for (int a = 0; a < 3; ++a) r[a] = __fadd_rn(f.mn[a], __fmul_rn((float)k[a], f.leaf));
}

// Writes one output row from a segment's sums.
__device__ __forceinline__ void finalize_row(const GIo& io, uint32_t want, int64_t row, int64_t N,
                                             const Acc& a, const uint64_t* rgb_wide,
                                             const CellOut& c) {
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
    const float px = io.vx[c.ref], py = io.vy[c.ref], pz = io.vz[c.ref];
    io.lx[row] = __fadd_rn(__fsub_rn(c.r[0], px), mean[0]);
    io.ly[row] = __fadd_rn(__fsub_rn(c.r[1], py), mean[1]);
    io.lz[row] = __fadd_rn(__fsub_rn(c.r[2], pz), mean[2]);
  }
  if (want & kOutRGB) {
    for (int i = 0; i < 3; ++i) {
      const uint64_t s = rgb_wide ? rgb_wide[i] : rgb_channel(a.rgb, i);
      io.crgb[3 * row + i] = (uint8_t)((s + a.n / 2) / a.n);
    }
  }
  if (want & kOutCount) io.count[row] = a.n;
  if (want & kOutKey) io.key[row] = ((uint64_t)c.hi << 32) | c.lo;
  if (want & kOutRef) io.ref_index[row] = c.ref;
}

__device__ __forceinline__ void write_pend(const Ws& ws, int t, int b, int j, const Acc& a,
                                           const CellOut& c, int64_t row) {
  Pend pd;
  pd.valid = 1u;
  pd.b = (uint32_t)b;
  pd.j = (uint32_t)j;
  pd.lo = c.lo;
  pd.hi = c.hi;
  for (int q = 0; q < 3; ++q) {
    pd.r[q] = c.r[q];
    pd.s[q] = a.s[q];
    pd.c[q] = a.c[q];
  }
  pd.row = row;
  pd.n = a.n;
  pd.pad = 0;
  pd.rgb = a.rgb;
  ws.pend[t] = pd;
}

// Fix-up of one reduce tile by one wave: a cell that began in an earlier tile
// gets the carry-out parts of the tiles it covers, summed in a fixed order.
template <class C>
__device__ void fix_tile(const Ws& ws, const GIo& io, int t, int key_mode, uint32_t want,
                         int64_t N, const BlockCtl& bc) {
  const int lane = threadIdx.x & 63;
  const Pend pd = ws.pend[t];
  if (!pd.valid) return;
  const int b = (int)pd.b, j = (int)pd.j;
  // one-phase launches hold every frame's descriptors in LDS
  const FrameDesc fd = bc.cached ? bc.fda[b] : ws.fd[b];
  // where the cell starts: at the last head of the nearest earlier tile that
  // has one (the tiles in between hold only points of this cell, and their
  // carry-outs say so); the wave reads 64 earlier carry-outs at a time
  uint32_t start = 0, ref = 0;
  for (int k0 = t - 1;; k0 -= 64) {
    const int k = k0 - lane;
    uint32_t hp = kNoHead, rf = 0;
    if (k >= fd.tr0) {
      hp = ws.frag[k].head_pos;
      rf = ws.frag[k].ref;
    }
    const uint64_t found = __ballot(hp != kNoHead);
    if (found) {
      const int src = __ffsll((unsigned long long)found) - 1;
      start = __shfl(hp, src);
      ref = __shfl(rf, src);
      break;
    }
    if (k0 - 64 < fd.tr0) {  // the frame's first tile always holds a head
      if (lane == 0) atomicOr(&ws.ctl->error, 1u);
      return;
    }
  }
  const int th = (int)(start / (uint32_t)C::TR);
  const int nf = j - th;
  const int tbase = fd.tr0 + th;
  Acc part;
  acc_zero(part);
  uint64_t rgb3[3] = {0ull, 0ull, 0ull};
  for (int k = lane; k < nf; k += 64) {
    const Frag fr = ws.frag[tbase + k];
    Acc a;
    a.n = fr.n;
    for (int q = 0; q < 3; ++q) {
      a.s[q] = fr.s[q];
      a.c[q] = fr.c[q];
    }
    a.rgb = 0ull;
    acc_merge(part, a);
#pragma unroll
    for (int q = 0; q < 3; ++q) rgb3[q] += rgb_channel(fr.rgb, q);
  }
  // butterfly over the wave; partners combine lower lane first, so both hold
  // the same sums
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    Acc o;
    o.n = __shfl_xor(part.n, off);
    for (int q = 0; q < 3; ++q) {
      o.s[q] = __shfl_xor(part.s[q], off);
      o.c[q] = __shfl_xor(part.c[q], off);
    }
    o.rgb = 0ull;
    uint64_t orgb[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      orgb[q] = ((uint64_t)__shfl_xor((uint32_t)(rgb3[q] >> 32), off) << 32) |
                (uint32_t)__shfl_xor((uint32_t)rgb3[q], off);
    }
    if (lane & off) {
      acc_merge(o, part);
      part = o;
    } else {
      acc_merge(part, o);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) rgb3[q] += orgb[q];
  }
  if (lane == 0) {
    Acc in_tile;
    in_tile.n = pd.n;
    for (int q = 0; q < 3; ++q) {
      in_tile.s[q] = pd.s[q];
      in_tile.c[q] = pd.c[q];
    }
    in_tile.rgb = 0ull;
    acc_merge(part, in_tile);
    uint64_t rgbw[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) rgbw[q] = rgb3[q] + rgb_channel(pd.rgb, q);
    CellOut c;
    c.lo = pd.lo;
    c.hi = pd.hi;
    c.ref = ref;
    for (int q = 0; q < 3; ++q) c.r[q] = pd.r[q];
    finalize_row(io, want, pd.row, N, part, rgbw, c);
  }
}

// Key, first index and corner of the cell whose first point is item `li` of
// the tile (keys and indices are in LDS; the corner is decoded from the key).
template <class C>
__device__ __forceinline__ CellOut cell_at(const typename C::RedSmem& S, const FrameParams& f,
                                           int key_mode, int li) {
  CellOut c;
  c.lo = S.klo[li];
  c.hi = f.wide ? S.khi[li] : 0u;
  c.ref = S.kid[li];
  corner_of_key(f, key_mode, c.lo, c.hi, c.r);
  return c;
}

// Reduce tiles of a frame past its valid points (all but its first tile) are
// skipped at dequeue.  The frame's last tile that is not skipped publishes
// their inclusive prefix, which is its own, so the look-back of later tiles
// passes through them, and writes the total rows if the frame is the last.
template <class C>
__device__ __forceinline__ void publish_skipped(const Ws& ws, const GIo& io, const FrameDesc& fd,
                                                int j, int64_t nv, int b, int B, uint64_t incl) {
  const int jl = nv > 0 ? (int)((nv - 1) / C::TR) : 0;
  if (j != jl) return;
  for (int k = jl + 1; k < fd.ntr; ++k) st_rlx64(&ws.rdesc[fd.tr0 + k], kFlagP64 | incl);
  if (b == B - 1) io.out_offsets[B] = (int64_t)incl;
}

template <class C>
__device__ void red_tile(const Ws& ws, const GIo& io, typename C::RedSmem& S, const FrameDesc& fd,
                         int b, int j, const FrameParams& f, int key_mode, uint32_t want, int B,
                         int NTr, int64_t N, bool persistent, int dt, int dlast, bool compact) {
  constexpr int K = C::RI;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int t = fd.tr0 + j;
  const int64_t nv = (f.status == kFrameOk) ? (int64_t)f.n_valid : 0;
  const int64_t s0 = (int64_t)j * C::TR;
  const int64_t e0 = min(s0 + (int64_t)C::TR, nv);
  const int cnt = e0 > s0 ? (int)(e0 - s0) : 0;
  const int fb = f.passes & 1;
  const uint32_t* klo = ws.lo[fb] + fd.off;
  const uint32_t* khi = ws.hi[fb] + fd.off;
  const uint32_t* kid = ws.idx[fb] + fd.off;
  const int base = threadIdx.x * K;
  const uint32_t Nm1 = (uint32_t)(N - 1);
  if (cnt == 0) {
    // past the frame's valid points: only the row count chain goes on
    if (threadIdx.x < 64) {
      uint64_t excl = 0;
      if (dt > 0) {
        if (threadIdx.x == 0) st_rlx64(&ws.rdesc[dt], kFlagA64);
        excl = look_back64_wave(ws.rdesc, dt - 1, ws.ctl);
      }
      if (threadIdx.x == 0) {
        st_rlx64(&ws.rdesc[dt], kFlagP64 | excl);
        if (j == 0) {
          io.out_offsets[b] = (int64_t)excl;
          io.frame_status[b] = ld_rlx(&ws.ctl->error) ? kFrameDeviceError : f.status;
        }
        if (dt == dlast) io.out_offsets[B] = (int64_t)excl;
        if (!compact) publish_skipped<C>(ws, io, fd, j, nv, b, B, excl);
      }
    }
    return;
  }

  // ---- keys and indices straight into LDS (global-to-LDS loads: lane l of
  // a wave fills word l of the wave's 64-word slot, no registers held); each
  // thread then owns items i*K .. i*K+K-1 of the tile (blocked) and gathers
  // their points into registers.  Addresses are clamped into the tile, so the
  // slots past its items hold copies of the last one.
  {
    const int64_t lastp = e0 - 1;
    const int wo = w * 64;
#pragma unroll
    for (int u = 0; u < K; ++u) {
      const int64_t pos = min(s0 + u * C::BLOCK + (int)threadIdx.x, lastp);
      lds_load_word(klo + pos, &S.klo[u * C::BLOCK + wo]);
      lds_load_word(kid + pos, &S.kid[u * C::BLOCK + wo]);
    }
    if (f.wide) {
#pragma unroll
      for (int u = 0; u < K; ++u)
        lds_load_word(khi + min(s0 + u * C::BLOCK + (int)threadIdx.x, lastp),
                      &S.khi[u * C::BLOCK + wo]);
    }
  }
  if (threadIdx.x == 0) {
    // the keys just before and just after the tile
    const int64_t ip = s0 > 0 ? s0 - 1 : s0;
    const int64_t in = e0 < nv ? e0 : e0 - 1;
    const uint32_t plo = klo[ip], phi = khi[ip], nlo = klo[in], nhi = khi[in];
    S.has_prev = s0 > 0 ? 1u : 0u;
    S.prev_lo = s0 > 0 ? plo : 0u;
    S.prev_hi = (s0 > 0 && f.wide) ? phi : 0u;
    S.has_next = e0 < nv ? 1u : 0u;
    S.next_lo = e0 < nv ? nlo : 0u;
    S.next_hi = (e0 < nv && f.wide) ? nhi : 0u;
  }
  lds_load_wait();
  __syncthreads();
  // ---- head flags: an item starts a cell when its key differs from the previous one
  uint32_t vmask = 0, hmask = 0;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const int li = base + i;
    if (li < cnt) {
      vmask |= 1u << i;
      bool head;
      if (li == 0) {
        head = !S.has_prev || S.klo[0] != S.prev_lo || (f.wide && S.khi[0] != S.prev_hi);
      } else {
        head = S.klo[li] != S.klo[li - 1] || (f.wide && S.khi[li] != S.khi[li - 1]);
      }
      if (head) hmask |= 1u << i;
    }
  }
  uint32_t H;
  const uint32_t hb = block_excl_scan<C::BLOCK>((uint32_t)__popc(hmask), S.wsum, H);
  {
    uint32_t r = hb;
#pragma unroll
    for (int i = 0; i < K; ++i)
      if ((hmask >> i) & 1u) S.hpos[r++] = (uint16_t)(base + i);
  }

  // ---- publish the tile's head count at once
  if (threadIdx.x == 0) st_rlx64(&ws.rdesc[dt], (dt == 0 ? kFlagP64 : kFlagA64) | H);

  // ---- gather the thread's points; they arrive during the look-back
  float px[K], py[K], pz[K];
  uint32_t c24[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const uint32_t id = min(S.kid[min(base + i, cnt - 1)], Nm1);
    const float4 r4 = ws.rec[id];
    px[i] = r4.x;
    py[i] = r4.y;
    pz[i] = r4.z;
    c24[i] = __float_as_uint(r4.w);
  }

  // ---- look-back over head counts: dense rows across frames
  if (threadIdx.x < 64) {
    uint64_t excl = 0;
    if (dt > 0) excl = look_back64_wave(ws.rdesc, dt - 1, ws.ctl);
    if (threadIdx.x == 0) {
      if (dt > 0) st_rlx64(&ws.rdesc[dt], kFlagP64 | (excl + H));
      S.excl = excl;
      if (j == 0) {
        io.out_offsets[b] = (int64_t)excl;
        io.frame_status[b] = ld_rlx(&ws.ctl->error) ? kFrameDeviceError : f.status;
      }
      if (dt == dlast) io.out_offsets[B] = (int64_t)(excl + H);
      if (!compact) publish_skipped<C>(ws, io, fd, j, nv, b, B, excl + H);
    }
  }
  __syncthreads();
  const int64_t excl_t = (int64_t)S.excl;

  // ---- one pass over the thread's items: the open ends (sums before its
  // first head, and from its last head on) and every cell that opens and
  // closes inside the thread, written at once; the row of each point
  Acc pre, cur;
  acc_zero(pre);
  acc_zero(cur);
  uint32_t lh = 0;  // heads seen
#pragma unroll
  for (int i = 0; i < K; ++i) {
    if (!((vmask >> i) & 1u)) continue;
    if ((hmask >> i) & 1u) {
      if (lh == 0) pre = cur;
      else
        finalize_row(io, want, excl_t + hb + lh - 1, N, cur, nullptr,
                     cell_at<C>(S, f, key_mode, S.hpos[hb + lh - 1]));
      acc_zero(cur);
      ++lh;
    }
    const float p[3] = {px[i], py[i], pz[i]};
    float r[3], dv[3];
    corner_of(f, p, r);
    for (int a = 0; a < 3; ++a) dv[a] = __fsub_rn(p[a], r[a]);
    acc_add(cur, dv, c24[i]);
    if (want & kOutPointCell)
      io.point_cell[min(S.kid[base + i], Nm1)] = (int32_t)(excl_t + hb + lh - 1);
  }
  const bool seen_head = lh > 0;
  if (!seen_head) pre = cur;

  // ---- block segmented scan of the threads' open ends
  Seg mine;
  mine.f = seen_head ? 1u : 0u;
  mine.a = seen_head ? cur : pre;
  const Seg incl = wave_incl_seg(mine);
  if (lane == 63) S.wtot[w] = incl;
  __syncthreads();
  Seg wp;
  wp.f = 0;
  acc_zero(wp.a);
  for (int i = 0; i < w; ++i) wp = seg_combine(wp, S.wtot[i]);
  Seg ex = seg_dpp<0x138, 0xf, true>(incl);  // the lane below's inclusive value
  ex = seg_combine(wp, ex);

  // (i) the cell open at this thread's start closes at its first head
  if (seen_head) {
    Acc tot = ex.a;
    acc_merge(tot, pre);
    if (tot.n > 0) {
      if (ex.f) {
        // its first point is the last head before this thread
        finalize_row(io, want, excl_t + hb - 1, N, tot, nullptr,
                     cell_at<C>(S, f, key_mode, S.hpos[hb - 1]));
      } else {
        // opened in an earlier tile (the tile's first item is one of its
        // points): the fix-up phase adds the earlier parts
        write_pend(ws, t, b, j, tot, cell_at<C>(S, f, key_mode, 0), excl_t - 1);
      }
    }
  }
  // (ii) the thread holding the tile's last item closes or hands on the last cell
  if (base < cnt && base + K >= cnt) {
    const Seg last = seg_combine(ex, mine);
    const int ll = cnt - 1;
    const bool cont = S.has_next && S.next_lo == S.klo[ll] && (!f.wide || S.next_hi == S.khi[ll]);
    if (cont) {
      Frag fr;
      fr.n = last.a.n;
      for (int a = 0; a < 3; ++a) {
        fr.s[a] = last.a.s[a];
        fr.c[a] = last.a.c[a];
      }
      const int hl = last.f ? (int)S.hpos[H - 1] : 0;
      fr.head_pos = last.f ? (uint32_t)(s0 + hl) : kNoHead;
      fr.ref = last.f ? S.kid[hl] : 0u;
      fr.pad = 0;
      fr.rgb = last.a.rgb;
      ws.frag[t] = fr;
      if (persistent) {  // one-phase launches hand the parts on at the kernel boundary
        fence_rel();
        st_rlx(&ws.fflag[t], 1u);
      }
    } else if (last.f) {
      finalize_row(io, want, excl_t + (int64_t)H - 1, N, last.a, nullptr,
                   cell_at<C>(S, f, key_mode, S.hpos[H - 1]));
    } else {
      write_pend(ws, t, b, j, last.a, cell_at<C>(S, f, key_mode, 0), excl_t - 1);
    }
  }
}

// ---------------------------------------------------------- pipeline ----
// Thread 0 of a workgroup: take the next item (a queue ticket, or with `stat`
// item blockIdx.x + k * gridDim.x on the k-th call), find its frame, wait for
// its inputs (once per frame and phase), prepare the frame's grid parameters.
// A launch of several radix passes (`multi`, not `persistent`) numbers its
// items pass after pass; a tile of pass p waits for pass p - 1 of its frame.
// Largest k in [0, n) with a[k] <= v, for a non-decreasing LDS table with
// a[0] <= v and n <= 4096: each lane of the wave probes one entry of a coarse
// grid, then one entry of the chosen interval; a ballot finds the last entry
// that is <= v at each level.  Every wave gets the same answer.
__device__ __forceinline__ int wave_search(const uint32_t* a, int n, uint32_t v) {
  const int lane = threadIdx.x & 63;
  const int step = (n + 63) >> 6;
  const int i1 = lane * step;
  const uint64_t m1 = __ballot(i1 < n && a[i1] <= v);
  int k = (63 - __clzll((long long)m1)) * step;
  if (step > 1) {
    const int i2 = k + lane;
    const uint64_t m2 = __ballot(lane < step && i2 < n && a[i2] <= v);
    k += 63 - __clzll((long long)m2);
  }
  return k;
}

template <class C>
__device__ __forceinline__ void next_item(const Ws& ws, const CallHdr& hdr, BlockCtl& bc,
                                       uint32_t* counter, bool persistent, bool multi, int ph_lo,
                                       uint32_t total, bool stat, uint32_t& sitem) {
  for (;;) {
    uint32_t item;
    if (stat) {  // tiles that wait on no tile: a fixed order
      item = sitem;
      sitem += gridDim.x;
    } else {
      item = atomicAdd(counter, 1u);
    }
    bc.item = item;
    bc.skip = 0;
    if (item >= total) return;
    int ph, t;
    uint32_t base;
    const uint32_t nb = (uint32_t)hdr.NTb, ns = (uint32_t)hdr.NTs;
    if (persistent) {
      if (item < nb) { ph = C::PH_BBOX; base = 0; }
      else if (item < 2 * nb) { ph = C::PH_HIST; base = nb; }
      else if (item < 2 * nb + C::MAXP * ns) {
        ph = C::PH_SORT0 + (int)((item - 2 * nb) / ns);
        base = 2 * nb + (uint32_t)(ph - C::PH_SORT0) * ns;
      } else if (item < 2 * nb + C::MAXP * ns + (uint32_t)hdr.NTr) {
        ph = C::PH_RED;
        base = 2 * nb + C::MAXP * ns;
      } else {
        ph = C::PH_FIX;
        base = 2 * nb + C::MAXP * ns + (uint32_t)hdr.NTr;
      }
    } else if (multi) {
      ph = ph_lo + (int)(item / ns);
      base = (uint32_t)(ph - ph_lo) * ns;
    } else {
      ph = ph_lo;
      base = 0;
    }
    t = (int)(item - base);
    if (ph == C::PH_FIX) {
      // fix-ups read the carry-out parts and pending cells of every reduce tile
      bc.ph = ph;
      bc.t = t;
      bc.b = 0;
      bc.j = 0;
      if (persistent && bc.dep_b[ph] != 0) {
        wait_geq(&ws.ctl->red_tiles_done, (uint32_t)hdr.NTr, ws.ctl);
        fence_acq();
        bc.dep_b[ph] = 0;
      }
      return;
    }
    const uint32_t tiling = ph <= C::PH_HIST ? 0u : (ph == C::PH_RED ? 2u : 1u);
    int b, j;
    if (tiling == 1 && bc.ilv_rounds > 0) {
      int lo = 0, hi = bc.ilv_rounds;  // largest round r with ilv_s[r] <= t
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int)bc.ilv_s[mid] <= t) lo = mid;
        else hi = mid;
      }
      b = (int)bc.ilv_perm[t - (int)bc.ilv_s[lo]];
      j = lo;
    } else if (hdr.B <= kLdsFrames) {
      const uint32_t* tp = bc.tp[tiling];
      int lo = 0, hi = hdr.B;  // largest b with tp[b] <= t
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int)tp[mid] <= t) lo = mid;
        else hi = mid;
      }
      b = lo;
      j = t - (int)tp[lo];
    } else {
      const uint32_t toff = tiling == 0 ? 0u : (tiling == 1 ? nb : nb + ns);
      const uint2 ti = ws.tinfo[toff + t];
      b = (int)ti.x;
      j = (int)ti.y;
    }
    if (bc.cached) {
      bc.fd = bc.fda[b];
      bc.fp = bc.fpa[b];
      bc.fd_b = bc.fp_b = b;
    } else if (bc.fd_b != b) {
      bc.fd = ws.fd[b];
      bc.fd_b = b;
    }
    bc.ph = ph;
    bc.t = t;
    bc.b = b;
    bc.j = j;
    if (ph == C::PH_BBOX) return;
    const FrameDesc& fd = bc.fd;
    // grid parameters need the frame's bounding box
    if (bc.fp_b != b) {
      if (persistent) {
        wait_geq(&ws.fs[b].bbox_done, (uint32_t)fd.ntb, ws.ctl);
        fence_acq();
      }
      bc.fp = frame_params(ws, b, hdr.key_mode, C::W);
      bc.fp_b = b;
    }
    const FrameParams& f = bc.fp;
    if (ph == C::PH_HIST) return;
    if (ph < C::PH_RED) {
      const int p = ph - C::PH_SORT0;
      if (p >= f.passes) {
        // no work for this frame in this pass: jump the queue past it, or past
        // every remaining pass once no frame needs this one
        // (in round-robin order a frame's tiles are not contiguous: skip one)
        uint32_t jump = bc.ilv_rounds > 0 ? 0u : base + (uint32_t)(fd.ts0 + fd.nts);
        const bool all_hist = wait_geq(&ws.ctl->hist_tiles_done, (uint32_t)hdr.NTb, ws.ctl);
        if (multi) fence_acq();
        if (all_hist && (uint32_t)p >= ld_rlx(&ws.ctl->max_passes))
          jump = persistent ? 2 * nb + C::MAXP * ns : total;
        if (jump) atomicMax(counter, jump);
        continue;
      }
      if (bc.dep_b[ph] != b) {
        if (multi) {
          wait_geq(&ws.fs[b].hist_done, (uint32_t)fd.ntb, ws.ctl);
          if (p > 0) wait_geq(&ws.fs[b].pass_done[p - 1], (uint32_t)fd.nts, ws.ctl);
          fence_acq();
        }
        bc.dep_b[ph] = b;
      }
      return;
    }
    if (ph == C::PH_RED) {
      // past the frame's valid points: skip the frame's remaining tiles (their
      // row prefix comes from the frame's last tile with points)
      const int64_t nv = f.status == kFrameOk ? (int64_t)f.n_valid : 0;
      if (j > 0 && (int64_t)j * C::TR >= nv) {
        atomicMax(counter, base + (uint32_t)(fd.tr0 + fd.ntr));
        continue;
      }
    }
    // reduce: the frame's last radix pass must be complete
    if (bc.dep_b[ph] != b) {
      if (persistent && f.passes > 0 && f.status == kFrameOk) {
        wait_geq(&ws.fs[b].hist_done, (uint32_t)fd.ntb, ws.ctl);
        wait_geq(&ws.fs[b].pass_done[f.passes - 1], (uint32_t)fd.nts, ws.ctl);
        fence_acq();
      }
      bc.dep_b[ph] = b;
    }
    return;
  }
}

// Kernel entry points.  KIND selects which phases a kernel holds: all of them
// (one persistent launch over the whole queue) or one phase kind (one launch
// per phase).  Every kind runs the same tile code; a kernel that holds one
// kind only is compiled with that kind's register and LDS needs.

// Waves per SIMD a kernel must fit: a 512-thread radix or reduce workgroup is
// 2 waves per SIMD, so two of them per CU need 128 VGPRs or fewer.
template <class C, int KIND>
constexpr int kMinWaves = ((KIND == 3 || KIND == 4) && C::BLOCK == 512) ? 4 : 1;

template <class C, int KIND>
__global__ __launch_bounds__(C::BLOCK, (kMinWaves<C, KIND>)) void vg_pipeline_kernel(Ws ws, int ph_lo, int ph_hi) {
  __shared__ typename SmemOf<C, KIND>::type sm;
  __shared__ BlockCtl bc;
  // after a device-side time-out (raised by an earlier launch of the call)
  // nothing more runs: inputs of later phases may be incomplete
  if (ld_rlx(&ws.ctl->error) != 0) return;
  const CallHdr hdr = *ws.hdr;
  const GIo io = global_view(*ws.io);
  const bool persistent = (ph_lo == 0 && ph_hi == C::NPH);
  // a launch of several radix passes holds only the passes some frame needs
  // (the histogram launch before it has set max_passes): when that is one
  // pass, it runs as a one-pass launch, with its own tile order and the fast
  // dispatch
  if (!persistent && ph_lo >= C::PH_SORT0 && ph_hi <= C::PH_RED && ph_hi - ph_lo > 1)
    ph_hi = max(ph_lo + 1, min(ph_hi, C::PH_SORT0 + (int)ld_rlx(&ws.ctl->max_passes)));
  const bool multi = ph_hi - ph_lo > 1;  // several phases: tiles wait on earlier phases
  // a launch of radix passes that no frame needs ends at once (the histogram
  // launch before it has set max_passes)
  if (!persistent && ph_lo >= C::PH_SORT0 && ph_lo < C::PH_RED &&
      (uint32_t)(ph_lo - C::PH_SORT0) >= ld_rlx(&ws.ctl->max_passes))
    return;
  uint32_t* counter = persistent ? &ws.ctl->queue[0] : &ws.ctl->queue[1 + ph_lo];
  uint32_t total;
  const uint32_t nfix = (uint32_t)((hdr.NTr + C::NW - 1) / C::NW);
  if (persistent) total = (uint32_t)(2 * hdr.NTb + C::MAXP * hdr.NTs + hdr.NTr) + nfix;
  else if (ph_lo <= C::PH_HIST) total = (uint32_t)hdr.NTb;
  else if (ph_lo == C::PH_RED) total = (uint32_t)hdr.NTr;
  else if (ph_lo == C::PH_FIX) total = nfix;
  else total = (uint32_t)(ph_hi - ph_lo) * (uint32_t)hdr.NTs;
  if (hdr.B <= kLdsFrames) {
    for (int i = threadIdx.x; i <= hdr.B; i += C::BLOCK) {
      bc.tp[0][i] = ws.tpb[i];
      bc.tp[1][i] = ws.tps[i];
      bc.tp[2][i] = ws.tpr[i];
    }
  }
  if (hdr.ilv_rounds > 0) {
    for (int i = threadIdx.x; i <= hdr.ilv_rounds; i += C::BLOCK) bc.ilv_s[i] = ws.ilv_s[i];
    for (int i = threadIdx.x; i < hdr.B; i += C::BLOCK) bc.ilv_perm[i] = ws.ilv_perm[i];
  }
  // a one-phase launch keeps the frame descriptors in LDS, and after the bbox
  // pass every frame's grid too (it is final by then)
  const bool cache_fd = !persistent && hdr.B <= kFpCache;
  const bool cache = cache_fd && ph_lo != C::PH_BBOX;
  if (cache_fd) {
    for (int i = threadIdx.x; i < hdr.B; i += C::BLOCK) {
      bc.fda[i] = ws.fd[i];
      if (cache) bc.fpa[i] = frame_params(ws, i, hdr.key_mode, C::W);
    }
  }
  if (threadIdx.x == 0) {
    bc.cached = cache ? 1 : 0;
    bc.ilv_rounds = hdr.ilv_rounds;
  }
  if constexpr (KIND == kRed) {
    // A one-phase reduce launch skips the tiles past each frame's valid points,
    // so its row-count chain runs over the other tiles only: frame b's tiles
    // hold descriptors vt0[b] .. vt0[b+1]-1 (at least one per frame).
    if (cache) {
      __syncthreads();
      uint32_t nvt = 0;
      if ((int)threadIdx.x < hdr.B) {
        const FrameParams& fp = bc.fpa[threadIdx.x];
        const int64_t nv = fp.status == kFrameOk ? (int64_t)fp.n_valid : 0;
        nvt = nv > 0 ? (uint32_t)((nv + C::TR - 1) / C::TR) : 1u;
      }
      uint32_t tot;
      const uint32_t ex = block_excl_scan<C::BLOCK>(nvt, bc.scan_w, tot);
      if ((int)threadIdx.x < hdr.B) bc.vt0[threadIdx.x] = ex;
      if (threadIdx.x == 0) bc.vt0[hdr.B] = tot;
    }
  }
  // a one-pass radix launch with every frame's grid at hand orders its tiles
  // round-robin over just the frames that need this pass
  const bool own_order = cache && !multi && ph_lo >= C::PH_SORT0 && ph_lo < C::PH_RED &&
                         hdr.ilv_rounds > 0 && hdr.B <= kIlvMaxFrames;
  if (own_order) {
    // the frames that need this pass, by descending count of tiles to run
    // (after the first pass, tiles past a frame's valid points have nothing
    // to do and are left out), ties in the host order; then the frames of
    // every round.  Scratch: tp[0] counts in host order, tp[1] the frames and
    // tp[2] the counts in the new order (one-pass radix launches use neither
    // tile prefix table).
    __syncthreads();
    const int p = ph_lo - C::PH_SORT0;
    const int i = threadIdx.x;
    uint32_t my = 0;
    uint32_t fr = 0;
    if (i < hdr.B) {
      fr = bc.ilv_perm[i];
      const FrameParams& fp = bc.fpa[fr];
      const uint32_t nts = (uint32_t)bc.fda[fr].nts;
      if (fp.passes > p) {
        my = nts;
        if (p > 0) my = min(nts, (uint32_t)((fp.n_valid + C::TS - 1) / C::TS));
      }
      bc.tp[0][i] = my;
    }
    __syncthreads();
    uint32_t nkeep = 0, rank = 0;
    for (int k = 0; k < hdr.B; ++k) {
      const uint32_t o = bc.tp[0][k];
      nkeep += o > 0 ? 1u : 0u;
      rank += (o > my || (o == my && k < i)) ? 1u : 0u;
    }
    if (my > 0) {
      bc.tp[1][rank] = fr;
      bc.tp[2][rank] = my;
      // the tiles left out still count as done, for launches that wait on them
      if (blockIdx.x == 0 && my < (uint32_t)bc.fda[fr].nts)
        atomicAdd(&ws.fs[fr].pass_done[p], (uint32_t)bc.fda[fr].nts - my);
    }
    __syncthreads();
    const int rounds = nkeep ? (int)bc.tp[2][0] : 0;
    // cnt(r) = kept frames with more than r tiles; ilv_s = exclusive prefix of cnt
    constexpr int PER = (kIlvMaxRounds + C::BLOCK - 1) / C::BLOCK;
    uint32_t cnts[PER];
    uint32_t mysum = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int r = i * PER + q;
      uint32_t c = 0;
      if (r < rounds)
        for (uint32_t k = 0; k < nkeep; ++k) c += (bc.tp[2][k] > (uint32_t)r) ? 1u : 0u;
      cnts[q] = c;
      mysum += c;
    }
    uint32_t total_items;
    uint32_t run = block_excl_scan<C::BLOCK>(mysum, bc.scan_w, total_items);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int r = i * PER + q;
      if (r < rounds) bc.ilv_s[r] = run;
      run += cnts[q];
    }
    for (int k = i; k < (int)nkeep; k += C::BLOCK) bc.ilv_perm[k] = bc.tp[1][k];
    if (i == 0) {
      bc.ilv_s[rounds] = total_items;
      bc.ilv_rounds = rounds;
      bc.ilv_total = total_items;
    }
  }
  if (threadIdx.x == 0) {
    bc.fp_b = -1;
    bc.fd_b = -1;
    for (int i = 0; i < kMaxPassSlots + 3; ++i) bc.dep_b[i] = -1;
    // a one-pass launch of a radix pass no frame needs ends at once
    bc.item = 0;
    if (!persistent && ph_lo >= C::PH_SORT0 && ph_lo < C::PH_RED &&
        (uint32_t)(ph_lo - C::PH_SORT0) >= ld_rlx(&ws.ctl->max_passes))
      bc.item = total;
  }
  __syncthreads();
  if (own_order) total = bc.ilv_total;
  if (bc.item >= total && total > 0) return;
  if constexpr (KIND == kBbox || KIND == kHist) {
    if (cache_fd && hdr.N > 0) {
      if (KIND == kBbox && (hdr.filt & kFiltView)) {
        if (io.rgb != nullptr) stream_big_tiles<C, KIND, true, true>(ws, io, hdr, bc, sm);
        else stream_big_tiles<C, KIND, false, true>(ws, io, hdr, bc, sm);
      } else if (KIND == kBbox && io.rgb != nullptr) {
        stream_big_tiles<C, KIND, true>(ws, io, hdr, bc, sm);
      } else {
        stream_big_tiles<C, KIND, false>(ws, io, hdr, bc, sm);
      }
      return;
    }
  }
  // One-phase radix (in their own order), reduce and fix-up launches with
  // every frame's tables in LDS take the fast dispatch: thread 0 only takes
  // the ticket, and every wave decodes it by itself, so a tile starts one
  // barrier after its ticket.  Other launches go through next_item on thread 0.
  const bool fast = cache && !persistent && !multi &&
                    (KIND == kSort ? own_order : (KIND == kRed || KIND == kFix));
  // fix-up tiles only read what the reduce launch wrote: workgroup g takes
  // items g, g + G, ... instead of queue tickets
  const bool stat = !persistent && KIND == kFix;
  uint32_t sitem = blockIdx.x;
  for (;;) {
    if (threadIdx.x == 0) {
      if (fast) {
        uint32_t item;
        if (stat) {
          item = sitem;
          sitem += gridDim.x;
        } else {
          item = atomicAdd(counter, 1u);
        }
        bc.item = item;
      } else {
        next_item<C>(ws, hdr, bc, counter, persistent, multi, ph_lo, total, stat, sitem);
      }
    }
    __syncthreads();
    const uint32_t item = bc.item;
    if (item >= total) break;
    int ph, t, b, j;
    const FrameDesc* fdp;
    const FrameParams* fpp;
    if (fast) {
      ph = ph_lo;
      t = (int)item;
      if (KIND == kSort) {
        j = wave_search(bc.ilv_s, bc.ilv_rounds, item);
        b = (int)bc.ilv_perm[item - bc.ilv_s[j]];
      } else if (KIND == kRed) {
        b = wave_search(bc.tp[2], hdr.B, item);
        j = (int)(item - bc.tp[2][b]);
      } else {
        b = 0;
        j = 0;
      }
      fdp = &bc.fda[b];
      fpp = &bc.fpa[b];
      if (KIND == kRed) {
        const int64_t nv = fpp->status == kFrameOk ? (int64_t)fpp->n_valid : 0;
        if (j > 0 && (int64_t)j * C::TR >= nv) {
          // past the frame's valid points: jump the queue past the frame's
          // remaining tiles (their row prefix comes from its last tile with
          // points)
          if (threadIdx.x == 0) atomicMax(counter, (uint32_t)(fdp->tr0 + fdp->ntr));
          __syncthreads();
          continue;
        }
      }
    } else {
      ph = bc.ph;
      t = bc.t;
      b = bc.b;
      j = bc.j;
      fdp = &bc.fd;
      fpp = &bc.fp;
    }
    const FrameDesc fd = *fdp;
    if (ph == C::PH_BBOX) {
      if constexpr (KIND == kAll || KIND == kBbox)
        bbox_tile<C>(ws, io, sm.bbox, fd, b, j, hdr.want, persistent);
    } else if (ph == C::PH_FIX) {
      if constexpr (KIND == kAll || KIND == kFix) {
        const int tf = t * C::NW + (int)(threadIdx.x >> 6);
        if (tf < hdr.NTr) fix_tile<C>(ws, io, tf, hdr.key_mode, hdr.want, hdr.N, bc);
      }
    } else {
      const FrameParams f = *fpp;
      if (ph == C::PH_HIST) {
        if constexpr (KIND == kAll || KIND == kHist)
          hist_tile<C>(ws, io, sm.hist, fd, b, j, f, hdr.key_mode, hdr.want, persistent);
      } else if (ph < C::PH_RED) {
        if constexpr (KIND == kAll || KIND == kSort)
          sort_tile<C>(ws, io, sm.sort, fd, b, j, ph - C::PH_SORT0, f, hdr.key_mode, multi);
      } else {
        if constexpr (KIND == kAll || KIND == kRed) {
          const int dt = fast ? (int)bc.vt0[b] + j : fd.tr0 + j;
          const int dlast = fast ? (int)bc.vt0[hdr.B] - 1 : hdr.NTr - 1;
          red_tile<C>(ws, io, sm.red, fd, b, j, f, hdr.key_mode, hdr.want, hdr.B, hdr.NTr, hdr.N,
                      persistent, dt, dlast, fast);
          if (persistent) {
            __syncthreads();
            if (threadIdx.x == 0) {
              // the frame's last tile with points also counts its skipped tiles
              const int64_t nv = f.status == kFrameOk ? (int64_t)f.n_valid : 0;
              const int jl = nv > 0 ? (int)((nv - 1) / C::TR) : 0;
              const uint32_t skipped = j == jl ? (uint32_t)(fd.ntr - jl - 1) : 0u;
              fence_rel();
              atomicAdd(&ws.ctl->red_tiles_done, 1u + skipped);
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

// Clears the per-call state and builds the tile -> (frame, tile) tables
// (a fill kernel: graph-safe, no memset nodes).
__global__ void vg_init_kernel(Ws ws) {
  const CallHdr hdr = *ws.hdr;
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nth = (size_t)gridDim.x * blockDim.x;
  uint32_t* ctl = reinterpret_cast<uint32_t*>(ws.ctl);
  constexpr size_t kErrWord = offsetof(Ctl, error) / 4;
  for (size_t i = tid; i < sizeof(Ctl) / 4; i += nth)
    ctl[i] = (i == kErrWord && hdr.fail_waits) ? 1u : 0u;
  uint32_t* fs = reinterpret_cast<uint32_t*>(ws.fs);
  for (size_t i = tid; i < (size_t)hdr.B * (sizeof(FrameState) / 4); i += nth) fs[i] = 0u;
  for (size_t i = tid; i < (size_t)hdr.B * ws.slots * ws.R; i += nth) ws.hist[i] = 0u;
  for (size_t i = tid; i < (size_t)hdr.NTr; i += nth) {
    ws.rdesc[i] = 0ull;
    ws.fflag[i] = 0u;
    ws.pend[i].valid = 0u;
  }
  const size_t ntot = (size_t)hdr.NTb + hdr.NTs + hdr.NTr;
  for (size_t i = tid; i < ntot; i += nth) {
    const uint32_t* tp;
    uint32_t t;
    if (i < (size_t)hdr.NTb) { tp = ws.tpb; t = (uint32_t)i; }
    else if (i < (size_t)hdr.NTb + hdr.NTs) { tp = ws.tps; t = (uint32_t)(i - hdr.NTb); }
    else { tp = ws.tpr; t = (uint32_t)(i - hdr.NTb - hdr.NTs); }
    int lo = 0, hi = hdr.B;  // largest b with tp[b] <= t
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (tp[mid] <= t) lo = mid;
      else hi = mid;
    }
    ws.tinfo[i] = make_uint2((uint32_t)lo, t - tp[lo]);
  }
}

// Last launch of a call: a device-side time-out anywhere in the call (a
// bounded wait that gave up, a cell head not found) marks every frame's status,
// whichever tile raised it and whenever.
__global__ void vg_status_kernel(Ws ws) {
  if (__hip_atomic_load(&ws.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
  const CallHdr hdr = *ws.hdr;
  int32_t* st = ws.io->frame_status;
  for (int b = threadIdx.x; b < hdr.B; b += blockDim.x) st[b] = kFrameDeviceError;
}

// A one-frame call's staged region passed by value (calls that copy nothing
// from host memory): header, I/O pointers, frame description, tile prefixes.
struct StageArgs {
  CallHdr hdr;
  Io io;
  FrameDesc fd;
  uint32_t tp[3][2];  // big / sort / reduce tile prefixes over the one frame
};

__global__ void vg_stage_kernel(Ws ws, StageArgs a) {
  if (threadIdx.x != 0) return;
  *ws.hdr = a.hdr;
  *ws.io = a.io;
  ws.fd[0] = a.fd;
  ws.tpb[0] = a.tp[0][0];
  ws.tpb[1] = a.tp[0][1];
  ws.tps[0] = a.tp[1][0];
  ws.tps[1] = a.tp[1][1];
  ws.tpr[0] = a.tp[2][0];
  ws.tpr[1] = a.tp[2][1];
}

// Result of a one-frame call on the device: its number of cells (0 unless the
// frame is VG_OK) and its status.
__global__ void vg_result_kernel(Ws ws, int64_t* m, int32_t* status) {
  if (threadIdx.x != 0) return;
  const Io io = *ws.io;
  const uint32_t err = __hip_atomic_load(&ws.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int32_t st = err ? (int32_t)kFrameDeviceError : io.frame_status[0];
  *status = st;
  *m = st == kFrameOk ? io.out_offsets[1] - io.out_offsets[0] : 0;
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

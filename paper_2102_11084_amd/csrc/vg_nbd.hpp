// Device side of the neighbour-bucket decimation (arXiv 2102.11084, Sec. II-C
// and Alg. 1), built on the voxel pipeline's sorted cell table.
//
// The pipeline gives every valid point its cell (the row of the cell in
// ascending key order), and every cell its key and point count.  Here:
//   scan      cell starts = exclusive prefix of the counts (the buckets)
//   scatter   points into bucket order: x, y, z, input index, cell
//   ranges    per cell, the 9 runs of cells around it (dy, dz in -1..1; the
//             three x neighbours are consecutive keys of a linear key, so each
//             run is one range of bucket-ordered points): the 27-bucket search
//   count     per point, its neighbours: points of the 9 ranges within the
//             radius (Eq. (1), in binary32 with one rounding per operation)
// and then rounds (Alg. 1's loop), each two launches:
//   round     the round's marked points are those present with more than
//             `umbral` neighbours.  An upper bound of their number (the last
//             round's count less its deletions: counts only fall) tells every
//             workgroup at once whether this is surely the last round (every
//             marked point is deleted) or else the priority window expected to
//             hold the round_size smallest priorities (with a wide margin); the
//             marked points in the window become candidates, and each
//             workgroup counts the marked points it saw.  The workgroup that
//             finishes last then has the exact count and picks: the round_size
//             candidates of smallest (priority, index), each ranked against the
//             others in LDS, are deleted (an exact radix select over every
//             marked point when the window falls short; every marked point when
//             there are at most round_size); the round counter advances
//   decrement the neighbours of every point deleted in the round lose one
//             from their count (no recount: a count only ever changes by the
//             deletions around it)
// Every round kernel exits at once after the last round, so rounds can be
// enqueued ahead of the host's check.
#pragma once

#include "vg_pipeline.hpp"
#include "vg_scan.hpp"

namespace vg {

constexpr int kNbdBlock = 256;

struct NbdCtl {
  float mn[3];
  float inv;
  uint32_t d[3];
  float r2;
  uint32_t m;           // cells
  uint32_t nv;          // valid points
  int32_t status;       // frame status of the pipeline (0, 3 overflow, 5 device)
  uint32_t umbral;
  uint32_t round_size;
  uint32_t pad0;
  uint64_t seed;
  uint32_t round;       // rounds finished
  uint32_t done;        // the last round has run
  uint32_t marked;      // at least the points marked at the start of the next round
  uint32_t ncand;       // candidates of the current round
  uint32_t ndel;        // points deleted in the current round (appends)
  uint32_t ndel_out;    // points deleted in the round just picked (for the decrement)
  uint32_t bstar;       // priority bucket of the round_size-th smallest
  uint32_t need;        // candidates still to delete from that bucket
  uint32_t n_in;        // length of the keep scan's input
  uint32_t nkeep;       // survivors
  uint32_t log_cap;     // entries of marked_log
  uint32_t scan_total;  // total of the last scan
  uint32_t exact;       // select through the exact path only
  uint32_t unmarked;    // points the last decrement took out of the marked set
  uint32_t pad2;
  uint64_t arrive;      // round launch: finished workgroups << 40 | marked points they saw
};

static_assert(offsetof(NbdCtl, done) == offsetof(NbdCtl, round) + 4 &&
                  offsetof(NbdCtl, marked) == offsetof(NbdCtl, round) + 8,
              "round, done, marked adjacent (read back together)");
static_assert(offsetof(NbdCtl, arrive) % 8 == 0, "64-bit arrival counter");

struct NbdCand {
  uint64_t pri;
  uint32_t idx;   // input index (ties of priority go to the smaller index)
  uint32_t pos;   // bucket-order position
};

struct NbdWs {
  NbdCtl* ctl;
  const float* x;
  const float* y;
  const float* z;
  const uint8_t* rgb;
  int64_t n;
  uint64_t* ckey;       // [n] cell keys (pipeline output)
  uint32_t* ccount;     // [n] cell counts (pipeline output)
  int32_t* pcell;       // [n] cell of every point (pipeline output)
  uint32_t* seg;        // [n + 1] cell starts
  uint32_t* cursor;     // [n] scatter cursors
  uint32_t* bsum;       // [scan workgroups + 1]
  float* sx;            // [n] bucket order
  float* sy;
  float* sz;
  uint32_t* sidx;
  uint32_t* scell;
  uint2* rng;           // [n * 9] point ranges of the 9 neighbour runs of a cell
  uint32_t* cnt;        // [n] present neighbours
  uint8_t* alive;       // [n]
  NbdCand* cand;        // [n]
  uint32_t* del;        // [round_size]
  int64_t* marked_log;  // [log_cap]
  uint32_t* keep;       // [n] survivor flags, input order
  uint32_t* kpos;       // [n + 1] their exclusive prefix
  // caller outputs (may be null)
  uint32_t* count0;
  uint32_t* keep_index;
  float* ox;
  float* oy;
  float* oz;
  uint8_t* orgb;
};

// ------------------------------------------------------------- helpers ----
// Squared distance from a to b: RN32(RN32(RN32(dx*dx) + RN32(dy*dy)) + RN32(dz*dz)),
// dx = RN32(bx - ax) and so on; symmetric in a and b.
__device__ __forceinline__ float nbd_d2(float ax, float ay, float az, float bx, float by,
                                        float bz) {
  const float dx = __fsub_rn(bx, ax), dy = __fsub_rn(by, ay), dz = __fsub_rn(bz, az);
  return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), word 0 of the output for
// counter (c0, c1, 0, 0) under key (k0, 0): ten rounds of two 64x64->128
// multiplications by the round constants, halves mixed with the other words
// and the key; the key advances by the Weyl constants between rounds.
__device__ __forceinline__ uint64_t philox4x64_w0(uint64_t c0, uint64_t c1, uint64_t k0) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = c0, x1 = c1, x2 = 0, x3 = 0, k1 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t hi0 = __umul64hi(kM0, x0), lo0 = kM0 * x0;
    const uint64_t hi1 = __umul64hi(kM1, x2), lo1 = kM1 * x2;
    const uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
  return x0;
}

__device__ __forceinline__ uint64_t nbd_priority(const NbdCtl& c, uint32_t idx, uint32_t round) {
  return philox4x64_w0((uint64_t)idx, (uint64_t)round, c.seed);
}

// ---------------------------------------------------------- setup ----
// Grid of the cloud from the pipeline's workspace (the same frame parameters
// its kernels used), the call's constants, and cleared tables.
__global__ void nbd_setup_kernel(Ws pws, NbdWs w, uint32_t umbral, uint32_t round_size,
                                 uint64_t seed, float r2, uint32_t log_cap, uint32_t exact) {
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nth = (size_t)gridDim.x * blockDim.x;
  for (size_t i = tid; i < (size_t)w.n; i += nth) {
    w.keep[i] = 0u;
    if (w.count0) w.count0[i] = 0u;
  }
  if (tid != 0) return;
  NbdCtl c;
  __builtin_memset(&c, 0, sizeof c);
  const FrameParams f = frame_params(pws, 0, 0, 8);
  const uint32_t err = ld_rlx(&pws.ctl->error);
  const int32_t fst = pws.io->frame_status[0];
  c.status = err ? (int32_t)kFrameDeviceError : fst;
  for (int a = 0; a < 3; ++a) {
    c.mn[a] = f.mn[a];
    c.d[a] = f.d[a];
  }
  c.inv = f.inv;
  c.r2 = r2;
  c.nv = c.status == kFrameOk ? f.n_valid : 0u;
  c.m = c.status == kFrameOk
            ? (uint32_t)(pws.io->out_offsets[1] - pws.io->out_offsets[0])
            : 0u;
  c.umbral = umbral;
  c.round_size = round_size;
  c.seed = seed;
  c.n_in = (uint32_t)w.n;
  c.log_cap = log_cap;
  c.exact = exact;
  // nothing to decimate: the loop is already over (one empty round)
  if (c.status != kFrameOk) c.done = 1;
  *w.ctl = c;
}

// ------------------------------------------------- buckets and counts ----
__global__ __launch_bounds__(kNbdBlock) void nbd_scatter_kernel(NbdWs w) {
  if (w.ctl->status != kFrameOk) return;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < w.n; i += nth) {
    const int32_t c = w.pcell[i];
    if (c < 0) continue;
    const uint32_t pos = atomicAdd(&w.cursor[c], 1u);
    w.sx[pos] = w.x[i];
    w.sy[pos] = w.y[i];
    w.sz[pos] = w.z[i];
    w.sidx[pos] = (uint32_t)i;
    w.scell[pos] = (uint32_t)c;
  }
}

// First cell with key >= k among ckey[0, m) (ascending).
__device__ __forceinline__ uint32_t nbd_lower_bound(const uint64_t* ck, uint32_t m, uint64_t k) {
  uint32_t lo = 0, hi = m;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (ck[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kNbdBlock) void nbd_ranges_kernel(NbdWs w) {
  const NbdCtl c = *w.ctl;
  if (c.status != kFrameOk) return;
  const uint32_t nth = gridDim.x * blockDim.x;
  const uint64_t d0 = c.d[0], d1 = c.d[1], d2 = c.d[2];
  for (uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x; cell < c.m; cell += nth) {
    const uint64_t key = w.ckey[cell];
    const uint64_t kx = key % d0, t = key / d0;
    const uint64_t ky = t % d1, kz = t / d1;
    const uint64_t xlo = kx > 0 ? kx - 1 : 0, xhi = kx + 1 < d0 ? kx + 1 : kx;
    int r = 0;
    for (int dz = -1; dz <= 1; ++dz) {
      for (int dy = -1; dy <= 1; ++dy, ++r) {
        const int64_t yy = (int64_t)ky + dy, zz = (int64_t)kz + dz;
        uint2 out = make_uint2(0u, 0u);
        if (yy >= 0 && yy < (int64_t)d1 && zz >= 0 && zz < (int64_t)d2) {
          const uint64_t row = (uint64_t)yy + d1 * (uint64_t)zz;
          const uint32_t lb = nbd_lower_bound(w.ckey, c.m, xlo + d0 * row);
          const uint32_t ub = nbd_lower_bound(w.ckey, c.m, xhi + d0 * row + 1);
          out = make_uint2(w.seg[lb], w.seg[ub]);
        }
        w.rng[(size_t)cell * 9 + r] = out;
      }
    }
  }
}

// Wave-aggregated add of a per-lane count (every lane of the wave active).
__device__ __forceinline__ void nbd_wave_add(uint32_t* ctr, uint32_t v) {
  const uint32_t tot = wave_incl_add(v);
  const uint32_t all = (uint32_t)__shfl((int)tot, 63);
  if ((threadIdx.x & 63) == 63 && all) atomicAdd(ctr, all);
}

// Neighbours of every point before any deletion, and the first round's marked
// count.
__global__ __launch_bounds__(kNbdBlock) void nbd_count_kernel(NbdWs w) {
  const NbdCtl c = *w.ctl;
  if (c.status != kFrameOk) return;
  const uint32_t nth = gridDim.x * blockDim.x;
  uint32_t marked = 0;
  for (uint32_t j0 = blockIdx.x * blockDim.x; j0 < c.nv; j0 += nth) {
    const uint32_t j = j0 + threadIdx.x;
    if (j >= c.nv) continue;
    const float px = w.sx[j], py = w.sy[j], pz = w.sz[j];
    const uint2* rg = w.rng + (size_t)w.scell[j] * 9;
    uint32_t cnt = 0;
    for (int r = 0; r < 9; ++r) {
      const uint2 q = rg[r];
      for (uint32_t k = q.x; k < q.y; ++k) {
        const float d2 = nbd_d2(px, py, pz, w.sx[k], w.sy[k], w.sz[k]);
        cnt += (k != j && d2 <= c.r2) ? 1u : 0u;
      }
    }
    w.cnt[j] = cnt;
    w.alive[j] = 1;
    marked += cnt > c.umbral ? 1u : 0u;
    if (w.count0) w.count0[w.sidx[j]] = cnt;
  }
  nbd_wave_add(&w.ctl->marked, marked);
}

// ----------------------------------------------------------- rounds ----
// The priority window [0, T) of a round with M marked points: expected to hold
// the round_size smallest priorities with a margin of 8 standard deviations
// (priorities are uniform: the count below T is binomial).  T only limits
// which points are candidates, never which are deleted.
__device__ __forceinline__ uint64_t nbd_window(uint32_t M, uint32_t K) {
  uint64_t T = ~0ull;
  if (M > K) {
    const double want = (double)K + 8.0 * sqrt((double)K) + 32.0;
    const double r = want / (double)M;
    if (r < 1.0) T = (uint64_t)(r * 18446744073709551616.0);
  }
  return T;
}

__device__ __forceinline__ bool nbd_marked(const NbdWs& w, uint32_t umbral, uint32_t j) {
  return w.alive[j] && w.cnt[j] > umbral;
}

__device__ __forceinline__ bool nbd_key_less(uint64_t pa, uint32_t ia, uint64_t pb, uint32_t ib) {
  return pa < pb || (pa == pb && ia < ib);
}

constexpr int kPickBlock = 1024;
constexpr int kPickCap = 4096;   // candidates bucketed in LDS
constexpr int kPickBins = 4096;  // buckets of the window
constexpr int kPickEdge = 256;   // candidates of the boundary bucket ranked in LDS
constexpr int kCollectItems = 2; // points per thread per collect step

// The round: every workgroup collects (in the last round every marked point
// is deleted; otherwise the marked points below the window become
// candidates, appends gathered per workgroup), and the workgroup that finishes
// last picks: the round_size marked points of smallest (priority, index)
// are deleted.  Usually from the window's candidates: they are counted into
// 4096 buckets by their priority's leading bits (priorities in the window are
// uniform, so a bucket holds about one); a block scan finds the bucket that
// holds the round_size-th smallest; candidates in lower buckets go, and those
// in that bucket are ranked against each other.  When the window holds fewer
// than round_size candidates (or more than fit in LDS), or the exact path is
// asked for, a radix select over every marked point, most significant byte
// first over the 64 priority bits and then the 32 index bits, decides
// instead.  Keys are distinct (indices are), so exactly round_size go.
__global__ __launch_bounds__(kPickBlock) void nbd_round_kernel(NbdWs w) {
  __shared__ uint64_t cp[kPickCap];
  __shared__ uint32_t ci[kPickCap];
  __shared__ uint32_t cpos[kPickCap];
  __shared__ uint32_t hb[kPickBins];
  __shared__ uint64_t ep[kPickEdge];
  __shared__ uint32_t ei[kPickEdge], epos[kPickEdge];
  __shared__ uint32_t ws[kPickBlock / 64];
  __shared__ uint32_t h[256];
  __shared__ uint64_t pfx_pri;
  __shared__ uint32_t pfx_idx, need_s, ndel_s, bnd_s, nedge_s, base_s, picker_s, mtot_s;
  const NbdCtl c = *w.ctl;
  if (c.done) return;
  const uint32_t t = threadIdx.x;
  const uint32_t K = c.round_size;
  const bool surely_last = c.marked <= K;
  // the window is sized for an estimate of this round's marked count: the
  // upper bound less twice the points the last decrement unmarked (a window
  // too narrow falls back to the exact select; one too wide costs LDS work)
  const uint32_t est = max(max(K + 1u, c.marked / 2u),
                           c.marked > 2u * c.unmarked ? c.marked - 2u * c.unmarked : 0u);
  const uint64_t window = nbd_window(est, K);

  // ---- collect, and count the marked points: chunks of kCollectItems *
  // kPickBlock consecutive points per workgroup, item u of thread t at
  // u * kPickBlock + t (independent priorities in flight together)
  uint32_t seen = 0;
  constexpr uint32_t chunk = kCollectItems * kPickBlock;
  const uint32_t stride = gridDim.x * chunk;
  if (surely_last || !c.exact) {
    for (uint32_t j0 = blockIdx.x * chunk; j0 < c.nv; j0 += stride) {
      bool sel[kCollectItems];
      uint64_t pri[kCollectItems];
#pragma unroll
      for (int u = 0; u < kCollectItems; ++u) {
        const uint32_t j = j0 + u * kPickBlock + t;
        sel[u] = false;
        pri[u] = 0;
        if (j < c.nv && nbd_marked(w, c.umbral, j)) {
          ++seen;
          if (surely_last) {
            sel[u] = true;
          } else {
            pri[u] = nbd_priority(c, w.sidx[j], c.round);
            sel[u] = pri[u] < window;
          }
        }
      }
      uint32_t mine = 0;
#pragma unroll
      for (int u = 0; u < kCollectItems; ++u) mine += sel[u] ? 1u : 0u;
      uint32_t tot;
      uint32_t at = block_excl_scan<kPickBlock>(mine, ws, tot);
      if (tot == 0) continue;
      if (t == 0) base_s = atomicAdd(surely_last ? &w.ctl->ndel : &w.ctl->ncand, tot);
      __syncthreads();
      at += base_s;
#pragma unroll
      for (int u = 0; u < kCollectItems; ++u) {
        if (!sel[u]) continue;
        const uint32_t j = j0 + u * kPickBlock + t;
        if (surely_last) {
          w.del[at] = j;
          w.alive[j] = 0;
        } else {
          NbdCand cd;
          cd.pri = pri[u];
          cd.idx = w.sidx[j];
          cd.pos = j;
          w.cand[at] = cd;
        }
        ++at;
      }
      __syncthreads();  // base_s is reused
    }
  } else {
    for (uint32_t j = blockIdx.x * kPickBlock + t; j < c.nv; j += gridDim.x * kPickBlock)
      seen += nbd_marked(w, c.umbral, j) ? 1u : 0u;
  }
  uint32_t wg_seen;
  (void)block_excl_scan<kPickBlock>(seen, ws, wg_seen);
  // ---- the workgroup that finishes last picks.  Every wave waits for its
  // appends to reach the L2 of its XCD, then one release per workgroup writes
  // them back before the workgroup counts itself in (a release in every wave
  // measured 16 times the write-backs, and 40 us per round); the picker's
  // acquire drops stale lines before its waves read the lists.  One 64-bit
  // add counts the workgroup in and adds its marked points.
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (t == 0) {
    fence_rel();
    const uint64_t before =
        atomicAdd((unsigned long long*)&w.ctl->arrive, (1ull << 40) | (uint64_t)wg_seen);
    picker_s = (uint32_t)(before >> 40) == gridDim.x - 1 ? 1u : 0u;
    mtot_s = (uint32_t)(before & ((1ull << 40) - 1ull)) + wg_seen;
    if (picker_s) fence_acq();
    ndel_s = 0u;
  }
  __syncthreads();
  if (!picker_s) return;
  const uint32_t M = mtot_s;  // the round's marked points
  const bool last = M <= K;
  if (last && !surely_last) {
    // every marked point goes (the collect took candidates instead); a point
    // is tested once, by one thread, before it can be deleted
    for (uint32_t j = t; j < c.nv; j += kPickBlock) {
      if (!nbd_marked(w, c.umbral, j)) continue;
      w.del[atomicAdd(&ndel_s, 1u)] = j;
      w.alive[j] = 0;
    }
  } else if (!last) {
    const uint32_t nc = ld_rlx(&w.ctl->ncand);
    if (!c.exact && nc >= K && nc <= (uint32_t)kPickCap) {
      // bucket of a priority in [0, window): its leading bits below the
      // window's top bit, 12 of them
      const int wbits = window == ~0ull ? 64 : 64 - __clzll(window);
      const int shift = max(0, wbits - 12);
      for (uint32_t k = t; k < (uint32_t)kPickBins; k += kPickBlock) hb[k] = 0u;
      if (t == 0) nedge_s = 0u;
      __syncthreads();
      for (uint32_t k = t; k < nc; k += kPickBlock) {
        const NbdCand cd = w.cand[k];
        cp[k] = cd.pri;
        ci[k] = cd.idx;
        cpos[k] = cd.pos;
        atomicAdd(&hb[(uint32_t)(cd.pri >> shift) & (kPickBins - 1)], 1u);
      }
      __syncthreads();
      constexpr int PB = kPickBins / kPickBlock;
      uint32_t v[PB], sum = 0;
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        v[q] = hb[t * PB + q];
        sum += v[q];
      }
      uint32_t tot;
      uint32_t run = block_excl_scan<kPickBlock>(sum, ws, tot);
      if (run < K && K <= run + sum) {
#pragma unroll
        for (int q = 0; q < PB; ++q) {
          if (run < K && K <= run + v[q]) {
            bnd_s = t * PB + q;
            need_s = K - run;
          }
          run += v[q];
        }
      }
      __syncthreads();
      const uint32_t bnd = bnd_s;
      for (uint32_t k = t; k < nc; k += kPickBlock) {
        const uint32_t bk = (uint32_t)(cp[k] >> shift) & (kPickBins - 1);
        if (bk < bnd) {
          w.del[atomicAdd(&ndel_s, 1u)] = cpos[k];
          w.alive[cpos[k]] = 0;
        } else if (bk == bnd) {
          const uint32_t e = atomicAdd(&nedge_s, 1u);
          if (e < (uint32_t)kPickEdge) {
            ep[e] = cp[k];
            ei[e] = ci[k];
            epos[e] = cpos[k];
          }
        }
      }
      __syncthreads();
      const uint32_t ne = min(nedge_s, (uint32_t)kPickEdge);
      if (nedge_s <= (uint32_t)kPickEdge) {
        // rank within the boundary bucket; the need_s smallest go
        if (t < ne) {
          uint32_t rank = 0;
          for (uint32_t k = 0; k < ne; ++k) rank += nbd_key_less(ep[k], ei[k], ep[t], ei[t]) ? 1u : 0u;
          if (rank < need_s) {
            w.del[atomicAdd(&ndel_s, 1u)] = epos[t];
            w.alive[epos[t]] = 0;
          }
        }
      } else {
        // a crowded boundary bucket (not expected): rank its members against
        // all candidates of the bucket, read from the candidate list
        for (uint32_t k = t; k < nc; k += kPickBlock) {
          if (((uint32_t)(cp[k] >> shift) & (kPickBins - 1)) != bnd) continue;
          uint32_t rank = 0;
          for (uint32_t q = 0; q < nc; ++q)
            rank += (((uint32_t)(cp[q] >> shift) & (kPickBins - 1)) == bnd &&
                     nbd_key_less(cp[q], ci[q], cp[k], ci[k])) ? 1u : 0u;
          if (rank < need_s) {
            w.del[atomicAdd(&ndel_s, 1u)] = cpos[k];
            w.alive[cpos[k]] = 0;
          }
        }
      }
      __syncthreads();
    } else {
      // exact path over every marked point
      if (t == 0) {
        pfx_pri = 0ull;
        pfx_idx = 0u;
        need_s = K;
      }
      __syncthreads();
      for (int level = 0; level < 12; ++level) {
        if (t < 256) h[t] = 0u;
        __syncthreads();
        const int pbits = min(64, 8 * level);
        const int ibits = max(0, 8 * level - 64);
        const uint64_t pmask = pbits == 0 ? 0ull : (pbits >= 64 ? ~0ull : ~((1ull << (64 - pbits)) - 1ull));
        const uint32_t imask = ibits == 0 ? 0u : ~((1u << (32 - ibits)) - 1u);  // ibits <= 24
        const uint64_t pp = pfx_pri;
        const uint32_t pi = pfx_idx;
        for (uint32_t j = t; j < c.nv; j += kPickBlock) {
          if (!nbd_marked(w, c.umbral, j)) continue;
          const uint32_t idx = w.sidx[j];
          const uint64_t pri = nbd_priority(c, idx, c.round);
          if ((pri & pmask) != pp || (idx & imask) != pi) continue;
          const uint32_t dig = level < 8 ? (uint32_t)(pri >> (56 - 8 * level)) & 255u
                                         : (idx >> (24 - 8 * (level - 8))) & 255u;
          atomicAdd(&h[dig], 1u);
        }
        __syncthreads();
        const uint32_t hv = t < 256 ? h[t] : 0u;
        uint32_t tot;
        const uint32_t before = block_excl_scan<kPickBlock>(hv, ws, tot);
        const uint32_t need = need_s;
        __syncthreads();
        if (t < 256 && before < need && need <= before + hv) {
          need_s = need - before;
          if (level < 8) pfx_pri = pp | ((uint64_t)t << (56 - 8 * level));
          else pfx_idx = pi | (t << (24 - 8 * (level - 8)));
        }
        __syncthreads();
      }
      const uint64_t tp = pfx_pri;
      const uint32_t ti = pfx_idx;
      // (a point is tested once, by one thread, before it can be deleted)
      for (uint32_t j = t; j < c.nv; j += kPickBlock) {
        if (!nbd_marked(w, c.umbral, j)) continue;
        const uint32_t idx = w.sidx[j];
        const uint64_t pri = nbd_priority(c, idx, c.round);
        if (!nbd_key_less(tp, ti, pri, idx)) {  // key <= the round_size-th smallest
          w.del[atomicAdd(&ndel_s, 1u)] = j;
          w.alive[j] = 0;
        }
      }
    }
  }
  __syncthreads();
  if (t == 0) {
    const uint32_t nd = surely_last ? ld_rlx(&w.ctl->ndel) : ndel_s;
    if (c.round < c.log_cap) w.marked_log[c.round] = (int64_t)M;
    w.ctl->ndel_out = nd;
    w.ctl->marked = M - nd;  // counts only fall: at least next round's marked points
    w.ctl->unmarked = c.marked - M;
    w.ctl->ndel = 0u;
    w.ctl->ncand = 0u;
    w.ctl->arrive = 0ull;
    w.ctl->round = c.round + 1u;
    if (last) w.ctl->done = 1u;
  }
}

// Every point deleted in the round (one wave each) takes one from the count of
// each of its neighbours.  The wave's lanes run over the 9 ranges as one
// concatenated list, so a deleted point costs ceil(candidates / 64) steps.
__global__ __launch_bounds__(kNbdBlock) void nbd_decrement_kernel(NbdWs w) {
  const NbdCtl c = *w.ctl;
  if (c.done) return;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t waves = gridDim.x * (kNbdBlock / 64);
  for (uint32_t g = blockIdx.x * (kNbdBlock / 64) + (threadIdx.x >> 6); g < c.ndel_out;
       g += waves) {
    const uint32_t d = w.del[g];
    const float px = w.sx[d], py = w.sy[d], pz = w.sz[d];
    const uint2* rg = w.rng + (size_t)w.scell[d] * 9;
    uint32_t lo[9], end[9];  // range r covers list positions [end[r-1], end[r])
    uint32_t total = 0;
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const uint2 q = rg[r];
      lo[r] = q.x;
      total += q.y - q.x;
      end[r] = total;
    }
    // four list positions per lane at a time: their loads are in flight together
    for (uint32_t k0 = lane; k0 < total; k0 += 4 * 64) {
      uint32_t q[4];
      float qx[4], qy[4], qz[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t k = k0 + 64 * u;
        uint32_t before = 0;
        q[u] = d;  // past the list: the deleted point itself, never counted
#pragma unroll
        for (int r = 0; r < 9; ++r) {
          if (k >= before && k < end[r]) q[u] = lo[r] + (k - before);
          before = end[r];
        }
        qx[u] = w.sx[q[u]];
        qy[u] = w.sy[q[u]];
        qz[u] = w.sz[q[u]];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float d2 = nbd_d2(px, py, pz, qx[u], qy[u], qz[u]);
        if (q[u] != d && d2 <= c.r2) atomicSub(&w.cnt[q[u]], 1u);
      }
    }
  }
}

// ----------------------------------------------------------- output ----
__global__ __launch_bounds__(kNbdBlock) void nbd_keep_kernel(NbdWs w) {
  const NbdCtl c = *w.ctl;
  const uint32_t nth = gridDim.x * blockDim.x;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < c.nv; j += nth)
    if (w.alive[j]) w.keep[w.sidx[j]] = 1u;
}

// Survivors in input order: their index and, when asked, their point.
__global__ __launch_bounds__(kNbdBlock) void nbd_emit_kernel(NbdWs w) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < w.n; i += nth) {
    if (!w.keep[i]) continue;
    const uint32_t k = w.kpos[i];
    if (w.keep_index) w.keep_index[k] = (uint32_t)i;
    if (w.ox) {
      w.ox[k] = w.x[i];
      w.oy[k] = w.y[i];
      w.oz[k] = w.z[i];
    }
    if (w.orgb && w.rgb) {
      w.orgb[3 * (size_t)k] = w.rgb[3 * (size_t)i];
      w.orgb[3 * (size_t)k + 1] = w.rgb[3 * (size_t)i + 1];
      w.orgb[3 * (size_t)k + 2] = w.rgb[3 * (size_t)i + 2];
    }
  }
}

}  // namespace vg

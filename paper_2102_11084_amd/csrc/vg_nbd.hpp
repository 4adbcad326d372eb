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
// and then rounds (Alg. 1's loop), each five launches:
//   mark      points present with more than `umbral` neighbours are marked;
//             their Philox priorities' top 16 bits are counted
//   select    (one workgroup) if at most round_size are marked this is the last
//             round; else the priority bucket holding the round_size-th smallest
//   collect   marked points below that bucket are deleted, those in it become
//             candidates; in the last round every marked point is deleted
//   pick      (one workgroup) radix select of the remaining candidates by
//             (priority, index); deleted; the round counter advances
//   decrement the neighbours of every point deleted in the round lose one
//             from their count (no recount: a count only ever changes by the
//             deletions around it)
// Every round kernel exits at once after the last round, so rounds can be
// enqueued ahead of the host's check.
#pragma once

#include "vg_pipeline.hpp"

namespace vg {

constexpr int kNbdBlock = 256;
constexpr int kNbdScanTile = 4096;      // elements per workgroup of the scans
constexpr int kNbdHistBins = 1 << 16;   // top 16 bits of a priority

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
  uint32_t last;        // the current round is the last one
  uint32_t marked;      // points marked in the current round
  uint32_t ncand;       // candidates of the current round
  uint32_t ndel;        // points deleted in the current round
  uint32_t bstar;       // priority bucket of the round_size-th smallest
  uint32_t need;        // candidates still to delete from that bucket
  uint32_t n_in;        // length of the keep scan's input
  uint32_t nkeep;       // survivors
  uint32_t log_cap;     // entries of marked_log
  uint32_t scan_total;  // total of the last scan
};

static_assert(offsetof(NbdCtl, done) == offsetof(NbdCtl, round) + 4, "round, done adjacent");

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
  uint32_t* hist;       // [kNbdHistBins]
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
                                 uint64_t seed, float r2, uint32_t log_cap) {
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nth = (size_t)gridDim.x * blockDim.x;
  for (size_t i = tid; i < (size_t)kNbdHistBins; i += nth) w.hist[i] = 0u;
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
  // nothing to decimate: the loop is already over (one empty round)
  if (c.status != kFrameOk) c.done = 1;
  *w.ctl = c;
}

// ----------------------------------------------------------- scans ----
// Exclusive prefix of in[0, len) in three launches: tile sums, the prefix of
// the tile sums (one workgroup), tile scans.  `len` is read on the device.
__global__ __launch_bounds__(kNbdBlock) void nbd_scan_tiles(const uint32_t* in, const uint32_t* len,
                                                            uint32_t* bsum) {
  __shared__ uint32_t ws[kNbdBlock / 64];
  const uint32_t n = *len;
  const uint32_t t0 = blockIdx.x * (uint32_t)kNbdScanTile;
  if (t0 >= n && blockIdx.x > 0) return;
  uint32_t s = 0;
  for (uint32_t i = t0 + threadIdx.x; i < min(n, t0 + (uint32_t)kNbdScanTile); i += kNbdBlock)
    s += in[i];
  uint32_t tot;
  (void)block_excl_scan<kNbdBlock>(s, ws, tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void nbd_scan_top(const uint32_t* len, uint32_t* bsum,
                                                     uint32_t* total) {
  __shared__ uint32_t ws[1024 / 64];
  const uint32_t n = *len;
  const uint32_t nb = n == 0 ? 1u : (n + kNbdScanTile - 1) / kNbdScanTile;
  uint32_t run = 0;
  for (uint32_t c0 = 0; c0 < nb; c0 += 1024) {
    const uint32_t i = c0 + threadIdx.x;
    const uint32_t v = i < nb ? bsum[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<1024>(v, ws, tot);
    if (i < nb) bsum[i] = run + ex;
    run += tot;
  }
  if (threadIdx.x == 0) *total = run;
}

// out[i] = exclusive prefix; cur (optional) gets a copy; out[len] = total.
__global__ __launch_bounds__(kNbdBlock) void nbd_scan_apply(const uint32_t* in, const uint32_t* len,
                                                            const uint32_t* bsum, uint32_t* out,
                                                            uint32_t* cur, const uint32_t* total) {
  __shared__ uint32_t ws[kNbdBlock / 64];
  constexpr int PER = kNbdScanTile / kNbdBlock;
  const uint32_t n = *len;
  const uint32_t t0 = blockIdx.x * (uint32_t)kNbdScanTile;
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = *total;
  if (t0 >= n) return;
  // each thread scans PER consecutive elements
  const uint32_t b0 = t0 + threadIdx.x * PER;
  uint32_t v[PER];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    v[k] = (b0 + k < n) ? in[b0 + k] : 0u;
    s += v[k];
  }
  uint32_t tot;
  uint32_t run = bsum[blockIdx.x] + block_excl_scan<kNbdBlock>(s, ws, tot);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    if (b0 + k < n) {
      out[b0 + k] = run;
      if (cur) cur[b0 + k] = run;
    }
    run += v[k];
  }
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

// Neighbours of every point before any deletion.
__global__ __launch_bounds__(kNbdBlock) void nbd_count_kernel(NbdWs w) {
  const NbdCtl c = *w.ctl;
  if (c.status != kFrameOk) return;
  const uint32_t nth = gridDim.x * blockDim.x;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < c.nv; j += nth) {
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
    if (w.count0) w.count0[w.sidx[j]] = cnt;
  }
}

// ----------------------------------------------------------- rounds ----
__global__ __launch_bounds__(kNbdBlock) void nbd_mark_kernel(NbdWs w) {
  const NbdCtl c = *w.ctl;
  if (c.done) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) w.ctl->ndel = 0u;  // the last round's deletions are done
  const uint32_t nth = gridDim.x * blockDim.x;
  const uint32_t lane = threadIdx.x & 63;
  for (uint32_t j0 = blockIdx.x * blockDim.x; j0 < c.nv; j0 += nth) {
    const uint32_t j = j0 + threadIdx.x;
    bool mk = false;
    if (j < c.nv && w.alive[j] && w.cnt[j] > c.umbral) {
      mk = true;
      const uint64_t pri = nbd_priority(c, w.sidx[j], c.round);
      atomicAdd(&w.hist[(uint32_t)(pri >> 48)], 1u);
    }
    const uint64_t b = __ballot(mk);
    if (lane == 0 && b) atomicAdd(&w.ctl->marked, (uint32_t)__popcll(b));
  }
}

__global__ __launch_bounds__(1024) void nbd_select_kernel(NbdWs w) {
  __shared__ uint32_t ws[1024 / 64];
  __shared__ uint32_t found[2];
  if (w.ctl->done) return;
  const uint32_t M = w.ctl->marked;
  const uint32_t K = w.ctl->round_size;
  const uint32_t round = w.ctl->round;
  __syncthreads();  // every thread has read the counters before thread 0 resets them
  constexpr int PER = kNbdHistBins / 1024;
  const uint32_t t = threadIdx.x;
  if (M > K) {
    uint32_t h[PER];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      h[k] = w.hist[t * PER + k];
      s += h[k];
    }
    uint32_t tot;
    const uint32_t before = block_excl_scan<1024>(s, ws, tot);
    if (before < K && K <= before + s) {
      uint32_t run = before;
      for (int k = 0; k < PER; ++k) {
        if (run + h[k] >= K) {
          found[0] = t * PER + k;
          found[1] = K - run;
          break;
        }
        run += h[k];
      }
    }
    __syncthreads();
  }
  // cleared for the next round (every bin was read above)
#pragma unroll
  for (int k = 0; k < PER; ++k) w.hist[t * PER + k] = 0u;
  if (t == 0) {
    if (round < w.ctl->log_cap) w.marked_log[round] = (int64_t)M;
    w.ctl->marked = 0u;
    w.ctl->ncand = 0u;
    if (M > K) {
      w.ctl->last = 0u;
      w.ctl->bstar = found[0];
      w.ctl->need = found[1];
    } else {
      w.ctl->last = 1u;
      w.ctl->bstar = 0u;
      w.ctl->need = 0u;
    }
  }
}

__global__ __launch_bounds__(kNbdBlock) void nbd_collect_kernel(NbdWs w) {
  const NbdCtl c = *w.ctl;
  if (c.done) return;
  const uint32_t nth = gridDim.x * blockDim.x;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < c.nv; j += nth) {
    if (!w.alive[j] || w.cnt[j] <= c.umbral) continue;
    if (c.last) {
      w.del[atomicAdd(&w.ctl->ndel, 1u)] = j;
      w.alive[j] = 0;
      continue;
    }
    const uint64_t pri = nbd_priority(c, w.sidx[j], c.round);
    const uint32_t top = (uint32_t)(pri >> 48);
    if (top < c.bstar) {
      w.del[atomicAdd(&w.ctl->ndel, 1u)] = j;
      w.alive[j] = 0;
    } else if (top == c.bstar) {
      NbdCand cd;
      cd.pri = pri;
      cd.idx = w.sidx[j];
      cd.pos = j;
      w.cand[atomicAdd(&w.ctl->ncand, 1u)] = cd;
    }
  }
}

// One workgroup: the `need` candidates of smallest (priority, index) are
// deleted.  Radix select, most significant byte first, over the 48 low bits
// of the priority (the top 16 are the bucket's) and then the 32 index bits;
// the key found last is the need-th smallest, and every candidate at or below
// it goes.  Keys are distinct (indices are), so exactly `need` go.
__global__ __launch_bounds__(kNbdBlock) void nbd_pick_kernel(NbdWs w) {
  __shared__ uint32_t h[256];
  __shared__ uint64_t pfx_pri;
  __shared__ uint32_t pfx_idx, need_s;
  if (w.ctl->done) return;
  const uint32_t t = threadIdx.x;
  if (!w.ctl->last) {
    const uint32_t nc = w.ctl->ncand;
    if (t == 0) {
      pfx_pri = (uint64_t)w.ctl->bstar << 48;
      pfx_idx = 0u;
      need_s = w.ctl->need;
    }
    __syncthreads();
    for (int level = 0; level < 10; ++level) {
      h[t] = 0u;
      __syncthreads();
      // bits of the key fixed so far: 16 + 8 * level of the priority, then index
      const int pbits = min(64, 16 + 8 * level);
      const int ibits = max(0, 8 * level - 48);
      const uint64_t pmask = pbits >= 64 ? ~0ull : ~((1ull << (64 - pbits)) - 1ull);
      const uint32_t imask = ibits == 0 ? 0u : ~((1u << (32 - ibits)) - 1u);  // ibits <= 24
      const uint64_t pp = pfx_pri;
      const uint32_t pi = pfx_idx;
      for (uint32_t k = t; k < nc; k += kNbdBlock) {
        const NbdCand cd = w.cand[k];
        if ((cd.pri & pmask) != pp || (cd.idx & imask) != pi) continue;
        const uint32_t dig = level < 6 ? (uint32_t)(cd.pri >> (40 - 8 * level)) & 255u
                                       : (cd.idx >> (24 - 8 * (level - 6))) & 255u;
        atomicAdd(&h[dig], 1u);
      }
      __syncthreads();
      if (t == 0) {
        uint32_t run = 0, need = need_s;
        for (uint32_t dgt = 0; dgt < 256; ++dgt) {
          if (run + h[dgt] >= need) {
            need_s = need - run;
            if (level < 6) pfx_pri = pp | ((uint64_t)dgt << (40 - 8 * level));
            else pfx_idx = pi | (dgt << (24 - 8 * (level - 6)));
            break;
          }
          run += h[dgt];
        }
      }
      __syncthreads();
    }
    const uint64_t tp = pfx_pri;
    const uint32_t ti = pfx_idx;
    for (uint32_t k = t; k < nc; k += kNbdBlock) {
      const NbdCand cd = w.cand[k];
      if (cd.pri < tp || (cd.pri == tp && cd.idx <= ti)) {
        w.del[atomicAdd(&w.ctl->ndel, 1u)] = cd.pos;
        w.alive[cd.pos] = 0;
      }
    }
  }
  __syncthreads();
  if (t == 0) {
    w.ctl->round = w.ctl->round + 1u;
    if (w.ctl->last) w.ctl->done = 1u;
  }
}

// Every point deleted in the round (one wave each) takes one from the count of
// each of its neighbours.
__global__ __launch_bounds__(kNbdBlock) void nbd_decrement_kernel(NbdWs w) {
  const NbdCtl c = *w.ctl;
  if (c.done) return;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t waves = gridDim.x * (kNbdBlock / 64);
  for (uint32_t g = blockIdx.x * (kNbdBlock / 64) + (threadIdx.x >> 6); g < c.ndel; g += waves) {
    const uint32_t d = w.del[g];
    const float px = w.sx[d], py = w.sy[d], pz = w.sz[d];
    const uint2* rg = w.rng + (size_t)w.scell[d] * 9;
    for (int r = 0; r < 9; ++r) {
      const uint2 q = rg[r];
      for (uint32_t k = q.x + lane; k < q.y; k += 64) {
        const float d2 = nbd_d2(px, py, pz, w.sx[k], w.sy[k], w.sz[k]);
        if (k != d && d2 <= c.r2) atomicSub(&w.cnt[k], 1u);
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

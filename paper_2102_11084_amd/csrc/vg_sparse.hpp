// Removal of sparse cells (the noise the filter is meant to take out,
// Sec. II-C): after the reduce and fix-up, rows whose cell holds fewer than
// its frame's minimum number of points are dropped and the rest renumbered
// densely, frame by frame, in key order.  Four steps after the pipeline:
//   flag     per row, whether it is kept (the row's frame by a binary search
//            of out_offsets)
//   scan     new row of every kept row (exclusive prefix of the flags)
//   gather   kept rows into scratch at their new row (the pipeline's key,
//            index and record buffers are free by then)
//   scatter  scratch back into the outputs, out_offsets and every point's row
//            renumbered
// Launched only for calls that ask for it; every kernel exits at once after a
// device-side time-out.
#pragma once

#include "vg_scan.hpp"

namespace vg {

constexpr int kSparseBlock = 256;

__device__ __forceinline__ bool sparse_active(const Ws& ws, const CallHdr& hdr) {
  return (hdr.filt & kFiltMinPts) && ld_rlx(&ws.ctl->error) == 0;
}

__global__ __launch_bounds__(kSparseBlock) void vg_sparse_flag_kernel(Ws ws) {
  const CallHdr hdr = *ws.hdr;
  if (!sparse_active(ws, hdr)) return;
  const Io io = *ws.io;
  const int64_t M = io.out_offsets[hdr.B];
  if (blockIdx.x == 0 && threadIdx.x == 0) ws.ctl->rows = (uint32_t)M;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += nth) {
    int lo = 0, hi = hdr.B;  // largest b with out_offsets[b] <= r
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (io.out_offsets[mid] <= r) lo = mid;
      else hi = mid;
    }
    const uint32_t minp = ws.xf[lo].minp;
    ws.rflag[r] = io.count[r] >= minp ? 1u : 0u;
  }
}

// Scratch rows: x, y, z -> lo[0], lo[1], hi[0]; count -> hi[1]; key -> idx[0],
// idx[1]; local means and packed colour -> rec; first index -> tx.
__global__ __launch_bounds__(kSparseBlock) void vg_sparse_gather_kernel(Ws ws) {
  const CallHdr hdr = *ws.hdr;
  if (!sparse_active(ws, hdr)) return;
  const Io io = *ws.io;
  const uint32_t want = hdr.want;
  const bool own_count = (hdr.filt & kFiltCountInternal) == 0;
  const int64_t M = ws.ctl->rows;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += nth) {
    if (!ws.rflag[r]) continue;
    const uint32_t k = ws.rpos[r];
    if (want & kOutXYZ) {
      ws.lo[0][k] = __float_as_uint(io.cx[r]);
      ws.lo[1][k] = __float_as_uint(io.cy[r]);
      ws.hi[0][k] = __float_as_uint(io.cz[r]);
    }
    if ((want & kOutCount) && own_count) ws.hi[1][k] = io.count[r];
    if (want & kOutKey) {
      const uint64_t key = io.key[r];
      ws.idx[0][k] = (uint32_t)key;
      ws.idx[1][k] = (uint32_t)(key >> 32);
    }
    float4 rc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (want & kOutLocal) rc = make_float4(io.lx[r], io.ly[r], io.lz[r], 0.f);
    if (want & kOutRGB) {
      const uint8_t* c = io.crgb + 3 * (size_t)r;
      rc.w = __uint_as_float((uint32_t)c[0] | ((uint32_t)c[1] << 8) | ((uint32_t)c[2] << 16));
    }
    if (want & (kOutLocal | kOutRGB)) ws.rec[k] = rc;
    if (want & kOutRef) ws.tx[k] = __uint_as_float(io.ref_index[r]);
  }
}

__global__ __launch_bounds__(kSparseBlock) void vg_sparse_scatter_kernel(Ws ws) {
  const CallHdr hdr = *ws.hdr;
  if (!sparse_active(ws, hdr)) return;
  const Io io = *ws.io;
  const uint32_t want = hdr.want;
  const bool own_count = (hdr.filt & kFiltCountInternal) == 0;
  const int64_t K = ws.ctl->rows_kept;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t k = tid; k < K; k += nth) {
    if (want & kOutXYZ) {
      io.cx[k] = __uint_as_float(ws.lo[0][k]);
      io.cy[k] = __uint_as_float(ws.lo[1][k]);
      io.cz[k] = __uint_as_float(ws.hi[0][k]);
    }
    if ((want & kOutCount) && own_count) io.count[k] = ws.hi[1][k];
    if (want & kOutKey) io.key[k] = ((uint64_t)ws.idx[1][k] << 32) | ws.idx[0][k];
    if (want & (kOutLocal | kOutRGB)) {
      const float4 rc = ws.rec[k];
      if (want & kOutLocal) {
        io.lx[k] = rc.x;
        io.ly[k] = rc.y;
        io.lz[k] = rc.z;
      }
      if (want & kOutRGB) {
        const uint32_t c = __float_as_uint(rc.w);
        io.crgb[3 * (size_t)k] = (uint8_t)c;
        io.crgb[3 * (size_t)k + 1] = (uint8_t)(c >> 8);
        io.crgb[3 * (size_t)k + 2] = (uint8_t)(c >> 16);
      }
    }
    if (want & kOutRef) io.ref_index[k] = __float_as_uint(ws.tx[k]);
  }
  for (int64_t b = tid; b <= hdr.B; b += nth) io.out_offsets[b] = (int64_t)ws.rpos[io.out_offsets[b]];
  if (want & kOutPointCell) {
    for (int64_t i = tid; i < hdr.N; i += nth) {
      const int32_t pc = io.point_cell[i];
      if (pc >= 0) io.point_cell[i] = ws.rflag[pc] ? (int32_t)ws.rpos[pc] : -1;
    }
  }
}

}  // namespace vg

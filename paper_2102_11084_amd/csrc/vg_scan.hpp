// Exclusive prefix sums of u32 arrays whose length is known only on the
// device (cell counts, survivor flags, kept rows), in three launches.
#pragma once

#include "vg_pipeline.hpp"

namespace vg {

constexpr int kScanBlock = 256;
constexpr int kScanTile = 4096;  // elements per workgroup

// Exclusive prefix of in[0, len) in three launches: tile sums, the prefix of
// the tile sums (one workgroup), tile scans.  `len` is read on the device.
__global__ __launch_bounds__(kScanBlock) void vg_scan_tiles(const uint32_t* in, const uint32_t* len,
                                                            uint32_t* bsum) {
  __shared__ uint32_t ws[kScanBlock / 64];
  const uint32_t n = *len;
  const uint32_t t0 = blockIdx.x * (uint32_t)kScanTile;
  if (t0 >= n && blockIdx.x > 0) return;
  uint32_t s = 0;
  for (uint32_t i = t0 + threadIdx.x; i < min(n, t0 + (uint32_t)kScanTile); i += kScanBlock)
    s += in[i];
  uint32_t tot;
  (void)block_excl_scan<kScanBlock>(s, ws, tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void vg_scan_top(const uint32_t* len, uint32_t* bsum,
                                                     uint32_t* total) {
  __shared__ uint32_t ws[1024 / 64];
  const uint32_t n = *len;
  const uint32_t nb = n == 0 ? 1u : (n + kScanTile - 1) / kScanTile;
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
__global__ __launch_bounds__(kScanBlock) void vg_scan_apply(const uint32_t* in, const uint32_t* len,
                                                            const uint32_t* bsum, uint32_t* out,
                                                            uint32_t* cur, const uint32_t* total) {
  __shared__ uint32_t ws[kScanBlock / 64];
  constexpr int PER = kScanTile / kScanBlock;
  const uint32_t n = *len;
  const uint32_t t0 = blockIdx.x * (uint32_t)kScanTile;
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
  uint32_t run = bsum[blockIdx.x] + block_excl_scan<kScanBlock>(s, ws, tot);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    if (b0 + k < n) {
      out[b0 + k] = run;
      if (cur) cur[b0 + k] = run;
    }
    run += v[k];
  }
}

}  // namespace vg

// Host side of libvg: argument checks, workspace layout, launch sequence,
// batch plans and hipGraph replay.  Device code lives in vg_pipeline.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/vg.h"
#include "vg_pipeline.hpp"
#include "vg_nbd.hpp"
#include "vg_sparse.hpp"
#include "vg_map.hpp"

namespace {

using namespace vg;

// ------------------------------------------------------------ variants ----
template <class C, int KIND>
int occupancy_kind() {
  // resident workgroups per CU of one kernel entry (the same on every gfx950)
  static const int occ = [] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, vg_pipeline_kernel<C, KIND>, C::BLOCK,
                                                     0) != hipSuccess)
      n = 1;
    return std::max(n, 1);
  }();
  return occ;
}

template <class C, int KIND>
void launch_kind(const Ws& ws, int lo, int hi, int cus, int bpc, hipStream_t s) {
  const int occ = occupancy_kind<C, KIND>();
  const int grid = cus * (bpc > 0 ? std::min(bpc, occ) : occ);
  hipLaunchKernelGGL((vg_pipeline_kernel<C, KIND>), dim3(grid), dim3(C::BLOCK), 0, s, ws, lo, hi);
}

// Launches phases [lo, hi): all of them in one persistent kernel, or one phase
// with the kernel compiled for that phase kind.  Grids are fixed per kernel
// (CUs x resident workgroups), independent of the call's sizes.
template <class C, bool ONE>
void launch_pipeline(const Ws& ws, int lo, int hi, int cus, int bpc, hipStream_t s) {
  if (lo == 0 && hi == C::NPH) {
    if constexpr (ONE) launch_kind<C, kAll>(ws, lo, hi, cus, bpc, s);
  } else if (lo == C::PH_BBOX) launch_kind<C, kBbox>(ws, lo, hi, cus, bpc, s);
  else if (lo == C::PH_HIST) launch_kind<C, kHist>(ws, lo, hi, cus, bpc, s);
  else if (lo == C::PH_RED) launch_kind<C, kRed>(ws, lo, hi, cus, bpc, s);
  else if (lo == C::PH_FIX) launch_kind<C, kFix>(ws, lo, hi, cus, bpc, s);
  else launch_kind<C, kSort>(ws, lo, hi, cus, bpc, s);
}

struct Variant {
  int block, sort_items, radix, red_items;
  int nph, maxp, R, TS, TB, TR, ph_red;
  bool one;  // built with the one-launch (persistent) form too
  void (*launch)(const Ws&, int ph_lo, int ph_hi, int cus, int bpc, hipStream_t);
};

template <int B, int SI, int W, int RI, bool ONE = false>
constexpr Variant make_variant() {
  using C = Cfg<B, SI, W, RI>;
  return Variant{B, SI, W, RI, C::NPH, C::MAXP, C::R, C::TS, C::TB, C::TR, C::PH_RED, ONE,
                 &launch_pipeline<C, ONE>};
}

// Built variants: (threads, sort items/thread, radix bits, reduce items/thread).
// The one-launch form, whose kernel holds every phase's registers at once, is
// built only where that kernel needs no scratch memory (4 reduce items per
// thread); the others spill their per-thread arrays to 576 B of scratch a lane.
const Variant kVariants[] = {
    make_variant<256, 16, 8, 8>(), make_variant<256, 8, 8, 8>(),  make_variant<256, 12, 8, 8>(),
    make_variant<256, 16, 8, 4>(), make_variant<256, 16, 7, 8>(), make_variant<512, 8, 8, 4, true>(),
    make_variant<512, 8, 8, 8>(),  make_variant<256, 16, 6, 8>(), make_variant<256, 8, 8, 4, true>(),
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

const vg_tuning kDefaultTuning = {512, 8, 8, 512, 8, 0, VG_EXEC_PHASED};

const Variant* find_variant(const vg_tuning* t) {
  if (!t) t = &kDefaultTuning;
  if (t->sort_block != t->reduce_block) return nullptr;
  if (t->exec_mode != VG_EXEC_PERSISTENT && t->exec_mode != VG_EXEC_PHASED) return nullptr;
  if (t->blocks_per_cu < 0 || t->blocks_per_cu > 64) return nullptr;
  for (int i = 0; i < kNumVariants; ++i) {
    const Variant& v = kVariants[i];
    if (v.block == t->sort_block && v.sort_items == t->sort_items && v.radix == t->radix_bits &&
        v.red_items == t->reduce_items)
      return (t->exec_mode == VG_EXEC_PERSISTENT && !v.one) ? nullptr : &v;
  }
  return nullptr;
}

// Compute units per device, looked up once.
std::mutex g_dev_mu;
int g_cus[64];

int device_cus(int dev) {
  if (dev < 0 || dev >= 64) return 0;
  std::lock_guard<std::mutex> lk(g_dev_mu);
  if (g_cus[dev] == 0) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
      return 0;
    g_cus[dev] = c;
  }
  return g_cus[dev];
}

// ------------------------------------------------------------ layout ----
constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  int64_t capN;
  int capB, capNTb, capNTs, capNTr, slots, R;
  size_t hdr, io, fd, tpb, tps, tpr, ilv_s, ilv_perm, xf, staged;  // staged: copied from the host
  size_t tinfo, ctl, fs, hist, sdesc, rdesc, fflag, frag, pend, lo0, lo1, hi0, hi1, id0, id1, rec,
      tx, ty, tz, rflag, rpos, bsum, outoff, fstat;
  size_t total;
};

int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

Layout make_layout(int64_t capN, int capB, const Variant& v) {
  Layout L;
  L.capN = std::max<int64_t>(capN, 1);
  L.capB = std::max(capB, 1);
  L.capNTb = (int)(div_up(L.capN, v.TB) + L.capB);
  L.capNTs = (int)(div_up(L.capN, v.TS) + L.capB);
  L.capNTr = (int)(div_up(L.capN, v.TR) + L.capB);
  L.slots = v.maxp;
  L.R = v.R;
  size_t o = 0;
  L.hdr = o;  o = align_up(o + sizeof(CallHdr));
  L.io = o;   o = align_up(o + sizeof(Io));
  L.fd = o;   o = align_up(o + sizeof(FrameDesc) * L.capB);
  L.tpb = o;  o = align_up(o + 4 * (size_t)(L.capB + 1));
  L.tps = o;  o = align_up(o + 4 * (size_t)(L.capB + 1));
  L.tpr = o;  o = align_up(o + 4 * (size_t)(L.capB + 1));
  L.ilv_s = o; o = align_up(o + 4 * (size_t)(kIlvMaxRounds + 1));
  L.ilv_perm = o; o = align_up(o + 4 * (size_t)kIlvMaxFrames);
  L.xf = o;   o = align_up(o + sizeof(FrameXf) * L.capB);
  L.staged = o;
  L.tinfo = o; o = align_up(o + 8 * ((size_t)L.capNTb + L.capNTs + L.capNTr));
  L.ctl = o;  o = align_up(o + sizeof(Ctl));
  L.fs = o;   o = align_up(o + sizeof(FrameState) * L.capB);
  L.hist = o; o = align_up(o + 4 * (size_t)L.capB * L.slots * L.R);
  L.sdesc = o; o = align_up(o + 4 * (size_t)L.slots * L.capNTs * L.R);
  L.rdesc = o; o = align_up(o + 8 * (size_t)L.capNTr);
  L.fflag = o; o = align_up(o + 4 * (size_t)L.capNTr);
  L.frag = o; o = align_up(o + sizeof(Frag) * (size_t)L.capNTr);
  L.pend = o; o = align_up(o + sizeof(Pend) * (size_t)L.capNTr);
  const size_t nb = 4 * (size_t)L.capN;
  L.lo0 = o; o = align_up(o + nb);
  L.lo1 = o; o = align_up(o + nb);
  L.hi0 = o; o = align_up(o + nb);
  L.hi1 = o; o = align_up(o + nb);
  L.id0 = o; o = align_up(o + nb);
  L.id1 = o; o = align_up(o + nb);
  L.rec = o; o = align_up(o + 16 * (size_t)L.capN);
  L.tx = o; o = align_up(o + nb);
  L.ty = o; o = align_up(o + nb);
  L.tz = o; o = align_up(o + nb);
  L.rflag = o; o = align_up(o + nb + 4);
  L.rpos = o; o = align_up(o + nb + 4);
  L.bsum = o; o = align_up(o + 4 * ((size_t)(L.capN + kScanTile - 1) / kScanTile + 1));
  L.outoff = o; o = align_up(o + 8 * (size_t)(L.capB + 1));
  L.fstat = o; o = align_up(o + 4 * (size_t)L.capB);
  L.total = o;
  return L;
}

Ws carve(const Layout& L, void* base) {
  char* b = static_cast<char*>(base);
  Ws w;
  w.hdr = reinterpret_cast<CallHdr*>(b + L.hdr);
  w.io = reinterpret_cast<Io*>(b + L.io);
  w.fd = reinterpret_cast<FrameDesc*>(b + L.fd);
  w.tpb = reinterpret_cast<uint32_t*>(b + L.tpb);
  w.tps = reinterpret_cast<uint32_t*>(b + L.tps);
  w.tinfo = reinterpret_cast<uint2*>(b + L.tinfo);
  w.tpr = reinterpret_cast<uint32_t*>(b + L.tpr);
  w.ilv_s = reinterpret_cast<uint32_t*>(b + L.ilv_s);
  w.ilv_perm = reinterpret_cast<uint32_t*>(b + L.ilv_perm);
  w.ctl = reinterpret_cast<Ctl*>(b + L.ctl);
  w.fs = reinterpret_cast<FrameState*>(b + L.fs);
  w.hist = reinterpret_cast<uint32_t*>(b + L.hist);
  w.sdesc = reinterpret_cast<uint32_t*>(b + L.sdesc);
  w.rdesc = reinterpret_cast<uint64_t*>(b + L.rdesc);
  w.fflag = reinterpret_cast<uint32_t*>(b + L.fflag);
  w.frag = reinterpret_cast<Frag*>(b + L.frag);
  w.pend = reinterpret_cast<Pend*>(b + L.pend);
  w.lo[0] = reinterpret_cast<uint32_t*>(b + L.lo0);
  w.lo[1] = reinterpret_cast<uint32_t*>(b + L.lo1);
  w.hi[0] = reinterpret_cast<uint32_t*>(b + L.hi0);
  w.hi[1] = reinterpret_cast<uint32_t*>(b + L.hi1);
  w.idx[0] = reinterpret_cast<uint32_t*>(b + L.id0);
  w.idx[1] = reinterpret_cast<uint32_t*>(b + L.id1);
  w.rec = reinterpret_cast<float4*>(b + L.rec);
  w.xf = reinterpret_cast<FrameXf*>(b + L.xf);
  w.tx = reinterpret_cast<float*>(b + L.tx);
  w.ty = reinterpret_cast<float*>(b + L.ty);
  w.tz = reinterpret_cast<float*>(b + L.tz);
  w.rflag = reinterpret_cast<uint32_t*>(b + L.rflag);
  w.rpos = reinterpret_cast<uint32_t*>(b + L.rpos);
  w.bsum = reinterpret_cast<uint32_t*>(b + L.bsum);
  w.capB = L.capB;
  w.capNTb = L.capNTb;
  w.capNTs = L.capNTs;
  w.capNTr = L.capNTr;
  w.slots = L.slots;
  w.R = L.R;
  w.capN = L.capN;
  return w;
}

// ---------------------------------------------------------- checks ----
bool leaf_inverse(float leaf, float* inv) {
  if (!std::isfinite(leaf) || !(leaf > 0.0f)) return false;
  volatile float one = 1.0f;
  float r = one / leaf;  // binary32 division, round to nearest even
  if (!std::isfinite(r)) return false;
  *inv = r;
  return true;
}

uint32_t want_mask(const vg_cells* c) {
  uint32_t w = 0;
  if (c->x && c->y && c->z) w |= kOutXYZ;
  if (c->rgb) w |= kOutRGB;
  if (c->count) w |= kOutCount;
  if (c->key) w |= kOutKey;
  if (c->point_cell) w |= kOutPointCell;
  if (c->ref_index) w |= kOutRef;
  if (c->lx && c->ly && c->lz) w |= kOutLocal;
  return w;
}

bool cells_consistent(const vg_cells* c) {
  // x/y/z and lx/ly/lz come as complete triples or not at all
  const int xyz = (c->x != nullptr) + (c->y != nullptr) + (c->z != nullptr);
  const int loc = (c->lx != nullptr) + (c->ly != nullptr) + (c->lz != nullptr);
  return (xyz == 0 || xyz == 3) && (loc == 0 || loc == 3);
}

// Fills the staged region (header, io, frame descriptors, tile prefixes) on
// the host.  Returns false if some frame is too large.
// Checks the per-frame filters (NULL: none).
bool filters_ok(const vg_filter* f, int B) {
  if (!f) return true;
  for (int b = 0; b < B; ++b) {
    if (std::isnan(f[b].z_min) || std::isnan(f[b].z_max) || f[b].z_min > f[b].z_max) return false;
    if (f[b].flags & ~(uint32_t)VG_FILTER_TRANSFORM) return false;
    if (f[b].flags & VG_FILTER_TRANSFORM) {
      for (int k = 0; k < 9; ++k)
        if (!std::isfinite(f[b].rot[k])) return false;
      for (int k = 0; k < 3; ++k)
        if (!std::isfinite(f[b].trans[k])) return false;
    }
  }
  return true;
}

bool fill_staging(char* st, const Layout& L, const Variant& v, const vg_points* p,
                  const int64_t* offs, const float* leaves, const float* invs, int B,
                  const vg_cells* out, int64_t* out_offsets, int32_t* frame_status, int key_mode,
                  int fail_waits, CallHdr* hdr_out, const Ws& ws,
                  const vg_filter* filters = nullptr, bool host_input = false) {
  CallHdr hdr;
  std::memset(&hdr, 0, sizeof hdr);
  hdr.B = B;
  hdr.key_mode = key_mode;
  hdr.N = offs[B] - offs[0];
  hdr.want = want_mask(out);
  hdr.fail_waits = fail_waits;
  if (!p->rgb) hdr.want &= ~(uint32_t)kOutRGB;
  Io io;
  std::memset(&io, 0, sizeof io);
  io.x = p->x;
  io.y = p->y;
  io.z = p->z;
  io.rgb = p->rgb;
  io.cx = out->x;
  io.cy = out->y;
  io.cz = out->z;
  io.crgb = out->rgb;
  io.count = out->count;
  io.key = out->key;
  io.point_cell = out->point_cell;
  io.ref_index = out->ref_index;
  io.lx = out->lx;
  io.ly = out->ly;
  io.lz = out->lz;
  io.out_offsets = out_offsets;
  io.frame_status = frame_status;
  // filters: the bbox pass writes the point view when some frame transforms or
  // limits its height; sparse cells go after the pipeline when some frame asks
  io.vx = p->x;
  io.vy = p->y;
  io.vz = p->z;
  if (filters) {
    FrameXf* xf = reinterpret_cast<FrameXf*>(st + L.xf);
    for (int b = 0; b < B; ++b) {
      const vg_filter& f = filters[b];
      FrameXf& x = xf[b];
      std::memset(&x, 0, sizeof x);
      if (f.flags & VG_FILTER_TRANSFORM) {
        x.on |= kXfRotate;
        for (int k = 0; k < 9; ++k) x.r[k] = f.rot[k];
        for (int k = 0; k < 3; ++k) x.t[k] = f.trans[k];
      }
      x.zlo = f.z_min;
      x.zhi = f.z_max;
      if (!(f.z_min == -INFINITY && f.z_max == INFINITY)) x.on |= kXfLimit;
      x.minp = f.min_points;
      if (x.on) hdr.filt |= kFiltView;
      if (f.min_points > 1) hdr.filt |= kFiltMinPts;
    }
    if (hdr.filt & kFiltView) {
      io.vx = ws.tx;
      io.vy = ws.ty;
      io.vz = ws.tz;
    }
    if ((hdr.filt & kFiltMinPts) && !io.count) {
      io.count = ws.rpos;  // counts for the sparse-cell pass only, not an output
      hdr.want |= kOutCount;
      hdr.filt |= kFiltCountInternal;
    }
  }
  // points in host memory: the bbox pass reads them once and writes the view
  // every later pass reads from device memory
  if (host_input) {
    if (!filters) std::memset(st + L.xf, 0, sizeof(FrameXf) * (size_t)B);
    hdr.filt |= kFiltView;
    io.vx = ws.tx;
    io.vy = ws.ty;
    io.vz = ws.tz;
  }
  FrameDesc* fd = reinterpret_cast<FrameDesc*>(st + L.fd);
  uint32_t* tpb = reinterpret_cast<uint32_t*>(st + L.tpb);
  uint32_t* tps = reinterpret_cast<uint32_t*>(st + L.tps);
  uint32_t* tpr = reinterpret_cast<uint32_t*>(st + L.tpr);
  int64_t tb = 0, ts = 0, tr = 0;
  for (int b = 0; b < B; ++b) {
    const int64_t n = offs[b + 1] - offs[b];
    if (n < 0 || n > kMaxFramePoints) return false;
    const int64_t nb = std::max<int64_t>(1, div_up(n, v.TB));
    const int64_t ns = std::max<int64_t>(1, div_up(n, v.TS));
    const int64_t nr = std::max<int64_t>(1, div_up(n, v.TR));
    fd[b].off = offs[b] - offs[0];
    fd[b].n = n;
    fd[b].leaf = leaves[b];
    fd[b].inv = invs[b];
    fd[b].tb0 = (int32_t)tb;
    fd[b].ts0 = (int32_t)ts;
    fd[b].tr0 = (int32_t)tr;
    fd[b].ntb = (int32_t)nb;
    fd[b].nts = (int32_t)ns;
    fd[b].ntr = (int32_t)nr;
    tpb[b] = (uint32_t)tb;
    tps[b] = (uint32_t)ts;
    tpr[b] = (uint32_t)tr;
    tb += nb;
    ts += ns;
    tr += nr;
  }
  tpb[B] = (uint32_t)tb;
  tps[B] = (uint32_t)ts;
  tpr[B] = (uint32_t)tr;
  if (tb > L.capNTb || ts > L.capNTs || tr > L.capNTr) return false;
  // round-robin order of the sort tiles over frames (when the tables fit)
  hdr.ilv_rounds = 0;
  if (B > 1 && B <= kIlvMaxFrames) {
    int32_t maxnt = 0;
    for (int b = 0; b < B; ++b) maxnt = std::max(maxnt, fd[b].nts);
    if (maxnt <= kIlvMaxRounds) {
      uint32_t* perm = reinterpret_cast<uint32_t*>(st + L.ilv_perm);
      uint32_t* S = reinterpret_cast<uint32_t*>(st + L.ilv_s);
      for (int b = 0; b < B; ++b) perm[b] = (uint32_t)b;
      std::stable_sort(perm, perm + B, [&](uint32_t a, uint32_t c) { return fd[a].nts > fd[c].nts; });
      int cnt = B;  // frames with more than r tiles
      S[0] = 0;
      for (int r = 0; r < maxnt; ++r) {
        while (cnt > 0 && fd[perm[cnt - 1]].nts <= r) --cnt;
        S[r + 1] = S[r] + (uint32_t)cnt;
      }
      hdr.ilv_rounds = maxnt;
    }
  }
  hdr.NTb = (int32_t)tb;
  hdr.NTs = (int32_t)ts;
  hdr.NTr = (int32_t)tr;
  std::memcpy(st + L.hdr, &hdr, sizeof hdr);
  std::memcpy(st + L.io, &io, sizeof io);
  *hdr_out = hdr;
  return true;
}

// Enqueues: staged copy, state reset, pipeline.  All launches have fixed
// shapes (no per-call kernel arguments), so the sequence can be captured.
// Radix passes launched one by one; later passes share a launch.
constexpr int kOwnPasses = 3;

// Optional per-launch timing: an event pair around every kernel launch.
struct LaunchTimer {
  static constexpr int kMax = 32;
  hipEvent_t ev[2 * kMax] = {};
  int kind[kMax] = {};
  int n = 0;
  bool ok = false;
  bool init() {
    for (int i = 0; i < 2 * kMax; ++i)
      if (hipEventCreate(&ev[i]) != hipSuccess) return false;
    ok = true;
    return true;
  }
  void release() {
    for (int i = 0; i < 2 * kMax; ++i)
      if (ev[i]) (void)hipEventDestroy(ev[i]);
  }
};

vg_kernel_kind kind_of_phase(const Variant& v, int lo, int hi) {
  if (hi - lo > 1) return (lo >= 2 && hi <= v.ph_red) ? VG_KERNEL_SORT : VG_KERNEL_PIPELINE;
  if (lo == 0) return VG_KERNEL_BBOX;
  if (lo == 1) return VG_KERNEL_HIST;
  if (lo == v.ph_red) return VG_KERNEL_REDUCE;
  if (lo == v.ph_red + 1) return VG_KERNEL_FIXUP;
  return VG_KERNEL_SORT;
}

// Enqueues: staged copy, state reset, pipeline.  All launches have fixed
// shapes (no per-call kernel arguments), so the sequence can be captured.
vg_status enqueue_kernels(const Variant& v, const Ws& ws, int exec_mode, int cus, int bpc,
                          hipStream_t s, LaunchTimer* tm = nullptr, bool sparse = false);

vg_status enqueue(const Variant& v, const Layout& L, const Ws& ws, const char* staging,
                  int exec_mode, int cus, int bpc, hipStream_t s, LaunchTimer* tm = nullptr,
                  bool sparse = false) {
  if (hipMemcpyAsync(ws.hdr, staging, L.staged, hipMemcpyHostToDevice, s) != hipSuccess)
    return VG_ERR_DEVICE;
  return enqueue_kernels(v, ws, exec_mode, cus, bpc, s, tm, sparse);
}

// The sparse-cell pass (launched when a call asks for a minimum of points per
// cell; its kernels read the call header and exit at once otherwise).
void enqueue_sparse(const Ws& ws, hipStream_t s) {
  const int64_t N = ws.capN;
  const int g = (int)std::max<int64_t>(1, std::min<int64_t>((N + kSparseBlock - 1) / kSparseBlock, 4096));
  const int nb = (int)((N + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(vg_sparse_flag_kernel, dim3(g), dim3(kSparseBlock), 0, s, ws);
  hipLaunchKernelGGL(vg_scan_tiles, dim3(nb), dim3(kScanBlock), 0, s, ws.rflag, &ws.ctl->rows,
                     ws.bsum);
  hipLaunchKernelGGL(vg_scan_top, dim3(1), dim3(1024), 0, s, &ws.ctl->rows, ws.bsum,
                     &ws.ctl->rows_kept);
  hipLaunchKernelGGL(vg_scan_apply, dim3(nb), dim3(kScanBlock), 0, s, ws.rflag, &ws.ctl->rows,
                     ws.bsum, ws.rpos, nullptr, &ws.ctl->rows_kept);
  hipLaunchKernelGGL(vg_sparse_gather_kernel, dim3(g), dim3(kSparseBlock), 0, s, ws);
  hipLaunchKernelGGL(vg_sparse_scatter_kernel, dim3(g), dim3(kSparseBlock), 0, s, ws);
}

// State reset, pipeline, status (the staged region must already be on its way).
vg_status enqueue_kernels(const Variant& v, const Ws& ws, int exec_mode, int cus, int bpc,
                          hipStream_t s, LaunchTimer* tm, bool sparse) {
  if (tm) tm->n = 0;
  auto mark = [&](int k, int which) {
    if (tm && tm->n < LaunchTimer::kMax) {
      tm->kind[tm->n] = k;
      (void)hipEventRecord(tm->ev[2 * tm->n + which], s);
      if (which) ++tm->n;
    }
  };
  mark(VG_KERNEL_INIT, 0);
  hipLaunchKernelGGL(vg_init_kernel, dim3(256), dim3(256), 0, s, ws);
  mark(VG_KERNEL_INIT, 1);
  if (exec_mode == VG_EXEC_PERSISTENT) {
    mark(VG_KERNEL_PIPELINE, 0);
    v.launch(ws, 0, v.nph, cus, bpc, s);
    mark(VG_KERNEL_PIPELINE, 1);
  } else {
    // one launch per phase, except that the radix passes from kOwnPasses on
    // (keys of more than 24 bits with 8-bit digits) share one launch, which
    // ends at once when no frame needs them
    for (int ph = 0; ph < v.nph;) {
      const int hi = (ph == 2 + kOwnPasses && v.ph_red > ph + 1) ? v.ph_red : ph + 1;
      const int k = kind_of_phase(v, ph, hi);
      mark(k, 0);
      v.launch(ws, ph, hi, cus, bpc, s);
      mark(k, 1);
      ph = hi;
    }
  }
  if (sparse) enqueue_sparse(ws, s);
  hipLaunchKernelGGL(vg_status_kernel, dim3(1), dim3(256), 0, s, ws);
  if (hipGetLastError() != hipSuccess) return VG_ERR_DEVICE;
  return VG_OK;
}

// Per host thread pinned staging for the synchronous single-cloud path.
struct ThreadStaging {
  char* buf = nullptr;
  size_t bytes = 0;
  ~ThreadStaging() {
    if (buf) (void)hipHostFree(buf);
  }
  char* get(size_t need) {
    if (bytes < need) {
      if (buf) (void)hipHostFree(buf);
      buf = nullptr;
      bytes = 0;
      if (hipHostMalloc(reinterpret_cast<void**>(&buf), need, hipHostMallocDefault) != hipSuccess)
        return nullptr;
      bytes = need;
    }
    return buf;
  }
};
thread_local ThreadStaging t_staging;

struct Readback {
  int64_t off[2];
  int32_t status;
  uint32_t error;
};

}  // namespace

// ================================================================ C ABI ====
extern "C" {

const char* vg_status_string(vg_status s) {
  switch (s) {
    case VG_OK: return "VG_OK";
    case VG_ERR_ARG: return "VG_ERR_ARG: invalid argument";
    case VG_ERR_LEAF: return "VG_ERR_LEAF: leaf must be finite and > 0 with a finite reciprocal";
    case VG_ERR_GRID_OVERFLOW: return "VG_ERR_GRID_OVERFLOW: more than 2^21 cells on an axis";
    case VG_ERR_WORKSPACE: return "VG_ERR_WORKSPACE: workspace too small";
    case VG_ERR_DEVICE: return "VG_ERR_DEVICE: HIP runtime error or device time-out";
  }
  return "VG_ERR_UNKNOWN";
}

vg_status vg_default_tuning(vg_tuning* t) {
  if (!t) return VG_ERR_ARG;
  *t = kDefaultTuning;
  return VG_OK;
}

vg_status vg_tuning_supported(const vg_tuning* t) {
  return (t && find_variant(t)) ? VG_OK : VG_ERR_ARG;
}

size_t vg_workspace_bytes(int64_t n_total, int n_frames, const vg_tuning* t) {
  const Variant* v = find_variant(t);
  if (!v || n_total < 0 || n_total > INT32_MAX || n_frames < 1) return 0;
  return make_layout(n_total, n_frames, *v).total;
}

}  // extern "C"

namespace {

// One cloud, optionally filtered (filter NULL: none).
vg_status downsample_one(const vg_points* p, int64_t n, float leaf, const vg_filter* filter,
                         vg_cells* out, int64_t* m, const vg_options* o) {
  if (m) *m = 0;
  if (!p || !out || !m || !o) return VG_ERR_ARG;
  if (!filters_ok(filter, 1)) return VG_ERR_ARG;
  if (n < 0 || n > kMaxFramePoints) return VG_ERR_ARG;
  if (o->key_mode != VG_KEY_LINEAR && o->key_mode != VG_KEY_MORTON) return VG_ERR_ARG;
  if (n > 0 && (!p->x || !p->y || !p->z)) return VG_ERR_ARG;
  if (!cells_consistent(out)) return VG_ERR_ARG;
  const Variant* v = find_variant(o->tuning);
  if (!v) return VG_ERR_ARG;
  float inv;
  if (!leaf_inverse(leaf, &inv)) return VG_ERR_LEAF;
  if (n == 0) return VG_OK;
  const Layout L = make_layout(n, 1, *v);
  if (o->workspace && o->workspace_bytes < L.total) return VG_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(o->stream);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return VG_ERR_DEVICE;
  const int cus = device_cus(dev);
  if (cus <= 0) return VG_ERR_DEVICE;
  const int bpc = o->tuning ? o->tuning->blocks_per_cu : 0;

  char* st = t_staging.get(L.staged + sizeof(Readback));
  if (!st) return VG_ERR_DEVICE;
  void* base = o->workspace;
  bool owned = false;
  if (!base) {
    if (hipMalloc(&base, L.total) != hipSuccess) return VG_ERR_DEVICE;
    owned = true;
  }
  Ws ws = carve(L, base);
  const int64_t offs[2] = {0, n};
  CallHdr hdr;
  int64_t* d_off = reinterpret_cast<int64_t*>(static_cast<char*>(base) + L.outoff);
  int32_t* d_st = reinterpret_cast<int32_t*>(static_cast<char*>(base) + L.fstat);
  vg_status rc = VG_OK;
  bool enqueued = false;
  if (!fill_staging(st, L, *v, p, offs, &leaf, &inv, 1, out, d_off, d_st, o->key_mode, 0, &hdr, ws,
                    filter)) {
    rc = VG_ERR_ARG;
  } else {
    const int mode = o->tuning ? o->tuning->exec_mode : kDefaultTuning.exec_mode;
    enqueued = true;
    rc = enqueue(*v, L, ws, st, mode, cus, bpc, s, nullptr, (hdr.filt & kFiltMinPts) != 0);
  }
  Readback* rb = reinterpret_cast<Readback*>(st + L.staged);
  if (rc == VG_OK) {
    bool ok = hipMemcpyAsync(&rb->off[0], d_off, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s) ==
                  hipSuccess &&
              hipMemcpyAsync(&rb->status, d_st, sizeof(int32_t), hipMemcpyDeviceToHost, s) ==
                  hipSuccess &&
              hipMemcpyAsync(&rb->error, &ws.ctl->error, sizeof(uint32_t), hipMemcpyDeviceToHost,
                             s) == hipSuccess &&
              hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
      rc = VG_ERR_DEVICE;
    } else if (rb->error) {
      rc = VG_ERR_DEVICE;
    } else if (rb->status == kFrameOverflow) {
      rc = VG_ERR_GRID_OVERFLOW;
    } else if (rb->status != kFrameOk) {
      rc = VG_ERR_DEVICE;
    } else {
      *m = rb->off[1] - rb->off[0];
    }
  }
  // On an error after something was enqueued, the staged copy may still be
  // reading this thread's pinned buffer, and the kernels the workspace: wait
  // before either can be reused.
  if (owned || (enqueued && rc != VG_OK)) (void)hipStreamSynchronize(s);
  if (owned) (void)hipFree(base);
  return rc;
}

}  // namespace

extern "C" {

vg_status vg_downsample_ex(const vg_points* p, int64_t n, float leaf, vg_cells* out, int64_t* m,
                           const vg_options* o) {
  return downsample_one(p, n, leaf, nullptr, out, m, o);
}

vg_status vg_downsample_filtered(const vg_points* p, int64_t n, float leaf, const vg_filter* f,
                                 vg_cells* out, int64_t* m, const vg_options* o) {
  if (m) *m = 0;
  if (!f) return VG_ERR_ARG;
  return downsample_one(p, n, leaf, f, out, m, o);
}

vg_status vg_downsample(const vg_points* p, int64_t n, float leaf, vg_cells* out, int64_t* m) {
  vg_options o;
  std::memset(&o, 0, sizeof o);
  o.key_mode = VG_KEY_LINEAR;
  return vg_downsample_ex(p, n, leaf, out, m, &o);
}

vg_status vg_downsample_backward(const float* gx, const float* gy, const float* gz,
                                 const uint32_t* count, int64_t m, const int32_t* point_cell,
                                 int64_t n, float* dx, float* dy, float* dz, void* stream) {
  if (n < 0 || n > INT32_MAX || m < 0) return VG_ERR_ARG;
  if (n == 0) return VG_OK;
  if (!point_cell || !dx || !dy || !dz) return VG_ERR_ARG;
  if (m > 0 && (!gx || !gy || !gz || !count)) return VG_ERR_ARG;
  const int block = 256;
  const int64_t blocks = std::min<int64_t>(div_up(n, block), 8192);
  hipLaunchKernelGGL(vg_backward_kernel, dim3((unsigned)blocks), dim3(block), 0,
                     static_cast<hipStream_t>(stream), gx, gy, gz, count, m, point_cell, n, dx, dy,
                     dz);
  return hipGetLastError() == hipSuccess ? VG_OK : VG_ERR_DEVICE;
}

}  // extern "C"

// ==================================== neighbour-bucket decimation ====
namespace {

struct NbdLayout {
  size_t ckey, ccount, pcell, ctl, seg, cursor, bsum, sx, sy, sz, sidx, scell, rng, cnt, alive,
      cand, del, mlog, keep, kpos, total;
  uint32_t log_cap;
  int scan_blocks;
};

// After the pipeline's own layout (which starts at 0).
NbdLayout make_nbd_layout(size_t o, int64_t n, int64_t round_size) {
  NbdLayout L;
  const size_t N = (size_t)std::max<int64_t>(n, 1);
  const size_t K = (size_t)std::max<int64_t>(1, std::min<int64_t>(round_size, (int64_t)N));
  L.scan_blocks = (int)((N + kScanTile - 1) / kScanTile);
  L.log_cap = (uint32_t)std::min<int64_t>((int64_t)N / (int64_t)K + 2, (int64_t)1 << 24);
  o = align_up(o);
  L.ckey = o;   o = align_up(o + 8 * N);
  L.ccount = o; o = align_up(o + 4 * N);
  L.pcell = o;  o = align_up(o + 4 * N);
  L.ctl = o;    o = align_up(o + sizeof(NbdCtl));
  L.seg = o;    o = align_up(o + 4 * (N + 1));
  L.cursor = o; o = align_up(o + 4 * N);
  L.bsum = o;   o = align_up(o + 4 * ((size_t)L.scan_blocks + 1));
  L.sx = o;     o = align_up(o + 4 * N);
  L.sy = o;     o = align_up(o + 4 * N);
  L.sz = o;     o = align_up(o + 4 * N);
  L.sidx = o;   o = align_up(o + 4 * N);
  L.scell = o;  o = align_up(o + 4 * N);
  L.rng = o;    o = align_up(o + 8 * 9 * N);
  L.cnt = o;    o = align_up(o + 4 * N);
  L.alive = o;  o = align_up(o + N);
  L.cand = o;   o = align_up(o + sizeof(NbdCand) * N);
  L.del = o;    o = align_up(o + 4 * K);
  L.mlog = o;   o = align_up(o + 8 * (size_t)L.log_cap);
  L.keep = o;   o = align_up(o + 4 * N);
  L.kpos = o;   o = align_up(o + 4 * (N + 1));
  L.total = o;
  return L;
}

struct NbdReadback {
  uint32_t round, done, marked;  // the same order as in NbdCtl: copied together
  uint32_t nkeep;
  int32_t status;
};

int grid_for(int64_t items, int per_block, int cap) {
  const int64_t b = (items + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

}  // namespace

extern "C" {

size_t vg_nbd_workspace_bytes(int64_t n, int32_t round_size) {
  if (n < 0 || n > kMaxFramePoints || round_size < 1) return 0;
  const Variant* v = find_variant(nullptr);
  const Layout L = make_layout(std::max<int64_t>(n, 1), 1, *v);
  return make_nbd_layout(L.total, n, round_size).total;
}

vg_status vg_nbd_decimate(const vg_points* p, int64_t n, const vg_nbd_params* prm,
                          vg_nbd_out* out, int64_t* n_keep, int64_t* rounds,
                          const vg_options* o) {
  if (n_keep) *n_keep = 0;
  if (rounds) *rounds = 0;
  if (!p || !prm || !out || !n_keep || !rounds) return VG_ERR_ARG;
  if (n < 0 || n > kMaxFramePoints) return VG_ERR_ARG;
  if (n > 0 && (!p->x || !p->y || !p->z)) return VG_ERR_ARG;
  if (out->marked_cap < 0 || (out->marked_cap > 0 && !out->marked)) return VG_ERR_ARG;
  const int nxyz = (out->x != nullptr) + (out->y != nullptr) + (out->z != nullptr);
  if (nxyz != 0 && nxyz != 3) return VG_ERR_ARG;
  if (prm->round_size < 1) return VG_ERR_ARG;
  float inv;
  if (!leaf_inverse(prm->leaf, &inv)) return VG_ERR_LEAF;
  if (!std::isfinite(prm->radius) || !(prm->radius > 0.0f) || !(prm->radius <= prm->leaf))
    return VG_ERR_ARG;
  const vg_tuning* tuning = o ? o->tuning : nullptr;
  const Variant* v = find_variant(tuning);
  if (!v) return VG_ERR_ARG;
  if (n == 0) {
    *rounds = 1;  // one round that marks nothing
    if (out->marked_cap > 0) out->marked[0] = 0;
    return VG_OK;
  }
  const Layout L = make_layout(n, 1, *v);
  const NbdLayout NL = make_nbd_layout(L.total, n, prm->round_size);
  if (o && o->workspace && o->workspace_bytes < NL.total) return VG_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(o ? o->stream : nullptr);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return VG_ERR_DEVICE;
  const int cus = device_cus(dev);
  if (cus <= 0) return VG_ERR_DEVICE;
  const int bpc = tuning ? tuning->blocks_per_cu : 0;
  char* st = t_staging.get(L.staged + sizeof(NbdReadback));
  if (!st) return VG_ERR_DEVICE;
  void* base = o ? o->workspace : nullptr;
  bool owned = false;
  if (!base) {
    if (hipMalloc(&base, NL.total) != hipSuccess) return VG_ERR_DEVICE;
    owned = true;
  }
  char* b = static_cast<char*>(base);
  Ws ws = carve(L, base);
  NbdWs w;
  w.ctl = reinterpret_cast<NbdCtl*>(b + NL.ctl);
  w.x = p->x;
  w.y = p->y;
  w.z = p->z;
  w.rgb = p->rgb;
  w.n = n;
  w.ckey = reinterpret_cast<uint64_t*>(b + NL.ckey);
  w.ccount = reinterpret_cast<uint32_t*>(b + NL.ccount);
  w.pcell = reinterpret_cast<int32_t*>(b + NL.pcell);
  w.seg = reinterpret_cast<uint32_t*>(b + NL.seg);
  w.cursor = reinterpret_cast<uint32_t*>(b + NL.cursor);
  w.bsum = reinterpret_cast<uint32_t*>(b + NL.bsum);
  w.sx = reinterpret_cast<float*>(b + NL.sx);
  w.sy = reinterpret_cast<float*>(b + NL.sy);
  w.sz = reinterpret_cast<float*>(b + NL.sz);
  w.sidx = reinterpret_cast<uint32_t*>(b + NL.sidx);
  w.scell = reinterpret_cast<uint32_t*>(b + NL.scell);
  w.rng = reinterpret_cast<uint2*>(b + NL.rng);
  w.cnt = reinterpret_cast<uint32_t*>(b + NL.cnt);
  w.alive = reinterpret_cast<uint8_t*>(b + NL.alive);
  w.cand = reinterpret_cast<NbdCand*>(b + NL.cand);
  w.del = reinterpret_cast<uint32_t*>(b + NL.del);
  w.marked_log = reinterpret_cast<int64_t*>(b + NL.mlog);
  w.keep = reinterpret_cast<uint32_t*>(b + NL.keep);
  w.kpos = reinterpret_cast<uint32_t*>(b + NL.kpos);
  w.count0 = out->count0;
  w.keep_index = out->keep_index;
  w.ox = out->x;
  w.oy = out->y;
  w.oz = out->z;
  w.orgb = p->rgb ? out->rgb : nullptr;

  // 1. the voxel pipeline: cell keys (linear), counts, every point's cell
  vg_points pin = *p;
  pin.rgb = nullptr;
  vg_cells cells;
  std::memset(&cells, 0, sizeof cells);
  cells.key = w.ckey;
  cells.count = w.ccount;
  cells.point_cell = w.pcell;
  const int64_t offs[2] = {0, n};
  const float leaf = prm->leaf;
  int64_t* d_off = reinterpret_cast<int64_t*>(b + L.outoff);
  int32_t* d_st = reinterpret_cast<int32_t*>(b + L.fstat);
  CallHdr hdr;
  vg_status rc = VG_OK;
  bool enqueued = false;
  if (!fill_staging(st, L, *v, &pin, offs, &leaf, &inv, 1, &cells, d_off, d_st, VG_KEY_LINEAR, 0,
                    &hdr, ws)) {
    rc = VG_ERR_ARG;
  } else {
    enqueued = true;
    rc = enqueue(*v, L, ws, st, tuning ? tuning->exec_mode : kDefaultTuning.exec_mode, cus, bpc, s);
  }
  NbdReadback* rb = reinterpret_cast<NbdReadback*>(st + L.staged);
  if (rc == VG_OK) {
    // 2. buckets, neighbour ranges, counts
    volatile float rr = prm->radius;
    const float r2 = rr * rr;  // binary32, round to nearest even
    const int nb = NL.scan_blocks;
    hipLaunchKernelGGL(nbd_setup_kernel, dim3(grid_for(n, kNbdBlock, 1024)), dim3(kNbdBlock), 0, s,
                       ws, w, prm->umbral, (uint32_t)prm->round_size, prm->seed, r2, NL.log_cap,
                       (prm->flags & VG_NBD_EXACT_SELECT) ? 1u : 0u);
    hipLaunchKernelGGL(vg_scan_tiles, dim3(nb), dim3(kScanBlock), 0, s, w.ccount, &w.ctl->m, w.bsum);
    hipLaunchKernelGGL(vg_scan_top, dim3(1), dim3(1024), 0, s, &w.ctl->m, w.bsum,
                       &w.ctl->scan_total);
    hipLaunchKernelGGL(vg_scan_apply, dim3(nb), dim3(kScanBlock), 0, s, w.ccount, &w.ctl->m,
                       w.bsum, w.seg, w.cursor, &w.ctl->scan_total);
    const int gp = grid_for(n, kNbdBlock, 8192);
    hipLaunchKernelGGL(nbd_scatter_kernel, dim3(gp), dim3(kNbdBlock), 0, s, w);
    hipLaunchKernelGGL(nbd_ranges_kernel, dim3(gp), dim3(kNbdBlock), 0, s, w);
    hipLaunchKernelGGL(nbd_count_kernel, dim3(gp), dim3(kNbdBlock), 0, s, w);
    // 3. rounds, enqueued in batches ahead of the host's look at the done flag
    //    (the round kernel's LDS allows one workgroup per CU; a workgroup
    //    collects kCollectItems * kPickBlock points per step)
    const int gr = grid_for(n, kCollectItems * kPickBlock, cus);
    const int gd = grid_for(std::min<int64_t>(prm->round_size, n), kNbdBlock / 64, 2048);
    // every round but the last deletes round_size marked points, so a round
    // count of marked / round_size + 1 is enough for what is left: the next
    // batch holds that many (at most 64), and few launches run after the last
    // round
    const int64_t max_rounds = n / prm->round_size + 2;
    int64_t issued = 0;
    int batch = 8;
    for (;;) {
      for (int r = 0; r < batch; ++r) {
        hipLaunchKernelGGL(nbd_round_kernel, dim3(gr), dim3(kPickBlock), 0, s, w);
        hipLaunchKernelGGL(nbd_decrement_kernel, dim3(gd), dim3(kNbdBlock), 0, s, w);
      }
      issued += batch;
      if (hipMemcpyAsync(&rb->round, &w.ctl->round, 3 * sizeof(uint32_t), hipMemcpyDeviceToHost,
                         s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        rc = VG_ERR_DEVICE;
        break;
      }
      if (rb->done) break;
      if (issued > max_rounds) {  // every round but the last deletes round_size points
        rc = VG_ERR_DEVICE;
        break;
      }
      batch = (int)std::min<int64_t>(64, (int64_t)rb->marked / prm->round_size + 1);
    }
  }
  if (rc == VG_OK) {
    // 4. survivors in input order
    hipLaunchKernelGGL(nbd_keep_kernel, dim3(grid_for(n, kNbdBlock, 8192)), dim3(kNbdBlock), 0, s, w);
    const int nb = NL.scan_blocks;
    hipLaunchKernelGGL(vg_scan_tiles, dim3(nb), dim3(kScanBlock), 0, s, w.keep, &w.ctl->n_in, w.bsum);
    hipLaunchKernelGGL(vg_scan_top, dim3(1), dim3(1024), 0, s, &w.ctl->n_in, w.bsum,
                       &w.ctl->scan_total);
    hipLaunchKernelGGL(vg_scan_apply, dim3(nb), dim3(kScanBlock), 0, s, w.keep, &w.ctl->n_in,
                       w.bsum, w.kpos, nullptr, &w.ctl->scan_total);
    hipLaunchKernelGGL(nbd_emit_kernel, dim3(grid_for(n, kNbdBlock, 8192)), dim3(kNbdBlock), 0, s, w);
    const bool ok =
        hipGetLastError() == hipSuccess &&
        hipMemcpyAsync(&rb->round, &w.ctl->round, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s) ==
            hipSuccess &&
        hipMemcpyAsync(&rb->nkeep, &w.ctl->scan_total, sizeof(uint32_t), hipMemcpyDeviceToHost,
                       s) == hipSuccess &&
        hipMemcpyAsync(&rb->status, &w.ctl->status, sizeof(int32_t), hipMemcpyDeviceToHost, s) ==
            hipSuccess &&
        hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
      rc = VG_ERR_DEVICE;
    } else if (rb->status == kFrameOverflow) {
      rc = VG_ERR_GRID_OVERFLOW;
    } else if (rb->status != kFrameOk) {
      rc = VG_ERR_DEVICE;
    } else {
      const int64_t nr = rb->round;
      const int64_t nl = std::min<int64_t>(std::min<int64_t>(nr, out->marked_cap), NL.log_cap);
      if (nl > 0 && (hipMemcpy(out->marked, w.marked_log, (size_t)nl * sizeof(int64_t),
                               hipMemcpyDeviceToHost) != hipSuccess))
        rc = VG_ERR_DEVICE;
      *n_keep = rb->nkeep;
      *rounds = nr;
    }
  }
  if (owned || (enqueued && rc != VG_OK)) (void)hipStreamSynchronize(s);
  if (owned) (void)hipFree(base);
  return rc;
}

}  // extern "C"

// ============================================ calls that cannot allocate ====
// The workspace of vg_downsample_noalloc: one fixed array per device, held
// until the process ends.  Host code uses the device address that
// hipGetSymbolAddress returns for it (scratch_base), never the array's name.
static __device__ __align__(256) unsigned char scratch[VG_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
void* g_scratch[64];

// Device address of this device's scratch array (looked up once per device,
// with that device current).
void* scratch_base(int dev) {
  if (dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

}  // namespace

extern "C" {

vg_status vg_downsample_noalloc(const vg_points* p, int64_t n, float leaf, vg_key_mode key_mode,
                                vg_cells* out, int64_t* d_m, int32_t* d_status, void* stream) {
  if (!p || !out || !d_m || !d_status) return VG_ERR_ARG;
  if (n < 0 || (key_mode != VG_KEY_LINEAR && key_mode != VG_KEY_MORTON)) return VG_ERR_ARG;
  if (n > VG_NOALLOC_MAX_POINTS) return VG_ERR_WORKSPACE;
  if (n > 0 && (!p->x || !p->y || !p->z)) return VG_ERR_ARG;
  if (!cells_consistent(out)) return VG_ERR_ARG;
  float inv;
  if (!leaf_inverse(leaf, &inv)) return VG_ERR_LEAF;
  const Variant* v = find_variant(nullptr);
  const Layout L = make_layout(std::max<int64_t>(n, 1), 1, *v);
  if (L.total > sizeof(scratch) || L.staged > 8192) return VG_ERR_WORKSPACE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return VG_ERR_DEVICE;
  const int cus = device_cus(dev);
  void* base = scratch_base(dev);
  if (cus <= 0 || !base) return VG_ERR_DEVICE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Ws ws = carve(L, base);
  // the staged region is built on the host as for the other calls, then
  // passed by value to a one-thread kernel (no host buffer, no copy)
  alignas(16) char st[8192];
  const int64_t offs[2] = {0, n};
  int64_t* w_off = reinterpret_cast<int64_t*>(static_cast<char*>(base) + L.outoff);
  int32_t* w_st = reinterpret_cast<int32_t*>(static_cast<char*>(base) + L.fstat);
  CallHdr hdr;
  if (!fill_staging(st, L, *v, p, offs, &leaf, &inv, 1, out, w_off, w_st, key_mode, 0, &hdr, ws))
    return VG_ERR_ARG;
  StageArgs a;
  std::memcpy(&a.hdr, st + L.hdr, sizeof a.hdr);
  std::memcpy(&a.io, st + L.io, sizeof a.io);
  std::memcpy(&a.fd, st + L.fd, sizeof a.fd);
  for (int k = 0; k < 2; ++k) {
    a.tp[0][k] = reinterpret_cast<const uint32_t*>(st + L.tpb)[k];
    a.tp[1][k] = reinterpret_cast<const uint32_t*>(st + L.tps)[k];
    a.tp[2][k] = reinterpret_cast<const uint32_t*>(st + L.tpr)[k];
  }
  hipLaunchKernelGGL(vg_stage_kernel, dim3(1), dim3(64), 0, s, ws, a);
  vg_status rc = enqueue_kernels(*v, ws, kDefaultTuning.exec_mode, cus, 0, s);
  hipLaunchKernelGGL(vg_result_kernel, dim3(1), dim3(64), 0, s, ws, d_m, d_status);
  if (rc == VG_OK && hipGetLastError() != hipSuccess) rc = VG_ERR_DEVICE;
  return rc;
}

}  // extern "C"

// ============================================================ batches ====
struct vg_batch_plan {
  int max_frames;
  int64_t max_points;
  int key_mode;
  vg_tuning tuning;
  const Variant* v;
  Layout L;
  void* ws_base;
  Ws ws;
  // Two staging slots: call k fills slot k & 1 (pinned descriptor block) and
  // replays that slot's graph, so the host waits only for call k - 2 before
  // it rewrites the slot, and call k + 1 can be enqueued while call k runs.
  // Calls share the workspace: each call's stream first waits for the call
  // before it (on the device).
  char* staging[2];    // pinned
  float* invs;         // host scratch [max_frames]
  int device;
  int cus;
  hipEvent_t done[2];
  bool pending[2];
  uint64_t calls;      // calls so far
  int use_graph;
  hipGraph_t graph[2];
  hipGraphExec_t gexec[2];
  LaunchTimer* timer;  // non-null while timing is on
  int fail_waits;      // test support: calls start with the time-out flag raised
  bool graph_sparse[2];  // the slot's captured graph holds the sparse-cell pass
  bool host_input;     // the points of later calls are in mapped host memory
};

namespace {

// Waits on the host for every call of the plan still in flight.
vg_status plan_wait_all(vg_batch_plan* P) {
  for (int k = 0; k < 2; ++k) {
    if (P->pending[k]) {
      if (hipEventSynchronize(P->done[k]) != hipSuccess) return VG_ERR_DEVICE;
      P->pending[k] = false;
    }
  }
  return VG_OK;
}

}  // namespace

extern "C" {

vg_status vg_batch_plan_create(int max_frames, int64_t max_total_points, vg_key_mode key_mode,
                               const vg_tuning* tuning, vg_batch_plan** plan) {
  if (!plan) return VG_ERR_ARG;
  *plan = nullptr;
  if (max_frames < 1 || max_frames > (1 << 20)) return VG_ERR_ARG;
  if (max_total_points < 0 || max_total_points > INT32_MAX) return VG_ERR_ARG;
  if (key_mode != VG_KEY_LINEAR && key_mode != VG_KEY_MORTON) return VG_ERR_ARG;
  const Variant* v = find_variant(tuning);
  if (!v) return VG_ERR_ARG;
  vg_batch_plan* P = new (std::nothrow) vg_batch_plan();
  if (!P) return VG_ERR_DEVICE;
  P->max_frames = max_frames;
  P->max_points = max_total_points;
  P->key_mode = key_mode;
  P->tuning = tuning ? *tuning : kDefaultTuning;
  P->v = v;
  P->L = make_layout(max_total_points, max_frames, *v);
  P->ws_base = nullptr;
  P->invs = nullptr;
  P->calls = 0;
  P->use_graph = 0;
  for (int k = 0; k < 2; ++k) {
    P->staging[k] = nullptr;
    P->pending[k] = false;
    P->graph[k] = nullptr;
    P->gexec[k] = nullptr;
    P->done[k] = nullptr;
    P->graph_sparse[k] = false;
  }
  P->timer = nullptr;
  P->fail_waits = 0;
  P->host_input = false;
  vg_status rc = VG_OK;
  if (hipGetDevice(&P->device) != hipSuccess) rc = VG_ERR_DEVICE;
  if (rc == VG_OK && (P->cus = device_cus(P->device)) <= 0) rc = VG_ERR_DEVICE;
  if (rc == VG_OK && hipMalloc(&P->ws_base, P->L.total) != hipSuccess) rc = VG_ERR_DEVICE;
  for (int k = 0; k < 2; ++k) {
    if (rc == VG_OK && hipHostMalloc(reinterpret_cast<void**>(&P->staging[k]), P->L.staged,
                                     hipHostMallocDefault) != hipSuccess)
      rc = VG_ERR_DEVICE;
    if (rc == VG_OK && hipEventCreateWithFlags(&P->done[k], hipEventDisableTiming) != hipSuccess)
      rc = VG_ERR_DEVICE;
  }
  if (rc == VG_OK) {
    P->invs = new (std::nothrow) float[max_frames];
    if (!P->invs) rc = VG_ERR_DEVICE;
  }
  if (rc != VG_OK) {
    vg_batch_plan_destroy(P);
    return rc;
  }
  P->ws = carve(P->L, P->ws_base);
  *plan = P;
  return VG_OK;
}

vg_status vg_batch_plan_set_graph(vg_batch_plan* plan, int use_graph) {
  if (!plan) return VG_ERR_ARG;
  plan->use_graph = use_graph ? 1 : 0;
  return VG_OK;
}

vg_status vg_batch_plan_set_host_input(vg_batch_plan* plan, int on) {
  if (!plan) return VG_ERR_ARG;
  plan->host_input = on != 0;
  return VG_OK;
}

vg_status vg_host_alloc(size_t bytes, void** host, void** device) {
  if (!host || !device) return VG_ERR_ARG;
  *host = nullptr;
  *device = nullptr;
  void* h = nullptr;
  if (hipHostMalloc(&h, bytes ? bytes : 1, hipHostMallocMapped | hipHostMallocPortable) !=
      hipSuccess)
    return VG_ERR_DEVICE;
  void* d = nullptr;
  if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess || !d) {
    (void)hipHostFree(h);
    return VG_ERR_DEVICE;
  }
  *host = h;
  *device = d;
  return VG_OK;
}

vg_status vg_host_free(void* host) {
  if (!host) return VG_ERR_ARG;
  return hipHostFree(host) == hipSuccess ? VG_OK : VG_ERR_DEVICE;
}

vg_status vg_batch_plan_set_fail_waits(vg_batch_plan* plan, int enable) {
  if (!plan) return VG_ERR_ARG;
  plan->fail_waits = enable ? 1 : 0;
  return VG_OK;
}

vg_status vg_batch_plan_set_timing(vg_batch_plan* plan, int enable) {
  if (!plan) return VG_ERR_ARG;
  if (plan_wait_all(plan) != VG_OK) return VG_ERR_DEVICE;
  if (!enable) {
    if (plan->timer) {
      plan->timer->release();
      delete plan->timer;
      plan->timer = nullptr;
    }
    return VG_OK;
  }
  if (plan->timer) return VG_OK;
  LaunchTimer* t = new (std::nothrow) LaunchTimer();
  if (!t) return VG_ERR_DEVICE;
  if (!t->init()) {
    t->release();
    delete t;
    return VG_ERR_DEVICE;
  }
  plan->timer = t;
  return VG_OK;
}

vg_status vg_batch_plan_kernel_times(vg_batch_plan* plan, int* kinds, float* ms, int cap,
                                     int* count) {
  if (!plan || !count || cap < 0 || (cap > 0 && (!kinds || !ms))) return VG_ERR_ARG;
  *count = 0;
  if (!plan->timer) return VG_ERR_ARG;
  LaunchTimer* t = plan->timer;
  if (t->n > 0 && hipEventSynchronize(t->ev[2 * t->n - 1]) != hipSuccess) return VG_ERR_DEVICE;
  const int n = std::min(t->n, cap);
  for (int i = 0; i < n; ++i) {
    float v = 0.f;
    if (hipEventElapsedTime(&v, t->ev[2 * i], t->ev[2 * i + 1]) != hipSuccess) return VG_ERR_DEVICE;
    kinds[i] = t->kind[i];
    ms[i] = v;
  }
  *count = n;
  return VG_OK;
}

}  // extern "C"

namespace {

vg_status downsample_batch(vg_batch_plan* P, const vg_points* p, const int64_t* offs,
                           const float* leaf, const vg_filter* filters, int B, vg_cells* out,
                           int64_t* out_offsets, int32_t* frame_status, void* stream) {
  if (!P || !p || !offs || !leaf || !out || !out_offsets || !frame_status) return VG_ERR_ARG;
  if (B < 1 || B > P->max_frames) return VG_ERR_ARG;
  if (offs[0] != 0) return VG_ERR_ARG;
  for (int b = 0; b < B; ++b)
    if (offs[b + 1] < offs[b] || offs[b + 1] - offs[b] > kMaxFramePoints) return VG_ERR_ARG;
  if (offs[B] > P->max_points) return VG_ERR_ARG;
  if (offs[B] > 0 && (!p->x || !p->y || !p->z)) return VG_ERR_ARG;
  if (!cells_consistent(out)) return VG_ERR_ARG;
  if (!filters_ok(filters, B)) return VG_ERR_ARG;
  for (int b = 0; b < B; ++b)
    if (!leaf_inverse(leaf[b], &P->invs[b])) return VG_ERR_LEAF;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // timed calls read their launch events after each call: one call at a time
  const int slot = P->timer ? 0 : (int)(P->calls & 1u);
  if (P->timer && plan_wait_all(P) != VG_OK) return VG_ERR_DEVICE;
  if (P->pending[slot]) {
    if (hipEventSynchronize(P->done[slot]) != hipSuccess) return VG_ERR_DEVICE;
    P->pending[slot] = false;
  }
  char* const stg = P->staging[slot];
  CallHdr hdr;
  if (!fill_staging(stg, P->L, *P->v, p, offs, leaf, P->invs, B, out, out_offsets,
                    frame_status, P->key_mode, P->fail_waits, &hdr, P->ws, filters,
                    P->host_input))
    return VG_ERR_ARG;
  // the call before this one uses the same workspace (on another stream,
  // perhaps): this call's stream waits for it on the device
  if (P->pending[slot ^ 1] && hipStreamWaitEvent(s, P->done[slot ^ 1], 0) != hipSuccess)
    return VG_ERR_DEVICE;
  const bool sparse = (hdr.filt & kFiltMinPts) != 0;
  vg_status rc = VG_OK;
  if (P->use_graph && !P->timer) {
    // the graph holds the sparse-cell pass once a call has needed it (its
    // kernels exit at once for calls that do not)
    if (P->gexec[slot] && sparse && !P->graph_sparse[slot]) {
      (void)hipGraphExecDestroy(P->gexec[slot]);
      (void)hipGraphDestroy(P->graph[slot]);
      P->gexec[slot] = nullptr;
      P->graph[slot] = nullptr;
    }
    if (!P->gexec[slot]) {
      hipStream_t cs;
      if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return VG_ERR_DEVICE;
      if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return VG_ERR_DEVICE;
      }
      rc = enqueue(*P->v, P->L, P->ws, stg, P->tuning.exec_mode, P->cus,
                   P->tuning.blocks_per_cu, cs, nullptr, sparse);
      hipGraph_t g = nullptr;
      const bool ok = hipStreamEndCapture(cs, &g) == hipSuccess && rc == VG_OK &&
                      hipGraphInstantiate(&P->gexec[slot], g, nullptr, nullptr, 0) == hipSuccess;
      (void)hipStreamDestroy(cs);
      if (!ok) {
        if (g) (void)hipGraphDestroy(g);
        P->gexec[slot] = nullptr;
        return VG_ERR_DEVICE;
      }
      P->graph[slot] = g;
      P->graph_sparse[slot] = sparse;
    }
    if (hipGraphLaunch(P->gexec[slot], s) != hipSuccess) rc = VG_ERR_DEVICE;
  } else {
    rc = enqueue(*P->v, P->L, P->ws, stg, P->tuning.exec_mode, P->cus,
                 P->tuning.blocks_per_cu, s, P->timer, sparse);
  }
  if (hipEventRecord(P->done[slot], s) == hipSuccess) P->pending[slot] = true;
  ++P->calls;
  return rc;
}

}  // namespace

extern "C" {

vg_status vg_downsample_batched(vg_batch_plan* P, const vg_points* p, const int64_t* offs,
                                const float* leaf, int B, vg_cells* out, int64_t* out_offsets,
                                int32_t* frame_status, void* stream) {
  return downsample_batch(P, p, offs, leaf, nullptr, B, out, out_offsets, frame_status, stream);
}

vg_status vg_downsample_batched_filtered(vg_batch_plan* P, const vg_points* p,
                                         const int64_t* offs, const float* leaf,
                                         const vg_filter* filters, int B, vg_cells* out,
                                         int64_t* out_offsets, int32_t* frame_status,
                                         void* stream) {
  if (!filters) return VG_ERR_ARG;
  return downsample_batch(P, p, offs, leaf, filters, B, out, out_offsets, frame_status, stream);
}

vg_status vg_batch_plan_destroy(vg_batch_plan* P) {
  if (!P) return VG_ERR_ARG;
  for (int k = 0; k < 2; ++k)
    if (P->pending[k] && P->done[k]) (void)hipEventSynchronize(P->done[k]);
  for (int k = 0; k < 2; ++k) {
    if (P->gexec[k]) (void)hipGraphExecDestroy(P->gexec[k]);
    if (P->graph[k]) (void)hipGraphDestroy(P->graph[k]);
    if (P->done[k]) (void)hipEventDestroy(P->done[k]);
    if (P->staging[k]) (void)hipHostFree(P->staging[k]);
  }
  if (P->timer) {
    P->timer->release();
    delete P->timer;
  }
  if (P->ws_base) (void)hipFree(P->ws_base);
  delete[] P->invs;
  delete P;
  return VG_OK;
}

}  // extern "C"

// ============================================================ voxel map ====
struct vg_map {
  MapWs ws;
  void* mem;
  int64_t cap;
  uint32_t* host;    // pinned readback
  uint32_t seq[4];   // operations so far of each counting kind: mark, clear, expire, export
};

namespace {

int map_grid(uint64_t items) {
  return (int)std::max<uint64_t>(1, std::min<uint64_t>((items + kMapBlock - 1) / kMapBlock, 8192));
}

bool frustum_ok(const vg_frustum* f) {
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(f->rot[k])) return false;
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(f->trans[k])) return false;
  const float v[6] = {f->fx, f->fy, f->cx, f->cy, f->z_near, f->z_far};
  for (float x : v)
    if (!std::isfinite(x)) return false;
  return f->width >= 1 && f->height >= 1 && f->z_near <= f->z_far;
}

// Counting kinds (vg_map::seq) and their counter pairs in MapCtl.
enum { kMapMark = 0, kMapClear = 1, kMapExpire = 2, kMapExport = 3 };

// Slot of the next operation of a kind (and count it).
uint32_t map_next_slot(vg_map* m, int kind) { return m->seq[kind]++ & 1u; }

// Slot the last operation of a kind counted into (slot 1 before the first,
// which is zero from creation).
uint32_t map_last_slot(const vg_map* m, int kind) { return (m->seq[kind] + 1u) & 1u; }

// Sync read of n counters of the map's control block (from index i0).
vg_status map_read(vg_map* m, int i0, int n, hipStream_t s) {
  const uint32_t* src = reinterpret_cast<const uint32_t*>(m->ws.ctl) + i0;
  if (hipMemcpyAsync(m->host, src, 4 * (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return VG_ERR_DEVICE;
  return VG_OK;
}

}  // namespace

extern "C" {

vg_status vg_map_create(int64_t capacity, float res, vg_map** map) {
  if (!map) return VG_ERR_ARG;
  *map = nullptr;
  if (capacity < 1 || capacity > ((int64_t)1 << 31)) return VG_ERR_ARG;
  float inv;
  if (!leaf_inverse(res, &inv)) return VG_ERR_LEAF;
  int64_t cap = 1024;
  while (cap < capacity) cap <<= 1;
  vg_map* m = new (std::nothrow) vg_map();
  if (!m) return VG_ERR_DEVICE;
  const size_t bytes = align_up(sizeof(MapCtl)) + (size_t)cap * (8 + 4 + 8 + 4);
  if (hipMalloc(&m->mem, bytes) != hipSuccess) {
    delete m;
    return VG_ERR_DEVICE;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&m->host), 64, hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(m->mem);
    delete m;
    return VG_ERR_DEVICE;
  }
  char* b = static_cast<char*>(m->mem);
  m->ws.ctl = reinterpret_cast<MapCtl*>(b);
  size_t o = align_up(sizeof(MapCtl));
  m->ws.keys = reinterpret_cast<uint64_t*>(b + o);    o += 8 * (size_t)cap;
  m->ws.tkeys = reinterpret_cast<uint64_t*>(b + o);   o += 8 * (size_t)cap;
  m->ws.stamps = reinterpret_cast<uint32_t*>(b + o);  o += 4 * (size_t)cap;
  m->ws.tstamps = reinterpret_cast<uint32_t*>(b + o);
  m->ws.mask = (uint64_t)cap - 1;
  m->ws.res = res;
  m->ws.inv = inv;
  m->cap = cap;
  hipLaunchKernelGGL(vg_map_reset_kernel, dim3(map_grid(cap)), dim3(kMapBlock), 0, nullptr, m->ws);
  if (hipMemsetAsync(m->ws.ctl, 0, sizeof(MapCtl), nullptr) != hipSuccess ||
      hipStreamSynchronize(nullptr) != hipSuccess) {
    vg_map_destroy(m);
    return VG_ERR_DEVICE;
  }
  *map = m;
  return VG_OK;
}

vg_status vg_map_destroy(vg_map* m) {
  if (!m) return VG_ERR_ARG;
  (void)hipDeviceSynchronize();
  if (m->host) (void)hipHostFree(m->host);
  if (m->mem) (void)hipFree(m->mem);
  delete m;
  return VG_OK;
}

vg_status vg_map_mark(vg_map* m, const float* x, const float* y, const float* z, int64_t n,
                      uint32_t stamp, void* stream) {
  if (!m || n < 0 || stamp == 0) return VG_ERR_ARG;
  if (n > 0 && (!x || !y || !z)) return VG_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // an empty mark still runs (one thread block) so that it counts 0 skipped
  const uint32_t slot = map_next_slot(m, kMapMark);
  hipLaunchKernelGGL(vg_map_mark_kernel, dim3(map_grid((uint64_t)std::max<int64_t>(n, 1))),
                     dim3(kMapBlock), 0, s, m->ws, x, y, z, n, stamp, slot);
  return hipGetLastError() == hipSuccess ? VG_OK : VG_ERR_DEVICE;
}

vg_status vg_map_clear_frustum(vg_map* m, const vg_frustum* f, void* stream) {
  if (!m || !f || !frustum_ok(f)) return VG_ERR_ARG;
  MapFrustum fr;
  for (int k = 0; k < 9; ++k) fr.r[k] = f->rot[k];
  for (int k = 0; k < 3; ++k) fr.t[k] = f->trans[k];
  fr.fx = f->fx;
  fr.fy = f->fy;
  fr.cx = f->cx;
  fr.cy = f->cy;
  fr.width = f->width;
  fr.height = f->height;
  fr.z_near = f->z_near;
  fr.z_far = f->z_far;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(vg_map_clear_kernel, dim3(map_grid((uint64_t)m->cap)), dim3(kMapBlock), 0, s,
                     m->ws, fr, map_next_slot(m, kMapClear));
  return hipGetLastError() == hipSuccess ? VG_OK : VG_ERR_DEVICE;
}

vg_status vg_map_expire(vg_map* m, uint32_t min_stamp, void* stream) {
  if (!m) return VG_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(vg_map_expire_kernel, dim3(map_grid((uint64_t)m->cap)), dim3(kMapBlock), 0, s,
                     m->ws, min_stamp, map_next_slot(m, kMapExpire));
  return hipGetLastError() == hipSuccess ? VG_OK : VG_ERR_DEVICE;
}

vg_status vg_map_export(vg_map* m, uint64_t* keys, uint32_t* stamps, int64_t cap, int64_t* n,
                        void* stream) {
  if (n) *n = 0;
  if (!m || !n || cap < 0 || (cap > 0 && (!keys || !stamps))) return VG_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint32_t slot = map_next_slot(m, kMapExport);
  hipLaunchKernelGGL(vg_map_export_kernel, dim3(map_grid((uint64_t)m->cap)), dim3(kMapBlock), 0, s,
                     m->ws, keys, stamps, (uint64_t)cap, slot);
  if (hipGetLastError() != hipSuccess) return VG_ERR_DEVICE;
  const vg_status rc = map_read(m, 0, (int)(offsetof(MapCtl, count) / 4), s);
  if (rc != VG_OK) return rc;
  *n = m->host[offsetof(MapCtl, live) / 4 + slot];
  return m->host[0] ? VG_ERR_WORKSPACE : VG_OK;
}

vg_status vg_map_compact(vg_map* m, void* stream) {
  if (!m) return VG_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int g = map_grid((uint64_t)m->cap);
  const uint32_t slot = map_next_slot(m, kMapExport);
  hipLaunchKernelGGL(vg_map_export_kernel, dim3(g), dim3(kMapBlock), 0, s, m->ws, m->ws.tkeys,
                     m->ws.tstamps, (uint64_t)m->cap, slot);
  hipLaunchKernelGGL(vg_map_reset_kernel, dim3(g), dim3(kMapBlock), 0, s, m->ws);
  hipLaunchKernelGGL(vg_map_reinsert_kernel, dim3(g), dim3(kMapBlock), 0, s, m->ws, slot);
  return hipGetLastError() == hipSuccess ? VG_OK : VG_ERR_DEVICE;
}

vg_status vg_map_stats(vg_map* m, vg_map_info* info, void* stream) {
  if (!m || !info) return VG_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(vg_map_zero2_kernel, dim3(1), dim3(64), 0, s, m->ws.ctl->count);
  hipLaunchKernelGGL(vg_map_count_kernel, dim3(map_grid((uint64_t)m->cap)), dim3(kMapBlock), 0, s,
                     m->ws, m->ws.ctl->count);
  if (hipGetLastError() != hipSuccess) return VG_ERR_DEVICE;
  const vg_status rc = map_read(m, 0, (int)(offsetof(MapCtl, pad) / 4), s);
  if (rc != VG_OK) return rc;
  const uint32_t* h = m->host;
  info->capacity = m->cap;
  info->occupied = h[offsetof(MapCtl, count) / 4];
  info->used_slots = h[offsetof(MapCtl, count) / 4 + 1];
  info->last_skipped = h[offsetof(MapCtl, skipped) / 4 + map_last_slot(m, kMapMark)];
  info->last_cleared = h[offsetof(MapCtl, cleared) / 4 + map_last_slot(m, kMapClear)];
  info->last_expired = h[offsetof(MapCtl, expired) / 4 + map_last_slot(m, kMapExpire)];
  info->full = h[0] ? 1 : 0;
  return VG_OK;
}

}  // extern "C"

// Shared definitions of the voxel-grid pipeline: workspace layout, per-frame
// state and small device helpers.  Device and host code of libvg include it;
// nothing here is exported.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace vg {

// Cells per axis are capped at 2^21: the 63-bit Morton key then fits, and
// every cell coordinate is exact in binary32.
constexpr float kMaxCellsPerAxis = 2097152.0f;
constexpr int kMaxPassSlots = 11;       // ceil(63 / 6): enough for radix_bits >= 6
constexpr int kMaxFramePoints = (1 << 30) - 1;

// Look-back descriptor flags (top two bits).
constexpr uint32_t kFlagA32 = 1u << 30;  // tile aggregate only
constexpr uint32_t kFlagP32 = 2u << 30;  // inclusive prefix
constexpr uint32_t kVal32 = (1u << 30) - 1;
constexpr uint64_t kFlagA64 = 1ull << 62;
constexpr uint64_t kFlagP64 = 2ull << 62;
constexpr uint64_t kVal64 = (1ull << 62) - 1;

enum FrameStatus : int32_t { kFrameOk = 0, kFrameOverflow = 3, kFrameDeviceError = 5 };

// Per-call header, copied from the host.
//   big tiles  (bbox, histogram):  NTb over all frames
//   sort tiles (radix passes):     NTs
//   reduce tiles:                  NTr
struct CallHdr {
  int32_t B;            // frames
  int32_t key_mode;     // 0 linear, 1 Morton
  int32_t NTb, NTs, NTr;
  uint32_t want;        // output mask (kOut*)
  int64_t N;            // points over all frames
  int32_t ilv_rounds;   // > 0: radix-pass tiles are taken round-robin over frames
  int32_t fail_waits;   // non-zero: the call starts with the time-out flag raised (tests of
                        // the error path: every kernel then exits without touching outputs)
  uint32_t filt;        // kFiltView: the bbox pass writes the point view (transform / height
                        // limit of some frame); kFiltMinPts: sparse cells are dropped after
  uint32_t pad2;
};

enum : uint32_t { kFiltView = 1, kFiltMinPts = 2, kFiltCountInternal = 4 };

// Per-frame input filter (the global-frame transform and height limit that
// the filter's input contract asks for, and the removal of sparse cells).
struct FrameXf {
  float r[9];       // rotation, row-major (applied when on & kXfRotate)
  float t[3];       // translation
  float zlo, zhi;   // height limit on the transformed z, inclusive
  uint32_t on;      // kXfRotate | kXfLimit
  uint32_t minp;    // cells with fewer points are dropped (<= 1: none)
};
enum : uint32_t { kXfRotate = 1, kXfLimit = 2 };

// Round-robin order of the radix-pass tiles: round j holds tile j of every
// frame with more than j sort tiles, frames by descending tile count.  Each
// frame's tiles stay in order, and tiles of one frame are spread in time, so
// the per-frame look-back chains stay short.
constexpr int kIlvMaxRounds = 1024;
constexpr int kIlvMaxFrames = 256;

enum : uint32_t {
  kOutXYZ = 1, kOutRGB = 2, kOutCount = 4, kOutKey = 8, kOutPointCell = 16, kOutRef = 32,
  kOutLocal = 64,
};

// Per-frame description, copied from the host.
struct FrameDesc {
  int64_t off;           // first point of the frame in the concatenated arrays
  int64_t n;             // points of the frame
  float leaf;
  float inv;             // RN32(1/leaf), computed on the host
  int32_t tb0, ts0, tr0; // first big / sort / reduce tile of the frame
  int32_t ntb, nts, ntr; // number of such tiles (each >= 1)
};

// Per-frame state written during a call; zeroed at the start of every call.
struct FrameState {
  uint32_t mn_neg[3];   // max of ~enc(v)  ->  ~result = enc(min)
  uint32_t mx[3];       // max of enc(v)
  uint32_t n_valid;
  uint32_t bbox_done;   // big tiles done
  uint32_t hist_done;   // big tiles done
  uint32_t pass_done[kMaxPassSlots];  // sort tiles done, per pass
  uint32_t pad[4];
};
static_assert(sizeof(FrameState) == 24 * 4, "FrameState layout");

// Carry-out fragment of a reduce tile: the partial sums of the segment that
// runs past the tile's end.
struct Frag {
  uint32_t n;
  float s[3];
  float c[3];
  uint32_t head_pos;  // frame position of the segment's first point if it lies in this tile,
                      // else kNoHead
  uint32_t ref;       // index of that first point (valid with head_pos)
  uint32_t pad;
  uint64_t rgb;       // packed colour sums, 21 bits per channel
};
constexpr uint32_t kNoHead = 0xffffffffu;

// A cell that starts in an earlier reduce tile and ends in this one: the part
// of its sums inside this tile and where its row goes.  The fix-up phase adds
// the earlier tiles' carry-out parts and writes the row.
struct Pend {
  uint32_t valid;
  uint32_t b, j;        // frame, reduce tile within the frame
  uint32_t lo, hi;      // cell key
  float r[3];           // cell corner
  int64_t row;
  uint32_t n;
  float s[3], c[3];
  uint32_t pad;
  uint64_t rgb;         // packed colour sums, 21 bits per channel
};

struct Ctl {
  uint32_t queue[16];        // [0]: persistent queue; [1 + phase]: phased queues
  uint32_t error;            // non-zero: a device-side wait timed out
  uint32_t max_passes;       // max radix passes over the frames of the call
  uint32_t hist_tiles_done;  // big tiles (all frames) whose histogram is done
  uint32_t red_tiles_done;   // reduce tiles (all frames) done
  uint32_t rows;             // rows of the call (for the sparse-cell pass)
  uint32_t rows_kept;        // rows left by the sparse-cell pass
  uint32_t pad[10];
};

struct Io;

// Device pointers of one workspace (passed to kernels by value).
struct Ws {
  CallHdr* hdr;
  FrameDesc* fd;
  uint32_t* tpb;        // [B+1] big-tile prefix over frames
  uint32_t* tps;        // [B+1] sort-tile prefix over frames
  uint32_t* tpr;        // [B+1] reduce-tile prefix over frames
  uint32_t* ilv_s;      // [rounds+1] first item of each round
  uint32_t* ilv_perm;   // [B] frames by descending sort-tile count
  uint2* tinfo;         // [NTb + NTs + NTr]: (frame, tile within frame)
  Ctl* ctl;
  FrameState* fs;       // [B]
  uint32_t* hist;       // [B][slots][R]
  uint32_t* sdesc;      // [slots][NTs][R]
  uint64_t* rdesc;      // [NTr]
  uint32_t* fflag;      // [NTr]
  Frag* frag;           // [NTr]
  Pend* pend;           // [NTr]
  uint32_t* lo[2];      // [N]
  uint32_t* hi[2];      // [N]
  uint32_t* idx[2];     // [N]
  float4* rec;          // [N] x, y, z and packed rgb of every point, written by the bbox pass
  FrameXf* xf;          // [B] per-frame filters (staged)
  float* tx;            // [N] the point view after transform and height limit
  float* ty;
  float* tz;
  uint32_t* rflag;      // [N + 1] rows kept by the sparse-cell pass
  uint32_t* rpos;       // [N + 1] their new rows (exclusive prefix)
  uint32_t* bsum;       // [scan tiles + 1]
  Io* io;               // inputs/outputs of the call (copied from the host)
  // capacities the workspace was carved for
  int32_t capB, capNTb, capNTs, capNTr, slots, R;
  int64_t capN;
};

// Inputs and outputs of one call (device pointers; the struct itself is
// copied to device memory with the call header, so launches carry no
// per-call arguments and can be replayed from a graph).
struct Io {
  const float* x;
  const float* y;
  const float* z;
  const float* vx;       // the points as every phase after the bbox pass sees them: x, y, z,
  const float* vy;       // or the transformed, height-limited copy the bbox pass writes
  const float* vz;
  const uint8_t* rgb;
  float* cx;
  float* cy;
  float* cz;
  uint8_t* crgb;
  uint32_t* count;
  uint64_t* key;
  int32_t* point_cell;
  uint32_t* ref_index;
  float* lx;
  float* ly;
  float* lz;
  int64_t* out_offsets;  // [B+1]
  int32_t* frame_status; // [B]
};

}  // namespace vg

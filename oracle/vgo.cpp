// Voxel-grid centroid downsampling -- plain CPU oracle.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  It shares no code,
// header, table or constant with the HIP library it checks.
//
// What it computes (arXiv 2102.11084, Sec. II-C):
//   * the space around the cloud is cut into a regular grid of cubes and every
//     point is classified into one cube (Sec. II-C; Alg. 1, the per-point
//     subdivision lookup);
//   * a sorted key/value table gives the points of each cube and their number
//     (Sec. II-C, the radix-sorted subdivision table);
//   * the filter the paper accelerates is the voxel filter of the point-cloud
//     library used by the costmap layer (Sec. I and Sec. II-C): every occupied
//     cube is replaced by the centroid of its points; the compacted cloud is
//     handed back (Alg. 1, final deletion/copy-back steps).
// The paper does not write the centroid step or any rounding rule down.  The
// readings taken here:
//   * the grid is anchored at the per-axis minimum of the valid points and has
//     cubic cells of edge `leaf` (the paper normalises into [-1,1]^3 and splits
//     2^n ways, which gives non-cubic cells on a non-cubic box);
//   * cell coordinate k = floor(RN32(RN32(p - min) * inv)), inv = RN32(1/leaf);
//     the paper's decision tree equals this floor on a uniform grid;
//   * a point is valid iff x, y and z are all finite (NaN or +-Inf rejected);
//   * at most 2^21 cells per axis, else GRID_OVERFLOW (the paper stops at 2^9);
//   * cells are emitted in ascending key order (the paper's table is sorted);
//   * colour is the per-channel mean rounded half up, in integers.
//
// Implementation style: one std::map keyed by the cell key, visited in
// ascending original index, FP64 accumulation.  Deliberately slow and plain.
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fno-fast-math -shared -fPIC
// (no FMA contraction, no flush-to-zero; x86-64 SSE arithmetic is IEEE
// binary32 round-to-nearest-even per operation).
// "parity pinned": every entry point is checked by the CPU test suite against
// closed forms, brute force and invariants.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <utility>
#include <vector>

namespace {

// Status values (numbered like the product library's, defined independently).
enum : int {
  VGO_OK = 0,
  VGO_ERR_ARG = 1,
  VGO_ERR_LEAF = 2,
  VGO_ERR_GRID_OVERFLOW = 3,
};

enum : int { VGO_KEY_LINEAR = 0, VGO_KEY_MORTON = 1 };

// A grid of at most 2^21 cells per axis keeps the 63-bit Morton key and every
// cell coordinate exactly representable in binary32 (the paper caps its grid
// at 2^9 per axis; Sec. II-C).
const float kMaxCellsPerAxis = 2097152.0f;  // 2^21

struct Grid {
  float inv;        // 1/leaf, binary32, round to nearest even
  float mn[3];      // bounding box of the valid points
  float mx[3];
  uint32_t d[3];    // cells per axis
  int64_t n_valid;
};

bool point_is_valid(float x, float y, float z) {
  return std::isfinite(x) && std::isfinite(y) && std::isfinite(z);
}

// Leaf check and inverse: the leaf must be a finite positive number whose
// binary32 reciprocal is finite.
int leaf_inverse(float leaf, float* inv) {
  if (!std::isfinite(leaf) || !(leaf > 0.0f)) return VGO_ERR_LEAF;
  float r = 1.0f / leaf;
  if (!std::isfinite(r)) return VGO_ERR_LEAF;
  *inv = r;
  return VGO_OK;
}

// One cell coordinate: floor(RN32(RN32(p - min) * inv)).
uint32_t cell_coord(float p, float mn, float inv) {
  float diff = p - mn;
  float t = diff * inv;
  return (uint32_t)std::floor(t);
}

// Bounding box, cell counts per axis, overflow check (Sec. II-C grid).
int make_grid(const float* x, const float* y, const float* z, int64_t n, float leaf, Grid* g) {
  int st = leaf_inverse(leaf, &g->inv);
  if (st != VGO_OK) return st;
  g->n_valid = 0;
  const float* c[3] = {x, y, z};
  for (int64_t i = 0; i < n; ++i) {
    if (!point_is_valid(x[i], y[i], z[i])) continue;
    for (int a = 0; a < 3; ++a) {
      float v = c[a][i];
      if (g->n_valid == 0) {
        g->mn[a] = v;
        g->mx[a] = v;
      } else {
        if (v < g->mn[a]) g->mn[a] = v;
        if (v > g->mx[a]) g->mx[a] = v;
      }
    }
    g->n_valid += 1;
  }
  if (g->n_valid == 0) {
    for (int a = 0; a < 3; ++a) { g->mn[a] = 0.0f; g->mx[a] = 0.0f; g->d[a] = 0; }
    return VGO_OK;
  }
  for (int a = 0; a < 3; ++a) {
    float extent = g->mx[a] - g->mn[a];
    float t = extent * g->inv;
    if (!(t < kMaxCellsPerAxis)) return VGO_ERR_GRID_OVERFLOW;
    g->d[a] = (uint32_t)std::floor(t) + 1u;
  }
  return VGO_OK;
}

// Linear key: x varies fastest, then y, then z.
uint64_t linear_key(const uint32_t k[3], const uint32_t d[3]) {
  return (uint64_t)k[0] + (uint64_t)d[0] * ((uint64_t)k[1] + (uint64_t)d[1] * (uint64_t)k[2]);
}

// Morton key: bit b of kx goes to bit 3b, of ky to 3b+1, of kz to 3b+2.
uint64_t morton_key(const uint32_t k[3]) {
  uint64_t key = 0;
  for (int b = 0; b < 21; ++b) {
    for (int a = 0; a < 3; ++a) {
      uint64_t bit = (k[a] >> b) & 1u;
      key |= bit << (3 * b + a);
    }
  }
  return key;
}

uint64_t point_key(const Grid& g, float px, float py, float pz, int mode) {
  uint32_t k[3];
  k[0] = cell_coord(px, g.mn[0], g.inv);
  k[1] = cell_coord(py, g.mn[1], g.inv);
  k[2] = cell_coord(pz, g.mn[2], g.inv);
  return mode == VGO_KEY_MORTON ? morton_key(k) : linear_key(k, g.d);
}

struct Cell {
  uint64_t n = 0;
  int64_t ref = -1;         // first (smallest) original index seen
  double ref_p[3] = {0, 0, 0};
  double sum[3] = {0, 0, 0};    // sum of p
  double local[3] = {0, 0, 0};  // sum of (p - p_ref)
  uint64_t rgb[3] = {0, 0, 0};
  int64_t rank = -1;
};

}  // namespace

extern "C" {

// Grid of a cloud: bounding box, cells per axis, valid count, and optionally
// every point's key (0 for invalid points) and validity flag.
int vgo_grid(const float* x, const float* y, const float* z, int64_t n, float leaf, int key_mode,
             float* mn3, float* mx3, uint32_t* d3, int64_t* n_valid, uint64_t* keys, uint8_t* valid) {
  if (n < 0 || (n > 0 && (!x || !y || !z))) return VGO_ERR_ARG;
  if (key_mode != VGO_KEY_LINEAR && key_mode != VGO_KEY_MORTON) return VGO_ERR_ARG;
  Grid g;
  int st = make_grid(x, y, z, n, leaf, &g);
  if (st != VGO_OK) return st;
  if (mn3) for (int a = 0; a < 3; ++a) mn3[a] = g.mn[a];
  if (mx3) for (int a = 0; a < 3; ++a) mx3[a] = g.mx[a];
  if (d3) for (int a = 0; a < 3; ++a) d3[a] = g.d[a];
  if (n_valid) *n_valid = g.n_valid;
  for (int64_t i = 0; i < n; ++i) {
    bool v = point_is_valid(x[i], y[i], z[i]);
    if (valid) valid[i] = v ? 1 : 0;
    if (keys) keys[i] = v ? point_key(g, x[i], y[i], z[i], key_mode) : 0;
  }
  return VGO_OK;
}

// Voxel-grid centroid filter of one cloud.  Outputs are written for cells
// 0..m-1 in ascending key order; every output pointer may be NULL.
//   c{x,y,z}   FP64 centroid  sum(p)/n
//   l{x,y,z}   FP64 local mean  sum(p - p_ref)/n, p_ref = point at ref_index
//   rgb_out    per channel floor((sum + floor(n/2)) / n), n x 3 interleaved
//   count, key, ref_index (smallest original index in the cell)
//   point_cell cell of every input point, -1 for invalid points
int vgo_downsample(const float* x, const float* y, const float* z, const uint8_t* rgb, int64_t n,
                   float leaf, int key_mode, double* cx, double* cy, double* cz, double* lx,
                   double* ly, double* lz, uint8_t* rgb_out, uint32_t* count, uint64_t* key,
                   int64_t* ref_index, int32_t* point_cell, int64_t* m) {
  if (!m) return VGO_ERR_ARG;
  *m = 0;
  if (n < 0 || (n > 0 && (!x || !y || !z))) return VGO_ERR_ARG;
  if (key_mode != VGO_KEY_LINEAR && key_mode != VGO_KEY_MORTON) return VGO_ERR_ARG;
  Grid g;
  int st = make_grid(x, y, z, n, leaf, &g);
  if (st != VGO_OK) return st;

  std::map<uint64_t, Cell> cells;
  std::vector<uint64_t> keys(n > 0 ? (size_t)n : 1u);
  for (int64_t i = 0; i < n; ++i) {
    if (point_is_valid(x[i], y[i], z[i])) {
      double p[3] = {(double)x[i], (double)y[i], (double)z[i]};
      uint64_t k = point_key(g, x[i], y[i], z[i], key_mode);
      keys[i] = k;
      Cell& c = cells[k];
      if (c.n == 0) {
        c.ref = i;
        for (int a = 0; a < 3; ++a) c.ref_p[a] = p[a];
      }
      c.n += 1;
      for (int a = 0; a < 3; ++a) {
        c.sum[a] += p[a];
        c.local[a] += p[a] - c.ref_p[a];
        if (rgb) c.rgb[a] += rgb[3 * i + a];
      }
    }
  }

  int64_t r = 0;
  for (auto& kv : cells) {
    Cell& c = kv.second;
    c.rank = r;
    double nn = (double)c.n;
    if (cx) cx[r] = c.sum[0] / nn;
    if (cy) cy[r] = c.sum[1] / nn;
    if (cz) cz[r] = c.sum[2] / nn;
    if (lx) lx[r] = c.local[0] / nn;
    if (ly) ly[r] = c.local[1] / nn;
    if (lz) lz[r] = c.local[2] / nn;
    if (rgb_out)
      for (int a = 0; a < 3; ++a) rgb_out[3 * r + a] = (uint8_t)((c.rgb[a] + c.n / 2) / c.n);
    if (count) count[r] = (uint32_t)c.n;
    if (key) key[r] = kv.first;
    if (ref_index) ref_index[r] = c.ref;
    ++r;
  }
  if (point_cell) {
    for (int64_t i = 0; i < n; ++i) {
      if (point_is_valid(x[i], y[i], z[i]))
        point_cell[i] = (int32_t)cells.find(keys[i])->second.rank;
      else
        point_cell[i] = -1;
    }
  }
  *m = r;
  return VGO_OK;
}

// Gradient of the centroids with respect to the input coordinates, with the
// cell assignment held fixed: dL/dp_i = G[cell(i)] / count[cell(i)], zero for
// points outside every cell.
int vgo_backward(const double* gx, const double* gy, const double* gz, const uint32_t* count,
                 int64_t m, const int32_t* point_cell, int64_t n, double* dx, double* dy,
                 double* dz) {
  if (n < 0 || m < 0) return VGO_ERR_ARG;
  for (int64_t i = 0; i < n; ++i) {
    int32_t c = point_cell[i];
    if (c < 0 || c >= m) {
      dx[i] = 0.0;
      dy[i] = 0.0;
      dz[i] = 0.0;
    } else {
      double nn = (double)count[c];
      dx[i] = gx[c] / nn;
      dy[i] = gy[c] / nn;
      dz[i] = gz[c] / nn;
    }
  }
  return VGO_OK;
}

// Centroids for a given (fixed) assignment, FP64 inputs: the function whose
// finite differences pin the backward formula.
int vgo_centroids_fixed(const double* x, const double* y, const double* z, int64_t n,
                        const int32_t* point_cell, int64_t m, double* cx, double* cy, double* cz) {
  if (n < 0 || m < 0) return VGO_ERR_ARG;
  std::vector<double> s(3 * (size_t)m, 0.0);
  std::vector<uint64_t> cnt((size_t)m, 0);
  for (int64_t i = 0; i < n; ++i) {
    int32_t c = point_cell[i];
    if (c < 0 || c >= m) continue;
    s[3 * c + 0] += x[i];
    s[3 * c + 1] += y[i];
    s[3 * c + 2] += z[i];
    cnt[c] += 1;
  }
  for (int64_t k = 0; k < m; ++k) {
    double nn = (double)cnt[k];
    cx[k] = cnt[k] ? s[3 * k + 0] / nn : 0.0;
    cy[k] = cnt[k] ? s[3 * k + 1] / nn : 0.0;
    cz[k] = cnt[k] ? s[3 * k + 2] / nn : 0.0;
  }
  return VGO_OK;
}


}  // extern "C"

// ---------------------------------------------------------------------------
// The filter's input contract in the costmap layer (Sec. II-C): the cloud is
// first brought into the global frame, so that its height can be limited, and
// the filter should also remove sensor noise.  As read here:
//   * rigid transform: p'_a = RN32(RN32(RN32(RN32(R[a][0]*x) + RN32(R[a][1]*y))
//     + RN32(R[a][2]*z)) + t[a]), R row-major, when asked for (else p' = p);
//   * height limit: a point is kept iff it is valid, p' is finite and
//     z_min <= p'_z <= z_max; the others are treated as invalid points;
//   * noise: cells with fewer than min_points points are dropped, the
//     remaining rows renumbered in key order (their points' point_cell too;
//     points of dropped cells get -1).
// The voxel filter itself is vgo_downsample on the transformed, cropped cloud.

extern "C" {

int vgo_downsample_filtered(const float* x, const float* y, const float* z, const uint8_t* rgb,
                            int64_t n, float leaf, int key_mode, const float* rot,
                            const float* trans, float z_min, float z_max, uint32_t min_points,
                            double* cx, double* cy, double* cz, double* lx, double* ly, double* lz,
                            uint8_t* rgb_out, uint32_t* count, uint64_t* key, int64_t* ref_index,
                            int32_t* point_cell, int64_t* m) {
  if (!m) return VGO_ERR_ARG;
  *m = 0;
  if (n < 0 || (n > 0 && (!x || !y || !z))) return VGO_ERR_ARG;
  if (std::isnan(z_min) || std::isnan(z_max) || z_min > z_max) return VGO_ERR_ARG;
  if (rot || trans) {
    if (!rot || !trans) return VGO_ERR_ARG;
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(rot[k])) return VGO_ERR_ARG;
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(trans[k])) return VGO_ERR_ARG;
  }
  const float nan = std::nanf("");
  std::vector<float> gx((size_t)std::max<int64_t>(n, 1)), gy(gx.size()), gz(gx.size());
  for (int64_t i = 0; i < n; ++i) {
    float p[3] = {x[i], y[i], z[i]};
    float q[3] = {p[0], p[1], p[2]};
    if (rot) {
      for (int a = 0; a < 3; ++a) {
        float s0 = rot[3 * a + 0] * p[0];
        float s1 = rot[3 * a + 1] * p[1];
        float s2 = rot[3 * a + 2] * p[2];
        float s01 = s0 + s1;
        float s012 = s01 + s2;
        q[a] = s012 + trans[a];
      }
    }
    bool keep = point_is_valid(p[0], p[1], p[2]) && point_is_valid(q[0], q[1], q[2]) &&
                q[2] >= z_min && q[2] <= z_max;
    gx[i] = keep ? q[0] : nan;
    gy[i] = keep ? q[1] : nan;
    gz[i] = keep ? q[2] : nan;
  }
  const size_t cap = (size_t)std::max<int64_t>(n, 1);
  std::vector<double> ax(cap), ay(cap), az(cap), bx(cap), by(cap), bz(cap);
  std::vector<uint8_t> argb(3 * cap);
  std::vector<uint32_t> acount(cap);
  std::vector<uint64_t> akey(cap);
  std::vector<int64_t> aref(cap);
  std::vector<int32_t> apc(cap);
  int64_t am = 0;
  int st = vgo_downsample(gx.data(), gy.data(), gz.data(), rgb, n, leaf, key_mode, ax.data(),
                          ay.data(), az.data(), bx.data(), by.data(), bz.data(), argb.data(),
                          acount.data(), akey.data(), aref.data(), apc.data(), &am);
  if (st != VGO_OK) return st;
  // drop the cells with fewer than min_points points
  std::vector<int64_t> row((size_t)std::max<int64_t>(am, 1), -1);
  int64_t r = 0;
  for (int64_t k = 0; k < am; ++k) {
    if (acount[k] < min_points) continue;
    row[k] = r;
    if (cx) cx[r] = ax[k];
    if (cy) cy[r] = ay[k];
    if (cz) cz[r] = az[k];
    if (lx) lx[r] = bx[k];
    if (ly) ly[r] = by[k];
    if (lz) lz[r] = bz[k];
    if (rgb_out)
      for (int a = 0; a < 3; ++a) rgb_out[3 * r + a] = argb[3 * k + a];
    if (count) count[r] = acount[k];
    if (key) key[r] = akey[k];
    if (ref_index) ref_index[r] = aref[k];
    ++r;
  }
  if (point_cell)
    for (int64_t i = 0; i < n; ++i) point_cell[i] = apc[i] < 0 ? -1 : (int32_t)row[apc[i]];
  *m = r;
  return VGO_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Global voxel map (Sec. II-C: the costmap layer marks the cells of each new
// cloud as occupied and clears, as free, the cells inside the sensor's view,
// on a sparse map of the whole space; the paper times these operations and
// names a GPU map as future work).  As read here:
//   * voxels of edge `res` on a grid fixed in the global frame:
//     k_a = floor(RN32(p_a * inv_res)), inv_res = RN32(1/res), for
//     -2^20 <= k_a < 2^20 (points outside, or not finite, are skipped);
//     key = (k_x + 2^20) | (k_y + 2^20) << 21 | (k_z + 2^20) << 42;
//   * mark: every voxel holding a point of the cloud gets the time stamp
//     (inserted, or re-stamped);
//   * clear: every voxel whose centre c_a = RN32(RN32(k_a + 0.5) * res) lies in
//     the camera frustum is removed.  With the camera pose (R, t) (camera to
//     global) and d_a = RN32(c_a - t_a), the centre in the camera frame is
//     q_j = RN32(RN32(RN32(R[0][j] d_0) + RN32(R[1][j] d_1)) + RN32(R[2][j] d_2));
//     it is inside iff z_near <= q_2 <= z_far and the pixel coordinates
//     u = RN32(RN32(fx * RN32(q_0 / q_2)) + cx), v = RN32(RN32(fy * RN32(q_1 / q_2)) + cy)
//     satisfy -0.5 <= u <= width - 0.5 and -0.5 <= v <= height - 0.5;
//   * expire: voxels stamped before a given stamp are removed (the layer's
//     temporal decay).
// The oracle keeps a std::map from key to stamp.

namespace {

struct VoxelMap {
  float res, inv;
  std::map<uint64_t, uint32_t> vox;
};

const int32_t kVoxelHalfRange = 1 << 20;

bool voxel_key(const VoxelMap& m, float x, float y, float z, uint64_t* key) {
  if (!point_is_valid(x, y, z)) return false;
  const float p[3] = {x, y, z};
  uint64_t k = 0;
  for (int a = 0; a < 3; ++a) {
    float t = p[a] * m.inv;
    float f = std::floor(t);
    if (!(f >= -(float)kVoxelHalfRange && f < (float)kVoxelHalfRange)) return false;
    int64_t c = (int64_t)f + kVoxelHalfRange;
    k |= (uint64_t)c << (21 * a);
  }
  *key = k;
  return true;
}

bool in_frustum(const VoxelMap& m, uint64_t key, const float* R, const float* t, float fx,
                float fy, float cx, float cy, int32_t width, int32_t height, float z_near,
                float z_far) {
  float d[3];
  for (int a = 0; a < 3; ++a) {
    int64_t k = (int64_t)((key >> (21 * a)) & ((1u << 21) - 1u)) - kVoxelHalfRange;
    float kc = (float)k + 0.5f;
    float c = kc * m.res;
    d[a] = c - t[a];
  }
  float q[3];
  for (int j = 0; j < 3; ++j) {
    float s0 = R[0 * 3 + j] * d[0];
    float s1 = R[1 * 3 + j] * d[1];
    float s2 = R[2 * 3 + j] * d[2];
    float s01 = s0 + s1;
    q[j] = s01 + s2;
  }
  if (!(q[2] >= z_near && q[2] <= z_far)) return false;
  float rx = q[0] / q[2];
  float ry = q[1] / q[2];
  float u = fx * rx + cx;
  float v = fy * ry + cy;
  return u >= -0.5f && u <= (float)width - 0.5f && v >= -0.5f && v <= (float)height - 0.5f;
}

}  // namespace

extern "C" {

void* vgo_map_create(float res) {
  if (!std::isfinite(res) || !(res > 0.0f)) return nullptr;
  VoxelMap* m = new VoxelMap();
  m->res = res;
  m->inv = 1.0f / res;
  return m;
}

void vgo_map_destroy(void* m) { delete static_cast<VoxelMap*>(m); }

// Marks the voxels of n points with `stamp`; returns the points skipped.
int64_t vgo_map_mark(void* mp, const float* x, const float* y, const float* z, int64_t n,
                     uint32_t stamp) {
  VoxelMap& m = *static_cast<VoxelMap*>(mp);
  int64_t skipped = 0;
  for (int64_t i = 0; i < n; ++i) {
    uint64_t k;
    if (voxel_key(m, x[i], y[i], z[i], &k)) m.vox[k] = stamp;
    else ++skipped;
  }
  return skipped;
}

// Clears the voxels in the frustum; returns how many.
int64_t vgo_map_clear(void* mp, const float* R, const float* t, float fx, float fy, float cx,
                      float cy, int32_t width, int32_t height, float z_near, float z_far) {
  VoxelMap& m = *static_cast<VoxelMap*>(mp);
  int64_t cleared = 0;
  for (auto it = m.vox.begin(); it != m.vox.end();) {
    if (in_frustum(m, it->first, R, t, fx, fy, cx, cy, width, height, z_near, z_far)) {
      it = m.vox.erase(it);
      ++cleared;
    } else {
      ++it;
    }
  }
  return cleared;
}

int64_t vgo_map_expire(void* mp, uint32_t min_stamp) {
  VoxelMap& m = *static_cast<VoxelMap*>(mp);
  int64_t gone = 0;
  for (auto it = m.vox.begin(); it != m.vox.end();) {
    if (it->second < min_stamp) {
      it = m.vox.erase(it);
      ++gone;
    } else {
      ++it;
    }
  }
  return gone;
}

// The voxels in ascending key order (at most cap); returns their number.
int64_t vgo_map_export(void* mp, uint64_t* keys, uint32_t* stamps, int64_t cap) {
  VoxelMap& m = *static_cast<VoxelMap*>(mp);
  int64_t i = 0;
  for (const auto& kv : m.vox) {
    if (i < cap) {
      keys[i] = kv.first;
      stamps[i] = kv.second;
    }
    ++i;
  }
  return i;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Neighbour-bucket decimation (arXiv 2102.11084, Sec. II-C, Alg. 1).
//
// What the paper's own GPU filter computes, as read here:
//   * the same grid as above (cubic cells of edge `leaf` anchored at the
//     valid points' minimum) is the paper's regular decomposition of space;
//     only the 27 cells around a point's cell are searched for its neighbours
//     (Sec. II-C), with the Euclidean distance of Eq. (1);
//   * q is a neighbour of p iff q != p, both are valid, their cell coordinates
//     differ by at most 1 on every axis, and d2(p, q) <= r2, where
//     d2 = RN32(RN32(RN32(dx*dx) + RN32(dy*dy)) + RN32(dz*dz)), dx = RN32(xq - xp)
//     (and so on), r2 = RN32(radius * radius), 0 < radius <= leaf;
//   * a round (Alg. 1, the loop body): every point still present counts its
//     neighbours that are still present; it is marked when the count exceeds
//     the threshold `umbral`; if more than `round_size` points are marked
//     (1000 in the paper), `round_size` of them chosen at random are deleted
//     for good and another round follows; otherwise the loop ends and every
//     marked point is deleted (Alg. 1, the final deletion);
//   * the random choice: marked point i gets the priority word 0 of
//     Philox4x64-10 (Salmon et al., SC'11) at counter (i, round, 0, 0) under
//     key (seed, 0); the `round_size` marked points of smallest
//     (priority, i) are the ones deleted.
// The oracle recounts every present point's neighbours in every round, from
// neighbour lists built once by the 27-bucket search.

namespace {

const uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
const uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
const uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
const uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;

void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

// Philox4x64 with 10 rounds: each round multiplies words 0 and 2 by the two
// round constants and mixes the halves with words 1 and 3 and the key; the
// key advances by the two Weyl constants between rounds.
void philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(kPhiloxM0, c[0], &hi0, &lo0);
    mulhilo64(kPhiloxM1, c[2], &hi1, &lo1);
    uint64_t n0 = hi1 ^ c[1] ^ k0;
    uint64_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}

float dist2(float ax, float ay, float az, float bx, float by, float bz) {
  float dx = bx - ax;
  float dy = by - ay;
  float dz = bz - az;
  float sx = dx * dx;
  float sy = dy * dy;
  float sz = dz * dz;
  float sxy = sx + sy;
  return sxy + sz;
}

}  // namespace

extern "C" {

// Philox4x64-10 of one counter (exposed so the tests can check it against an
// independent implementation).
void vgo_philox4x64(const uint64_t* ctr, const uint64_t* key, uint64_t* out) {
  philox4x64_10(ctr, key, out);
}

// Neighbour-bucket decimation of one cloud.  keep[i] = 1 for the points that
// survive (invalid points never do); count0[i] = neighbours of i before any
// deletion (0 for invalid points); marked[r] = points marked in round r for
// r < cap_rounds; *rounds = rounds run.  Every output pointer but rounds may
// be NULL.
int vgo_nbd(const float* x, const float* y, const float* z, int64_t n, float leaf, float radius,
            uint32_t umbral, uint64_t seed, int64_t round_size, uint8_t* keep, uint32_t* count0,
            int64_t* marked, int64_t cap_rounds, int64_t* rounds) {
  if (!rounds) return VGO_ERR_ARG;
  *rounds = 0;
  if (n < 0 || (n > 0 && (!x || !y || !z)) || round_size < 1 || cap_rounds < 0)
    return VGO_ERR_ARG;
  Grid g;
  int st = make_grid(x, y, z, n, leaf, &g);
  if (st != VGO_OK) return st;
  if (!std::isfinite(radius) || !(radius > 0.0f) || !(radius <= leaf)) return VGO_ERR_ARG;
  const float r2 = radius * radius;

  // buckets: cell coordinates -> the valid points in it, ascending index
  std::map<std::array<uint32_t, 3>, std::vector<int64_t>> bucket;
  std::vector<std::array<uint32_t, 3>> cell((size_t)std::max<int64_t>(n, 1));
  std::vector<uint8_t> valid((size_t)std::max<int64_t>(n, 1), 0);
  for (int64_t i = 0; i < n; ++i) {
    if (!point_is_valid(x[i], y[i], z[i])) continue;
    valid[i] = 1;
    cell[i] = {cell_coord(x[i], g.mn[0], g.inv), cell_coord(y[i], g.mn[1], g.inv),
               cell_coord(z[i], g.mn[2], g.inv)};
    bucket[cell[i]].push_back(i);
  }
  // neighbour lists by the 27-bucket search
  std::vector<std::vector<int64_t>> nbr((size_t)std::max<int64_t>(n, 1));
  for (int64_t i = 0; i < n; ++i) {
    if (!valid[i]) continue;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int64_t c[3] = {(int64_t)cell[i][0] + dx, (int64_t)cell[i][1] + dy,
                                (int64_t)cell[i][2] + dz};
          if (c[0] < 0 || c[1] < 0 || c[2] < 0) continue;
          auto it = bucket.find({(uint32_t)c[0], (uint32_t)c[1], (uint32_t)c[2]});
          if (it == bucket.end()) continue;
          for (int64_t q : it->second) {
            if (q == i) continue;
            if (dist2(x[i], y[i], z[i], x[q], y[q], z[q]) <= r2) nbr[i].push_back(q);
          }
        }
  }
  std::vector<uint8_t> present(valid);
  if (count0)
    for (int64_t i = 0; i < n; ++i) count0[i] = valid[i] ? (uint32_t)nbr[i].size() : 0u;
  const uint64_t key[2] = {seed, 0};
  for (int64_t round = 0;; ++round) {
    // count the present neighbours of every present point; mark
    std::vector<int64_t> m;
    for (int64_t i = 0; i < n; ++i) {
      if (!present[i]) continue;
      uint64_t cnt = 0;
      for (int64_t q : nbr[i]) cnt += present[q];
      if (cnt > umbral) m.push_back(i);
    }
    if (marked && round < cap_rounds) marked[round] = (int64_t)m.size();
    *rounds = round + 1;
    if ((int64_t)m.size() > round_size) {
      // delete the round_size marked points of smallest (priority, index)
      std::vector<std::pair<uint64_t, int64_t>> pri;
      for (int64_t i : m) {
        const uint64_t ctr[4] = {(uint64_t)i, (uint64_t)round, 0, 0};
        uint64_t out[4];
        philox4x64_10(ctr, key, out);
        pri.push_back({out[0], i});
      }
      std::sort(pri.begin(), pri.end());
      for (int64_t k = 0; k < round_size; ++k) present[pri[k].second] = 0;
    } else {
      for (int64_t i : m) present[i] = 0;
      break;
    }
  }
  if (keep)
    for (int64_t i = 0; i < n; ++i) keep[i] = present[i];
  return VGO_OK;
}

}  // extern "C"

// Internal declarations shared by the host grid layer, the C ABI and the HIP
// kernels of libsgcm.  Not part of the public interface (include/sgcm.h).
#pragma once

#include <atomic>
#include <cstdint>
#include <memory>
#include <mutex>
#include <vector>

#include "sgcm.h"

namespace sgcm {

constexpr int kMaxDim = 8;
constexpr int kMaxLevel = 5;
constexpr int kMaxPoints = (1 << kMaxLevel) + 1;  // 1-D points at the finest level
constexpr int kMaxDevices = 64;

// 1-D point ids (see the canonical order in sgcm.h): level of id e.
inline int point_level(int e) {
  if (e == 0) return 1;
  if (e <= 2) return 2;
  int l = 0;
  while ((1 << (l + 1)) <= e - 1) ++l;  // floor(log2(e - 1))
  return l + 2;
}
// Offset t of point e inside X^{point_level(e)} (0-based, increasing coordinate).
inline int point_offset(int e) {
  if (e == 0) return 0;
  if (e == 1) return 0;
  if (e == 2) return 2;
  int i = point_level(e);
  return 2 * (e - (1 << (i - 2)) - 1) + 1;
}
// Number of 1-D points whose level excess (level - 1) is at most b.
inline int points_upto(int b) { return b <= 0 ? 1 : (1 << b) + 1; }

// Device copies of a grid's tables on one device (made by sgcm_grid_upload).
struct GridDevice {
  std::atomic<bool> ready{false};  // set once every table below is in place
  double* node_xi = nullptr;     // M x d node coordinates in [0, 1]
  int32_t* by_level = nullptr;   // node indices grouped by total excess
  int32_t* tables = nullptr;     // int tables (see Grid::itab)
  double* dtab = nullptr;        // double tables (see Grid::dtab)
  int32_t* sub_map = nullptr;    // Grid::sub_map
  double* scratch = nullptr;     // M x 3 doubles: lower-level surpluses during a build
};

struct Grid {
  int d = 0, level = 0, P = 1;   // P = number of 1-D points (points_upto(level))
  int64_t M = 0;
  double lo[kMaxDim], hi[kMaxDim], inv_width[kMaxDim];
  std::vector<int32_t> keys;     // M x d point ids, canonical order
  std::vector<double> xi;        // M x d coordinates in [0,1]
  std::vector<int32_t> by_level; // node indices ordered by total excess
  std::vector<int64_t> level_start;  // by_level[level_start[l] .. level_start[l+1])
  // Integer tables, one array:
  //   [0, P)                        excess of each 1-D point
  //   [P, P + level + 1)            points_upto(b)
  //   [itab_off, ...)               child offsets off[r][b][e], r = 1..d,
  //                                 index ((r-1)*(level+1) + b)*P + e
  std::vector<int32_t> itab;
  int itab_off = 0;
  // Double tables, per 1-D point e >= 1 (level i = point_level(e)):
  //   [0, P)            the points of the finest set X^{level+1}, increasing
  //   [P, 2P)           scale[e] = 1 / prod_{s != t(e)} (x_t - x_s) over X^i
  std::vector<double> dtab;
  // The grids of the lower levels (sub[l] of level l < level, without grids
  // of their own) and, for each, the index in this grid of each of its nodes:
  // sub_map[sub_map_off[l] + i] for node i of sub[l] (the grids are nested).
  std::vector<std::unique_ptr<Grid>> sub;
  std::vector<int64_t> sub_map_off;
  std::vector<int32_t> sub_map;
  std::mutex mu;
  GridDevice dev[kMaxDevices];
};

// Host grid construction (grid.cpp); with_sub also builds the lower-level
// grids and their node maps.
int build_grid(int d, int level, const double* lo, const double* hi, Grid* g, bool with_sub = true);

// Coordinate in [0,1] of offset t in X^i (i >= 2), t = 0..2^{i-1}.
double cgl_coordinate(int i, int t);

// Free a grid's device tables on every device that has them (interp.hip).
void free_device_tables(Grid& G);

// Make a grid's device tables (and those of its lower-level grids) on device
// dev, copied on stream s (interp.hip).
int upload_device_tables(Grid& G, int dev, void* s);

}  // namespace sgcm

struct sgcm_grid {
  sgcm::Grid g;
};

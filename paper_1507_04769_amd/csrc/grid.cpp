// Host grid layer: the Smolyak sparse grid on the nested CGL (Clenshaw-Curtis)
// sets (Sec. 3.2, eq. CGL) in the canonical order of sgcm.h, plus the small
// integer and double tables the HIP kernels walk.
//
// Layout idea: order every 1-D point by the level at which it appears; then
// the children of any prefix (e_0, .., e_{k-1}) of a node key that keep the
// total level excess within a budget b form a contiguous id range
// [0, points_upto(b)), and the nodes below a prefix are contiguous in the
// lexicographic order.  A kernel can therefore walk the grid as a trie with
// uniform control flow and read the surplus table as a stream.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "sgcm_internal.h"

namespace sgcm {

double cgl_coordinate(int i, int t) {
  // (1 - cos(t pi / n)) / 2 with n = 2^{i-1}, written as (1 - sin(pi (n - 2t) / (2n))) / 2:
  // the argument is a dyadic multiple of pi, so a point shared by two levels
  // gets bitwise the same coordinate, the middle point is exactly 1/2 and the
  // end points are exactly 0 and 1.
  if (i == 1) return 0.5;
  const double n = std::ldexp(1.0, i - 1);
  const double arg = (M_PI * (n - 2.0 * t)) / (2.0 * n);
  return 0.5 * (1.0 - std::sin(arg));
}

namespace {

// number of nodes of an r-dimensional grid with excess budget b
int64_t subgrid_size(int r, int b, std::vector<int64_t>& memo, int L) {
  if (r == 0) return 1;
  int64_t& slot = memo[(size_t)r * (L + 1) + b];
  if (slot >= 0) return slot;
  int64_t s = 0;
  for (int e = 0; e < points_upto(b); ++e) s += subgrid_size(r - 1, b - (point_level(e) - 1), memo, L);
  return slot = s;
}

void enumerate(int k, int d, int b, std::vector<int32_t>& cur, std::vector<int32_t>& keys) {
  if (k == d) {
    keys.insert(keys.end(), cur.begin(), cur.end());
    return;
  }
  for (int e = 0; e < points_upto(b); ++e) {
    cur[k] = e;
    enumerate(k + 1, d, b - (point_level(e) - 1), cur, keys);
  }
}

}  // namespace

int build_grid(int d, int level, const double* lo, const double* hi, Grid* g, bool with_sub) {
  if (d < 1 || d > kMaxDim || level < 0 || level > kMaxLevel || !lo || !hi || !g)
    return SGCM_EINVAL;
  for (int j = 0; j < d; ++j)
    if (!(std::isfinite(lo[j]) && std::isfinite(hi[j]) && lo[j] < hi[j])) return SGCM_EINVAL;
  const int L = level;
  g->d = d;
  g->level = L;
  g->P = points_upto(L);
  for (int j = 0; j < d; ++j) {
    g->lo[j] = lo[j];
    g->hi[j] = hi[j];
    g->inv_width[j] = 1.0 / (hi[j] - lo[j]);
  }
  // nodes in lexicographic key order
  std::vector<int32_t> cur(d, 0);
  g->keys.clear();
  enumerate(0, d, L, cur, g->keys);
  g->M = (int64_t)(g->keys.size() / d);
  // 1-D coordinates of every point id, all from the finest set X^{L+1}
  const int P = g->P;
  std::vector<double> coord(P);
  for (int e = 0; e < P; ++e) {
    int i = point_level(e), t = point_offset(e);
    coord[e] = (i == 1) ? 0.5 : cgl_coordinate(L + 1, t << (L + 1 - i));
  }
  g->xi.resize((size_t)g->M * d);
  for (size_t a = 0; a < g->keys.size(); ++a) g->xi[a] = coord[g->keys[a]];
  // nodes grouped by total excess (stable within a group)
  std::vector<int> tot(g->M);
  for (int64_t a = 0; a < g->M; ++a) {
    int s = 0;
    for (int j = 0; j < d; ++j) s += point_level(g->keys[a * d + j]) - 1;
    tot[a] = s;
  }
  g->by_level.clear();
  g->level_start.assign(L + 2, 0);
  for (int l = 0; l <= L; ++l) {
    g->level_start[l] = (int64_t)g->by_level.size();
    for (int64_t a = 0; a < g->M; ++a)
      if (tot[a] == l) g->by_level.push_back((int32_t)a);
  }
  g->level_start[L + 1] = (int64_t)g->by_level.size();
  // integer tables
  std::vector<int64_t> memo((size_t)(d + 1) * (L + 1), -1);
  g->itab.assign(P + (L + 1), 0);
  for (int e = 0; e < P; ++e) g->itab[e] = point_level(e) - 1;
  for (int b = 0; b <= L; ++b) g->itab[P + b] = points_upto(b);
  g->itab_off = (int)g->itab.size();
  g->itab.resize(g->itab.size() + (size_t)d * (L + 1) * P, 0);
  for (int r = 1; r <= d; ++r)
    for (int b = 0; b <= L; ++b) {
      int64_t acc = 0;
      for (int e = 0; e < points_upto(b); ++e) {
        g->itab[g->itab_off + ((r - 1) * (L + 1) + b) * P + e] = (int32_t)acc;
        acc += subgrid_size(r - 1, b - (point_level(e) - 1), memo, L);
      }
    }
  // double tables: finest points and Lagrange scale factors
  g->dtab.assign(2 * (size_t)P, 0.0);
  for (int t = 0; t < P; ++t) g->dtab[t] = (L == 0) ? 0.5 : cgl_coordinate(L + 1, t);
  g->dtab[P] = 1.0;
  for (int e = 1; e < P; ++e) {
    int i = point_level(e), t = point_offset(e);
    int n = (1 << (i - 1)) + 1;
    double xt = cgl_coordinate(i, t), prod = 1.0;
    for (int s = 0; s < n; ++s)
      if (s != t) prod *= xt - cgl_coordinate(i, s);
    g->dtab[P + e] = 1.0 / prod;
  }
  // lower-level grids: both node lists are in lexicographic key order and
  // the lower grid's keys are a subset, so one merge pass maps them
  g->sub.clear();
  g->sub_map.clear();
  g->sub_map_off.assign(1, 0);
  if (with_sub) {
    for (int l = 0; l < L; ++l) {
      g->sub.emplace_back(new Grid());
      Grid* s = g->sub.back().get();
      const int rc = build_grid(d, l, lo, hi, s, false);
      if (rc != SGCM_OK) return rc;
      int64_t a = 0;
      for (int64_t i = 0; i < s->M; ++i) {
        while (a < g->M && !std::equal(s->keys.begin() + i * d, s->keys.begin() + (i + 1) * d,
                                       g->keys.begin() + a * d))
          ++a;
        if (a == g->M) return SGCM_EINVAL;  // not nested: cannot happen for these grids
        g->sub_map.push_back((int32_t)a);
      }
      g->sub_map_off.push_back((int64_t)g->sub_map.size());
    }
  }
  return SGCM_OK;
}

}  // namespace sgcm

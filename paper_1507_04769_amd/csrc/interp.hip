// Sparse-grid interpolant on gfx950: hierarchical surpluses (Sec. 3.3,
// eq. interpo) and the on-line evaluation of the feedback interpolant.
//
// Both kernels share one device routine: the sum over sparse-grid nodes of
// w(node) * prod_k a^{i_k}(xi_k).  The nodes are stored in lexicographic order
// of their point-id keys, with 1-D point ids ordered by level, so the node set
// is a trie whose children at every depth form a contiguous id range
// [0, points_upto(budget)).  One lane owns one evaluation point; every lane
// walks the same trie with the same (uniform) control flow, so the surplus
// table is read through scalar loads and multiplied into per-lane partial
// products:
//     acc += p_{d-2} * sum_{e} b_{d-1}[e] * w[base + e],
//     p_k = p_{k-1} * b_k[e_k]  at every trie node.
// The 1-D basis values b_k[e] (Lagrange polynomials on X^i for the new points
// of level i, Sec. 3.3) are built once per lane by prefix/suffix products over
// X^i: the innermost dimension lives in registers, the outer ones in LDS laid
// out [dim][point][lane] so that every LDS access is lane-private and
// conflict free.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <vector>

#include "sgcm_internal.h"
#include "trace.h"

namespace sgcm {
namespace {

struct GridArgs {
  int d, L, P;
  const int32_t* excess;  // P
  const int32_t* off;     // child offsets [(r-1)*(L+1) + b][P]
  const double* X;        // finest 1-D set X^{L+1} (P points)
  const double* scale;    // P Lagrange scale factors
  double lo[kMaxDim], inv_width[kMaxDim];
};

__host__ __device__ constexpr int upto(int b) { return b <= 0 ? 1 : (1 << b) + 1; }

// Lagrange basis values of the new points of level I (2 <= I <= L+1) at xi,
// from prefix and suffix products of (xi - x_s) over X^I.
// F is the arithmetic type (double; float for the FP32 evaluation path, whose
// point and scale tables are rounded from the FP64 ones).
template <int L, int I, typename F = double, int IMAX = L + 1>
__device__ __forceinline__ void level_basis(const GridArgs& g, F xi, F (&out)[kMaxPoints]) {
  if constexpr (I <= IMAX) {
    constexpr int n = (1 << (I - 1)) + 1;
    constexpr int stride = 1 << (L + 1 - I);
    // suffix products suf[s] = prod_{s' > s} (xi - x_s'), then one forward
    // sweep with a running prefix product
    F suf[n];
    suf[n - 1] = F(1);
#pragma unroll
    for (int s = n - 2; s >= 0; --s) suf[s] = suf[s + 1] * (xi - (F)g.X[(s + 1) * stride]);
    F pre = F(1);
#pragma unroll
    for (int s = 0; s < n; ++s) {
      if constexpr (I == 2) {
        if (s != 1) out[1 + s / 2] = pre * suf[s] * (F)g.scale[1 + s / 2];
      } else {
        if (s & 1) {
          constexpr int base = (1 << (I - 2)) + 1;
          out[base + s / 2] = pre * suf[s] * (F)g.scale[base + s / 2];
        }
      }
      pre *= xi - (F)g.X[s * stride];
    }
    level_basis<L, I + 1, F, IMAX>(g, xi, out);
  }
}

__host__ __device__ constexpr int bit_length(int v) { return v == 0 ? 0 : 1 + bit_length(v >> 1); }

// The basis value of point E of the nested 1-D sets at xi, alone: the
// Lagrange polynomial on X^I (I the level of E) that is 1 at the point, with
// the factors of level_basis in the same order (the prefix, then the suffix
// from the right, then the scale), so the same bits as level_basis.
template <int L, int E, typename F>
__device__ __forceinline__ F basis_point(const GridArgs& g, F xi) {
  if constexpr (E == 0) {
    return F(1);
  } else {
    constexpr int I = E <= 2 ? 2 : bit_length(E - 1) + 1;
    constexpr int n = (1 << (I - 1)) + 1;
    constexpr int stride = 1 << (L + 1 - I);
    constexpr int s = I == 2 ? 2 * (E - 1) : 2 * (E - ((1 << (I - 2)) + 1)) + 1;
    F suf = F(1);
#pragma unroll
    for (int t = n - 1; t > s; --t) suf = suf * (xi - (F)g.X[t * stride]);
    F pre = F(1);
#pragma unroll
    for (int t = 0; t < s; ++t) pre *= xi - (F)g.X[t * stride];
    return pre * suf * (F)g.scale[E];
  }
}

// basis_point for a run-time point e < N (a wave-uniform value)
template <int L, int E, int N, typename F>
__device__ __forceinline__ F basis_point_rt(const GridArgs& g, F xi, int e) {
  if constexpr (E + 1 < N) {
    if (e == E) return basis_point<L, E, F>(g, xi);
    return basis_point_rt<L, E + 1, N, F>(g, xi, e);
  } else {
    return basis_point<L, E, F>(g, xi);
  }
}

template <int L, typename F = double>
__device__ __forceinline__ void basis_row_l(const GridArgs& g, F xi, F (&out)[kMaxPoints]) {
  out[0] = F(1);
  level_basis<L, 2, F>(g, xi, out);
}

// The values of the points below the finest level (out[0 .. upto(L - 1))).
template <int L, typename F>
__device__ __forceinline__ void basis_row_below(const GridArgs& g, F xi, F (&out)[kMaxPoints]) {
  out[0] = F(1);
  level_basis<L, 2, F, L>(g, xi, out);
}

__device__ __forceinline__ void basis_row(const GridArgs& g, double xi, double (&out)[kMaxPoints]) {
  switch (g.L) {
    case 0: basis_row_l<0>(g, xi, out); break;
    case 1: basis_row_l<1>(g, xi, out); break;
    case 2: basis_row_l<2>(g, xi, out); break;
    case 3: basis_row_l<3>(g, xi, out); break;
    case 4: basis_row_l<4>(g, xi, out); break;
    default: basis_row_l<5>(g, xi, out); break;
  }
}

// t += sum over the first N points of the last dimension of bin[e] w[e]
// (unrolled: static indices into bin, no predicated iterations past N).
template <int N, int MC>
__device__ __forceinline__ void last_dim_sum(const double (&bin)[kMaxPoints], const double* __restrict__ wb, int m,
                                             double (&t)[MC]) {
#pragma unroll
  for (int e = 0; e < N; ++e)
#pragma unroll
    for (int c = 0; c < MC; ++c) t[c] = fma(bin[e], wb[(int64_t)e * m + c], t[c]);
}

// Walk the trie below depth K.  bL: excess budget of the storage layout (the
// full grid), bE: excess budget of the nodes summed (bE <= bL; a smaller bE
// evaluates a coarser interpolant I^{q'} with the same surplus table).
template <int K, int D, int MC>
__device__ __forceinline__ void walk(const GridArgs& g, const double* __restrict__ w, int m,
                                     int col0, int bL, int bE, int64_t base, double p,
                                     double (&acc)[MC], const double (&bin)[kMaxPoints],
                                     const double* lds_lane) {
  if constexpr (K == D - 1) {
    const int cE = upto(bE);
    const double* wb = w + base * m + col0;
    double t[MC];
#pragma unroll
    for (int c = 0; c < MC; ++c) t[c] = 0.0;
    static_assert(kMaxPoints == 33, "the point counts of the levels 0..5");
    switch (cE) {  // upto(bE): 1, 3, 5, 9, 17 or 33 points
      case 1: last_dim_sum<1, MC>(bin, wb, m, t); break;
      case 3: last_dim_sum<3, MC>(bin, wb, m, t); break;
      case 5: last_dim_sum<5, MC>(bin, wb, m, t); break;
      case 9: last_dim_sum<9, MC>(bin, wb, m, t); break;
      case 17: last_dim_sum<17, MC>(bin, wb, m, t); break;
      default: last_dim_sum<33, MC>(bin, wb, m, t); break;
    }
#pragma unroll
    for (int c = 0; c < MC; ++c) acc[c] = fma(p, t[c], acc[c]);
  } else {
    const int cE = upto(bE);
    const int32_t* offrow = g.off + ((D - K - 1) * (g.L + 1) + bL) * g.P;
    for (int e = 0; e < cE; ++e) {
      const int ex = g.excess[e];
      const double pk = (K == 0) ? lds_lane[(K * g.P + e) * 64] : p * lds_lane[(K * g.P + e) * 64];
      walk<K + 1, D, MC>(g, w, m, col0, bL - ex, bE - ex, base + offrow[e], pk, acc, bin, lds_lane);
    }
  }
}

// Basis tables of one lane at xi[0..D-1]: dims 0..D-2 to LDS, dim D-1 to bin.
template <int D>
__device__ __forceinline__ void lane_tables(const GridArgs& g, const double (&xi)[D], double* lds_lane,
                                            double (&bin)[kMaxPoints]) {
  double row[kMaxPoints];
#pragma unroll
  for (int k = 0; k < D - 1; ++k) {
    basis_row(g, xi[k], row);
#pragma unroll
    for (int e = 0; e < kMaxPoints; ++e)
      if (e < g.P) lds_lane[(k * g.P + e) * 64] = row[e];
  }
  basis_row(g, xi[D - 1], bin);
}

template <int D, int MC>
__global__ __launch_bounds__(64) void k_eval(GridArgs g, const double* __restrict__ w, int m, int col0,
                                             int64_t nq, const double* __restrict__ xq,
                                             double* __restrict__ uq) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x;
  const int64_t q = (int64_t)blockIdx.x * 64 + lane;
  const bool active = q < nq;
  double xi[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xi[k] = active ? (xq[q * D + k] - g.lo[k]) * g.inv_width[k] : 0.5;
  double bin[kMaxPoints];
  double* lds_lane = lds + lane;
  lane_tables<D>(g, xi, lds_lane, bin);
  double acc[MC];
#pragma unroll
  for (int c = 0; c < MC; ++c) acc[c] = 0.0;
  walk<0, D, MC>(g, w, m, col0, g.L, g.L, 0, 1.0, acc, bin, lds_lane);
  if (active) {
#pragma unroll
    for (int c = 0; c < MC; ++c) uq[q * m + col0 + c] = acc[c];
  }
}

template <int D, int MC>
__global__ __launch_bounds__(64) void k_surplus_level(GridArgs g, const double* __restrict__ f,
                                                      double* w, int m, int col0, int lv,
                                                      const int32_t* __restrict__ nodes, int64_t count,
                                                      const double* __restrict__ node_xi) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const bool active = i < count;
  const int64_t node = active ? nodes[i] : 0;
  double xi[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xi[k] = node_xi[node * D + k];
  double bin[kMaxPoints];
  double* lds_lane = lds + lane;
  lane_tables<D>(g, xi, lds_lane, bin);
  double acc[MC];
#pragma unroll
  for (int c = 0; c < MC; ++c) acc[c] = 0.0;
  if (lv > 0) walk<0, D, MC>(g, w, m, col0, g.L, lv - 1, 0, 1.0, acc, bin, lds_lane);
  if (active) {
#pragma unroll
    for (int c = 0; c < MC; ++c) w[node * m + col0 + c] = f[node * m + col0 + c] - acc[c];
  }
}

// ---- the generic walk split over the wavefronts of a workgroup -----------------
//
// The generic kernels keep (d - 1) * 33 basis values per lane in LDS (50 KB per
// wavefront at d = 4), so a one-wavefront workgroup leaves a compute unit
// three wavefronts, each walking its whole trie alone.  Here kGenWaves
// wavefronts share one copy of the tables of their 64 points and split the
// walk's outermost loop (the points e0 of dimension 0) into contiguous
// blocks (gen_bounds); the block sums are added from zero in wavefront order.

constexpr int kGenWaves = 4;

// The rows of dimensions 0..D-2 into the group's LDS (dimension k by
// wavefront k mod kGenWaves), the last one into bin (every wavefront); ends
// with a barrier.
template <int D>
__device__ __forceinline__ void gen_tables(const GridArgs& g, const double (&xi)[D], int wave, double* lds_lane,
                                           double (&bin)[kMaxPoints]) {
  double row[kMaxPoints];
#pragma unroll
  for (int k = 0; k < D - 1; ++k) {
    if (k % kGenWaves == wave) {
      basis_row(g, xi[k], row);
#pragma unroll
      for (int e = 0; e < kMaxPoints; ++e)
        if (e < g.P) lds_lane[(k * g.P + e) * 64] = row[e];
    }
  }
  basis_row(g, xi[D - 1], bin);
  __syncthreads();
}

// walk<0, D, MC> restricted to the points e0 in [e_lo, e_hi) of dimension 0.
template <int D, int MC>
__device__ __forceinline__ void walk0_range(const GridArgs& g, const double* __restrict__ w, int m, int col0,
                                            int bL, int bE, int e_lo, int e_hi, double (&acc)[MC],
                                            const double (&bin)[kMaxPoints], const double* lds_lane) {
  static_assert(D >= 2, "the split walks the first of at least two dimensions");
  const int cE = upto(bE);
  const int hi = e_hi < cE ? e_hi : cE;
  const int32_t* offrow = g.off + ((D - 1) * (g.L + 1) + bL) * g.P;
  for (int e = e_lo; e < hi; ++e) {
    const int ex = g.excess[e];
    walk<1, D, MC>(g, w, m, col0, bL - ex, bE - ex, offrow[e], lds_lane[e * 64], acc, bin, lds_lane);
  }
}

// The block sums (this wavefront's in acc) added from zero in wavefront order
// by wavefront 0 (into its acc).
template <int MC>
__device__ __forceinline__ void gen_reduce(double* part, int wave, int lane, double (&acc)[MC]) {
#pragma unroll
  for (int c = 0; c < MC; ++c) part[(wave * 64 + lane) * MC + c] = acc[c];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int c = 0; c < MC; ++c) {
      double t = 0.0;
#pragma unroll
      for (int r = 0; r < kGenWaves; ++r) t += part[(r * 64 + lane) * MC + c];
      acc[c] = t;
    }
  }
}

// Wavefront s walks the points e0 from byte s - 1 of bounds (0 for s = 0) up
// to byte s (0xff: to the end).
__device__ __forceinline__ int gen_lo(uint32_t bounds, int s) {
  return s == 0 ? 0 : (int)((bounds >> (8 * (s - 1))) & 0xffu);
}
__device__ __forceinline__ int gen_hi(uint32_t bounds, int s) { return (int)((bounds >> (8 * s)) & 0xffu); }

template <int D, int MC>
__global__ __launch_bounds__(64 * kGenWaves) void k_eval_gs(GridArgs g, const double* __restrict__ w, int m,
                                                            int col0, int64_t nq, const double* __restrict__ xq,
                                                            double* __restrict__ uq, uint32_t bounds) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t q = (int64_t)blockIdx.x * 64 + lane;
  const bool active = q < nq;
  double xi[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xi[k] = active ? (xq[q * D + k] - g.lo[k]) * g.inv_width[k] : 0.5;
  double bin[kMaxPoints];
  double* lds_lane = lds + lane;
  gen_tables<D>(g, xi, wave, lds_lane, bin);
  double acc[MC];
#pragma unroll
  for (int c = 0; c < MC; ++c) acc[c] = 0.0;
  walk0_range<D, MC>(g, w, m, col0, g.L, g.L, gen_lo(bounds, wave), gen_hi(bounds, wave), acc, bin, lds_lane);
  gen_reduce<MC>(lds + (D - 1) * g.P * 64, wave, lane, acc);
  if (wave == 0 && active) {
#pragma unroll
    for (int c = 0; c < MC; ++c) uq[q * m + col0 + c] = acc[c];
  }
}

template <int D, int MC>
__global__ __launch_bounds__(64 * kGenWaves) void k_surplus_level_gs(GridArgs g, const double* __restrict__ f,
                                                                     double* w, int m, int col0, int lv,
                                                                     const int32_t* __restrict__ nodes,
                                                                     int64_t count,
                                                                     const double* __restrict__ node_xi,
                                                                     uint32_t bounds) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const bool active = i < count;
  const int64_t node = active ? nodes[i] : 0;
  double xi[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xi[k] = node_xi[node * D + k];
  double bin[kMaxPoints];
  double* lds_lane = lds + lane;
  gen_tables<D>(g, xi, wave, lds_lane, bin);
  double acc[MC];
#pragma unroll
  for (int c = 0; c < MC; ++c) acc[c] = 0.0;
  if (lv > 0)
    walk0_range<D, MC>(g, w, m, col0, g.L, lv - 1, gen_lo(bounds, wave), gen_hi(bounds, wave), acc, bin, lds_lane);
  gen_reduce<MC>(lds + (D - 1) * g.P * 64, wave, lane, acc);
  if (wave == 0 && active) {
#pragma unroll
    for (int c = 0; c < MC; ++c) w[node * m + col0 + c] = f[node * m + col0 + c] - acc[c];
  }
}

// ---- evaluation with the inner trie unrolled at compile time -----------------
//
// For a fixed (d, level, m) the trie below any prefix of the outer dimensions
// depends only on the remaining excess budget, so the sum over the four
// innermost dimensions is generated at compile time: their basis values sit in
// registers with static indices, the surplus is read at immediate offsets from
// a uniform base (scalar loads), and no loop or LDS access remains in the hot
// part.  The outer dimensions are walked at run time with their basis values
// in LDS, as in the generic kernel.

__host__ __device__ constexpr int excess_of(int e) {
  if (e == 0) return 0;
  if (e <= 2) return 1;
  int l = 0;
  while ((1 << (l + 1)) <= e - 1) ++l;
  return l + 1;
}

__host__ __device__ constexpr int subgrid(int r, int b) {
  if (r == 0) return 1;
  int s = 0;
  for (int e = 0; e < upto(b); ++e) s += subgrid(r - 1, b - excess_of(e));
  return s;
}

__host__ __device__ constexpr int child_off(int r, int b, int e) {
  int s = 0;
  for (int q = 0; q < e; ++q) s += subgrid(r - 1, b - excess_of(q));
  return s;
}

// Up to level 3 (P <= 9 points per dimension), a sum over the last dimension
// of fewer points than kShortTail adds each term to the accumulator with its
// own product pe * b (one multiply per point); otherwise it sums b * w first
// and multiplies by pe once, which costs a copy of its first surplus into a
// register (two moves per component).  Per group of n points: 4n against
// 3n + 7 VALU instructions at m = 3, so the groups of 3 and 5 points take the
// short form.  At level 3 it also frees registers (a fifth wavefront per SIMD
// at m = 3): 7 % less time per query.  At level 4, with three wavefronts per
// SIMD, the one accumulator chain per component of the short form hid less
// latency than the instructions it saves (1e6 queries: 0.6 % slower).
constexpr int kShortTail = 7;
constexpr int kShortTailMaxPoints = 9;

// Sum over the subtree of R remaining (unrolled) dimensions with budget B whose
// nodes start at offset OFF; E is the child being visited.  bv[j] holds the
// basis values of unrolled dimension j.
template <int KU, int P, int M, int R, int B, int OFF, int E, typename F>
__device__ __forceinline__ void uwalk(const F (&bv)[KU][P], const F* __restrict__ w, F p, F (&acc)[M]) {
  if constexpr (E < upto(B)) {
    constexpr int ex = excess_of(E);
    constexpr int off = OFF + child_off(R, B, E);
    if constexpr (R == 1) {
      const F pe = p * bv[KU - 1][E];
#pragma unroll
      for (int c = 0; c < M; ++c) acc[c] = fma(pe, w[off * M + c], acc[c]);
    } else if constexpr (R == 2) {
      // the sum over the last dimension starts from its first point, whose
      // basis value is the constant 1: the term is the surplus itself, and
      // where it is the only term (no budget left) it goes straight into acc
      constexpr int n = upto(B - ex);
      const F pe = p * bv[KU - 2][E];
      if constexpr (n == 1) {
#pragma unroll
        for (int c = 0; c < M; ++c) acc[c] = fma(pe, w[off * M + c], acc[c]);
      } else if constexpr (n < kShortTail && P <= kShortTailMaxPoints) {
        // short sums: every term straight into acc, the first with pe, the
        // others with pe times their basis value
#pragma unroll
        for (int c = 0; c < M; ++c) acc[c] = fma(pe, w[off * M + c], acc[c]);
#pragma unroll
        for (int q = 1; q < n; ++q) {
          const F pq = pe * bv[KU - 1][q];
#pragma unroll
          for (int c = 0; c < M; ++c) acc[c] = fma(pq, w[(off + q) * M + c], acc[c]);
        }
      } else {
        F t[M];
#pragma unroll
        for (int c = 0; c < M; ++c) t[c] = w[off * M + c];
#pragma unroll
        for (int q = 1; q < n; ++q)
#pragma unroll
          for (int c = 0; c < M; ++c) t[c] = fma(bv[KU - 1][q], w[(off + q) * M + c], t[c]);
#pragma unroll
        for (int c = 0; c < M; ++c) acc[c] = fma(pe, t[c], acc[c]);
      }
    } else {
      uwalk<KU, P, M, R - 1, B - ex, off, 0, F>(bv, w, p * bv[KU - R][E], acc);
    }
    uwalk<KU, P, M, R, B, OFF, E + 1, F>(bv, w, p, acc);
  }
}

template <int KU, int P, int M, int BB, typename F>
__device__ __forceinline__ void uwalk_budget(int b, const F (&bv)[KU][P], const F* __restrict__ w, F p,
                                             F (&acc)[M]) {
  if (b == BB) {
    uwalk<KU, P, M, KU, BB, 0, 0, F>(bv, w, p, acc);
  } else if constexpr (BB > 0) {
    uwalk_budget<KU, P, M, BB - 1, F>(b, bv, w, p, acc);
  }
}

// The outer (run-time) dimensions of the trie walk, their basis values in LDS
// at lds_lane[(K * P + e) * 64].  With LOW0, dimension 0 keeps only its
// values of the finest level there, after the other outer dimensions' (at
// [((KO - 1) * P + e - upto(L - 1)) * 64]), and its lower-level values are
// formed from xi0 when the walk reaches them (each once per query): half the
// LDS per lane, so more waves per compute unit.
template <int D, int L, int M, int KO, int KU, int K, bool LOW0, typename F>
__device__ __forceinline__ void owalk(const GridArgs& g, const F* __restrict__ w, int bL, int64_t base, F p,
                                      F (&acc)[M], const F (&bv)[KU][upto(L)], const F* lds_lane, F xi0) {
  constexpr int P = upto(L);
  if constexpr (K == KO) {
    uwalk_budget<KU, P, M, L, F>(bL, bv, w + base * M, p, acc);
  } else {
    const int cE = upto(bL);
    const int32_t* offrow = g.off + ((D - K - 1) * (L + 1) + bL) * P;
    for (int e = 0; e < cE; ++e) {
      const int ex = g.excess[e];
      F pk;
      if constexpr (K == 0 && LOW0) {
        constexpr int PL = upto(L - 1);
        pk = e < PL ? basis_point_rt<L, 0, PL, F>(g, xi0, e) : lds_lane[((KO - 1) * P + e - PL) * 64];
      } else if constexpr (K == 0) {
        pk = lds_lane[e * 64];
      } else {
        pk = p * lds_lane[((LOW0 ? K - 1 : K) * P + e) * 64];
      }
      owalk<D, L, M, KO, KU, K + 1, LOW0, F>(g, w, bL - ex, base + offrow[e], pk, acc, bv, lds_lane, xi0);
    }
  }
}

// The interpolant of a level-L grid (d = D, m = M) at one point per lane:
// xi_of(k) is the lane's coordinate in [0, 1] along dimension k.
template <int D, int L, int M, typename F, typename XiOf>
__device__ __forceinline__ void fast_point(const GridArgs& g, const F* __restrict__ w, XiOf xi_of, F (&acc)[M]) {
  constexpr int P = upto(L);
  constexpr int KU = D < 4 ? D : 4;
  constexpr int KO = D - KU;
  extern __shared__ double lds_d[];
  F* lds = reinterpret_cast<F*>(lds_d);
  const int lane = threadIdx.x;
  F* lds_lane = lds + lane;
  F bv[KU][P];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const F xi = xi_of(k);
    F row[kMaxPoints];
    basis_row_l<L, F>(g, xi, row);
    if (k < KO) {
#pragma unroll
      for (int e = 0; e < P; ++e) lds_lane[(k * P + e) * 64] = row[e];
    } else {
#pragma unroll
      for (int e = 0; e < P; ++e) bv[k - KO][e] = row[e];
    }
  }
#pragma unroll
  for (int c = 0; c < M; ++c) acc[c] = F(0);
  owalk<D, L, M, KO, KU, 0, false, F>(g, w, L, 0, F(1), acc, bv, lds_lane, F(0));
}

// ---- the evaluation walk with the finest level formed where it is used -------
//
// A point of the finest level of a dimension has the whole excess budget, so
// it appears in exactly one trie path per evaluation point: the one where
// every other dimension sits at its level-1 point.  Its basis value is then
// formed where that path reaches it (basis_point: the same bits as the row
// computation) instead of being kept for the whole walk: per lane only the
// values below the finest level stay in registers (the inner dimensions) and
// LDS (the outer ones but the first, whose values are all used once and all
// formed where reached), which leaves room for more wavefronts per SIMD.
// That pays where the registers bound the kernel at one wavefront per SIMD
// (FP64 at level 5: two instead of one, half the time); at the lower levels
// and in FP32 the values formed again cost more than the occupancy gains.

// Basis value of point E of inner dimension J.
template <int L, int KU, int J, int E, typename F>
__device__ __forceinline__ F ubasis(const GridArgs& g, const F (&bv)[KU][upto(L - 1)], const F (&xin)[KU]) {
  if constexpr (E < upto(L - 1)) {
    return bv[J][E];
  } else {
    return basis_point<L, E, F>(g, xin[J]);
  }
}

// t += sum over points Q..N-1 of the last dimension of b[Q] w[OFF + Q].
template <int L, int KU, int M, int Q, int N, int OFF, typename F>
__device__ __forceinline__ void utail(const GridArgs& g, const F (&bv)[KU][upto(L - 1)], const F (&xin)[KU],
                                      const F* __restrict__ w, F (&t)[M]) {
  if constexpr (Q < N) {
    const F b = ubasis<L, KU, KU - 1, Q, F>(g, bv, xin);
#pragma unroll
    for (int c = 0; c < M; ++c) t[c] = fma(b, w[(OFF + Q) * M + c], t[c]);
    utail<L, KU, M, Q + 1, N, OFF, F>(g, bv, xin, w, t);
  }
}

// uwalk with the finest level formed where reached.
template <int L, int KU, int M, int R, int B, int OFF, int E, typename F>
__device__ __forceinline__ void uwalk_f(const GridArgs& g, const F (&bv)[KU][upto(L - 1)], const F (&xin)[KU],
                                        const F* __restrict__ w, F p, F (&acc)[M]) {
  if constexpr (E < upto(B)) {
    constexpr int ex = excess_of(E);
    constexpr int off = OFF + child_off(R, B, E);
    if constexpr (R == 1) {
      const F pe = p * ubasis<L, KU, KU - 1, E, F>(g, bv, xin);
#pragma unroll
      for (int c = 0; c < M; ++c) acc[c] = fma(pe, w[off * M + c], acc[c]);
    } else if constexpr (R == 2) {
      constexpr int n = upto(B - ex);
      const F pe = p * ubasis<L, KU, KU - 2, E, F>(g, bv, xin);
      if constexpr (n == 1) {
#pragma unroll
        for (int c = 0; c < M; ++c) acc[c] = fma(pe, w[off * M + c], acc[c]);
      } else {
        F t[M];
#pragma unroll
        for (int c = 0; c < M; ++c) t[c] = w[off * M + c];
        utail<L, KU, M, 1, n, off, F>(g, bv, xin, w, t);
#pragma unroll
        for (int c = 0; c < M; ++c) acc[c] = fma(pe, t[c], acc[c]);
      }
    } else {
      uwalk_f<L, KU, M, R - 1, B - ex, off, 0, F>(g, bv, xin, w, p * ubasis<L, KU, KU - R, E, F>(g, bv, xin), acc);
    }
    uwalk_f<L, KU, M, R, B, OFF, E + 1, F>(g, bv, xin, w, p, acc);
  }
}

template <int L, int KU, int M, int BB, typename F>
__device__ __forceinline__ void uwalk_f_budget(int b, const F (&bv)[KU][upto(L - 1)], const F (&xin)[KU],
                                               const GridArgs& g, const F* __restrict__ w, F p, F (&acc)[M]) {
  if (b == BB) {
    uwalk_f<L, KU, M, KU, BB, 0, 0, F>(g, bv, xin, w, p, acc);
  } else if constexpr (BB > 0) {
    uwalk_f_budget<L, KU, M, BB - 1, F>(b, bv, xin, g, w, p, acc);
  }
}

// The outer dimensions: dimension 0's values formed where reached (each is
// used once), those of dimensions 1..KO-1 below the finest level in LDS at
// lds_lane[((K - 1) * upto(L - 1) + e) * 64].
template <int D, int L, int M, int KO, int KU, int K, typename F>
__device__ __forceinline__ void owalk_f(const GridArgs& g, const F* __restrict__ w, int bL, int64_t base, F p,
                                        F (&acc)[M], const F (&bv)[KU][upto(L - 1)], const F (&xin)[KU],
                                        const F (&xout)[KO], const F* lds_lane) {
  constexpr int P = upto(L), PL = upto(L - 1);
  if constexpr (K == KO) {
    uwalk_f_budget<L, KU, M, L, F>(bL, bv, xin, g, w + base * M, p, acc);
  } else {
    const int cE = upto(bL);
    const int32_t* offrow = g.off + ((D - K - 1) * (L + 1) + bL) * P;
    for (int e = 0; e < cE; ++e) {
      const int ex = g.excess[e];
      F pk;
      if constexpr (K == 0) {
        pk = basis_point_rt<L, 0, P, F>(g, xout[0], e);
      } else {
        pk = p * (e < PL ? lds_lane[((K - 1) * PL + e) * 64] : basis_point_rt<L, PL, P, F>(g, xout[K], e));
      }
      owalk_f<D, L, M, KO, KU, K + 1, F>(g, w, bL - ex, base + offrow[e], pk, acc, bv, xin, xout, lds_lane);
    }
  }
}

// Whether the evaluation kernel forms dimension 0's lower-level basis values
// when reached instead of keeping them in LDS: in FP64 up to level 4, where the
// LDS bounds the waves per compute unit (at level 4: 9 workgroups of 17 KB,
// 12 of 13 KB), not at level 5 (bound by registers) or in FP32 (by registers
// after the first halving).
template <int L, typename F>
__host__ __device__ constexpr bool eval_low0() {
  return sizeof(F) == 8 && L <= 4;
}

// Whether the evaluation takes k_eval_fine (the finest level formed where
// used): FP64 at level 5, where k_eval_fast needs 256 registers.
template <int L, typename F>
__host__ __device__ constexpr bool eval_fine() {
  return sizeof(F) == 8 && L >= 5;
}

// F = double: the FP64 path.  F = float: the FP32 path (surplus, states and
// outputs in FP32; the map to the unit cube in FP64, then rounded).
// (The body is fast_point's, written out: through the shared routine the
// compiler allocated this kernel's registers differently and it ran slower.)
template <int D, int L, int M, typename F = double>
__global__ __launch_bounds__(64) void k_eval_fast(GridArgs g, const F* __restrict__ w, int64_t nq,
                                                  const F* __restrict__ xq, F* __restrict__ uq) {
  constexpr int P = upto(L);
  constexpr int KU = D < 4 ? D : 4;
  constexpr int KO = D - KU;
  extern __shared__ double lds_d[];
  F* lds = reinterpret_cast<F*>(lds_d);
  const int lane = threadIdx.x;
  const int64_t q = (int64_t)blockIdx.x * 64 + lane;
  const bool active = q < nq;
  F* lds_lane = lds + lane;
  F bv[KU][P];
  F xi0 = F(0);
  constexpr bool LOW0 = eval_low0<L, F>();
  constexpr int PL = upto(L - 1);  // dimension 0's points below the finest level
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const F xi = active ? (F)(((double)xq[q * D + k] - g.lo[k]) * g.inv_width[k]) : F(0.5);
    F row[kMaxPoints];
    basis_row_l<L, F>(g, xi, row);
    if (k == 0 && LOW0) {
      xi0 = xi;
#pragma unroll
      for (int e = PL; e < P; ++e) lds_lane[((KO - 1) * P + e - PL) * 64] = row[e];
    } else if (k < KO) {
#pragma unroll
      for (int e = 0; e < P; ++e) lds_lane[((LOW0 ? k - 1 : k) * P + e) * 64] = row[e];
    } else {
#pragma unroll
      for (int e = 0; e < P; ++e) bv[k - KO][e] = row[e];
    }
  }
  F acc[M];
#pragma unroll
  for (int c = 0; c < M; ++c) acc[c] = F(0);
  owalk<D, L, M, KO, KU, 0, LOW0, F>(g, w, L, 0, F(1), acc, bv, lds_lane, xi0);
  if (active) {
#pragma unroll
    for (int c = 0; c < M; ++c) uq[q * M + c] = acc[c];
  }
}

// The evaluation kernel with the walk of owalk_f (same results, bit for bit).
template <int D, int L, int M, typename F = double>
__global__ __launch_bounds__(64) void k_eval_fine(GridArgs g, const F* __restrict__ w, int64_t nq,
                                                  const F* __restrict__ xq, F* __restrict__ uq) {
  constexpr int PL = upto(L - 1);
  constexpr int KU = D < 4 ? D : 4;
  constexpr int KO = D - KU;
  static_assert(KO >= 1, "the evaluation kernel walks at least one outer dimension");
  extern __shared__ double lds_d[];
  F* lds = reinterpret_cast<F*>(lds_d);
  const int lane = threadIdx.x;
  const int64_t q = (int64_t)blockIdx.x * 64 + lane;
  const bool active = q < nq;
  F* lds_lane = lds + lane;
  F bv[KU][PL], xin[KU], xout[KO];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const F xi = active ? (F)(((double)xq[q * D + k] - g.lo[k]) * g.inv_width[k]) : F(0.5);
    if (k == 0) {
      xout[0] = xi;
      continue;
    }
    F row[kMaxPoints];
    basis_row_below<L, F>(g, xi, row);
    if (k < KO) {
      xout[k] = xi;
#pragma unroll
      for (int e = 0; e < PL; ++e) lds_lane[((k - 1) * PL + e) * 64] = row[e];
    } else {
      xin[k - KO] = xi;
#pragma unroll
      for (int e = 0; e < PL; ++e) bv[k - KO][e] = row[e];
    }
  }
  F acc[M];
#pragma unroll
  for (int c = 0; c < M; ++c) acc[c] = F(0);
  owalk_f<D, L, M, KO, KU, 0, F>(g, w, L, 0, F(1), acc, bv, xin, xout, lds_lane);
  if (active) {
#pragma unroll
    for (int c = 0; c < M; ++c) uq[q * M + c] = acc[c];
  }
}

// ---- surplus build with the unrolled walk (d = 6, m <= 3) --------------------
//
// The surplus of a node of total excess lv is f - I^{lv-1}(f) at the node
// (eq. interpo), where I^{lv-1} is the interpolant of the level-(lv - 1) grid:
// its nodes are the nodes of excess < lv, with the same surpluses (the grids
// are nested).  One level is then a gather of the lower levels' surpluses
// into that grid's canonical order, and the unrolled evaluation of that grid
// at the level-lv nodes with f - I^{lv-1}(f) stored as their surpluses.

// Excess 0 and 1: the center node's surplus is its value; I^0 is that
// constant.  nodes: the center, then the n - 1 nodes of excess 1.
__global__ __launch_bounds__(64) void k_surplus_low(const int32_t* __restrict__ nodes, int64_t n, int m,
                                                    const double* __restrict__ f, double* __restrict__ w) {
  const int64_t q = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (q >= n * m) return;
  const int64_t i = q / m;
  const int c = (int)(q - i * m);
  const int64_t c0 = nodes[0], ni = nodes[i];
  w[ni * m + c] = i == 0 ? f[c0 * m + c] : f[ni * m + c] - f[c0 * m + c];
}

// out[i][c] = w[map[i]][c], i < n
__global__ __launch_bounds__(256) void k_gather_rows(const int32_t* __restrict__ map, int64_t n, int m,
                                                     const double* __restrict__ w, double* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= n * m) return;
  const int64_t i = q / m;
  const int c = (int)(q - i * m);
  out[q] = w[(int64_t)map[i] * m + c];
}

// Surpluses of the n nodes nodes[0 .. n) (node coordinates node_xi of the
// full grid) from the level-L grid g with surpluses wsub.
template <int D, int L, int M>
__global__ __launch_bounds__(64) void k_surplus_fast(GridArgs g, const double* __restrict__ wsub, int64_t n,
                                                     const int32_t* __restrict__ nodes,
                                                     const double* __restrict__ node_xi,
                                                     const double* __restrict__ f, double* __restrict__ w) {
  const int64_t q = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const bool active = q < n;
  const int64_t node = active ? nodes[q] : 0;
  double acc[M];
  fast_point<D, L, M, double>(g, wsub, [&](int k) { return active ? node_xi[node * D + k] : 0.5; }, acc);
  if (active) {
#pragma unroll
    for (int c = 0; c < M; ++c) w[node * M + c] = f[node * M + c] - acc[c];
  }
}

// The subtrees of the pairs (e0, e1) of points of the two outermost
// dimensions that wavefront s of k_surplus_split walks: o[e0 * 17 + e1] == s
// (-1: no such pair).  Made on the host by a longest-first assignment.
struct SplitOwners {
  int8_t o[17 * 17];
};

// k_surplus_fast with the walk of each group of 64 nodes split over S
// wavefronts of one workgroup: wavefront s sums the subtrees of the pairs
// (e0, e1) it owns, and the S partial sums are added in wavefront order.  At
// the levels where a build launch holds a few dozen wavefronts on the whole
// device, this divides the length of its serial walk (the largest subtree,
// that of e0 = e1 = 0, is about a third of the walk at level 3).
template <int D, int L, int M, int S>
__global__ __launch_bounds__(64 * S) void k_surplus_split(GridArgs g, const double* __restrict__ wsub, int64_t n,
                                                          const int32_t* __restrict__ nodes,
                                                          const double* __restrict__ node_xi,
                                                          const double* __restrict__ f, double* __restrict__ w,
                                                          SplitOwners own) {
  static_assert(D == 6 && L >= 1 && L <= 4, "the split build covers d = 6, levels 1..4");
  constexpr int P = upto(L), KU = 4, KO = D - KU;
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t q = (int64_t)blockIdx.x * 64 + lane;
  const bool active = q < n;
  const int64_t node = active ? nodes[q] : 0;
  double* lds_lane = lds + wave * (KO * P * 64) + lane;
  double bv[KU][P];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double xi = active ? node_xi[node * D + k] : 0.5;
    double row[kMaxPoints];
    basis_row_l<L, double>(g, xi, row);
    if (k < KO) {
#pragma unroll
      for (int e = 0; e < P; ++e) lds_lane[(k * P + e) * 64] = row[e];
    } else {
#pragma unroll
      for (int e = 0; e < P; ++e) bv[k - KO][e] = row[e];
    }
  }
  double acc[M];
#pragma unroll
  for (int c = 0; c < M; ++c) acc[c] = 0.0;
  const int32_t* off0 = g.off + ((D - 1) * (L + 1) + L) * P;
  for (int e0 = 0; e0 < P; ++e0) {
    const int b1 = L - g.excess[e0];
    const int64_t base0 = off0[e0];
    const double p0 = lds_lane[e0 * 64];
    const int32_t* off1 = g.off + ((D - 2) * (L + 1) + b1) * P;
    const int c1 = upto(b1);
    for (int e1 = 0; e1 < c1; ++e1) {
      if (own.o[e0 * 17 + e1] != wave) continue;
      const double p1 = p0 * lds_lane[(P + e1) * 64];
      uwalk_budget<KU, P, M, L, double>(b1 - g.excess[e1], bv, wsub + (base0 + off1[e1]) * M, p1, acc);
    }
  }
  double* part = lds + S * KO * P * 64;  // S x 64 x M partial sums
#pragma unroll
  for (int c = 0; c < M; ++c) part[(wave * 64 + lane) * M + c] = acc[c];
  __syncthreads();
  if (wave == 0 && active) {
#pragma unroll
    for (int c = 0; c < M; ++c) {
      double t = part[lane * M + c];
#pragma unroll
      for (int r = 1; r < S; ++r) t += part[(r * 64 + lane) * M + c];
      w[node * M + c] = f[node * M + c] - t;
    }
  }
}

// ---- host side -------------------------------------------------------------

void release(GridDevice& gd) {
  (void)hipFree(gd.node_xi);
  (void)hipFree(gd.by_level);
  (void)hipFree(gd.tables);
  (void)hipFree(gd.dtab);
  (void)hipFree(gd.sub_map);
  (void)hipFree(gd.scratch);
  gd.node_xi = gd.dtab = gd.scratch = nullptr;
  gd.by_level = gd.tables = gd.sub_map = nullptr;
  gd.ready.store(false);
}

// Whether the tables of G and of its lower-level grids are on device dev.
bool tables_ready(const Grid& G, int dev) {
  if (!G.dev[dev].ready.load(std::memory_order_acquire)) return false;
  for (const auto& sg : G.sub)
    if (!tables_ready(*sg, dev)) return false;
  return true;
}

GridArgs make_args(const Grid& G, const GridDevice& gd) {
  GridArgs a;
  a.d = G.d;
  a.L = G.level;
  a.P = G.P;
  a.excess = gd.tables;
  a.off = gd.tables + G.itab_off;
  a.X = gd.dtab;
  a.scale = gd.dtab + G.P;
  for (int k = 0; k < kMaxDim; ++k) {
    a.lo[k] = k < G.d ? G.lo[k] : 0.0;
    a.inv_width[k] = k < G.d ? G.inv_width[k] : 0.0;
  }
  return a;
}

size_t lds_bytes(const Grid& G) { return (size_t)(G.d - 1) * G.P * 64 * sizeof(double); }

// The blocks of the points e0 of dimension 0 for the kGenWaves wavefronts of
// a split walk of budget bE in d dimensions (packed as gen_lo / gen_hi read
// them): contiguous, the largest block's subtree nodes as few as possible
// (the first such partition found), trailing blocks empty when there are
// fewer points than wavefronts.
uint32_t gen_bounds(int d, int bE) {
  const int n = upto(bE < 0 ? 0 : bE);
  std::vector<int64_t> pre(n + 1, 0);
  for (int e = 0; e < n; ++e) pre[e + 1] = pre[e] + subgrid(d - 1, bE - excess_of(e));
  const int S = kGenWaves;
  // best[k][i]: smallest largest block of points i..n-1 in k non-empty blocks
  const int64_t inf = INT64_MAX;
  std::vector<std::vector<int64_t>> best(S + 1, std::vector<int64_t>(n + 1, inf));
  std::vector<std::vector<int>> cut(S + 1, std::vector<int>(n + 1, n));
  for (int i = 0; i < n; ++i) best[1][i] = pre[n] - pre[i];
  for (int k = 2; k <= S; ++k)
    for (int i = 0; i + k <= n; ++i)
      for (int j = i + 1; j + k - 1 <= n; ++j) {
        const int64_t v = std::max(pre[j] - pre[i], best[k - 1][j]);
        if (v < best[k][i]) {
          best[k][i] = v;
          cut[k][i] = j;
        }
      }
  int kb = 1;
  for (int k = 2; k <= S && k <= n; ++k)
    if (best[k][0] < best[kb][0]) kb = k;
  uint32_t packed = 0;
  int i = 0;
  for (int s = 0; s < S - 1; ++s) {
    const int k = kb - s;  // blocks left, this one included
    const int end = k >= 2 ? cut[k][i] : n;
    packed |= (uint32_t)(s < kb ? end : n) << (8 * s);
    if (s < kb) i = end;
  }
  return packed | (0xffu << (8 * (S - 1)));
}

template <int D, int MC>
hipError_t launch_eval(const GridArgs& a, size_t lds, const double* w, int m, int col0, int64_t nq,
                       const double* xq, double* uq, hipStream_t s) {
  if constexpr (D >= 2) {
    auto kern = k_eval_gs<D, MC>;
    const size_t lds_s = lds + (size_t)kGenWaves * 64 * MC * sizeof(double);
    if (lds_s > 65536) {
      hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds_s);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)((nq + 63) / 64)), dim3(64 * kGenWaves), lds_s, s, a, w, m, col0, nq,
                       xq, uq, gen_bounds(D, a.L));
    return hipGetLastError();
  }
  auto kern = k_eval<D, MC>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  const int64_t blocks = (nq + 63) / 64;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64), lds, s, a, w, m, col0, nq, xq, uq);
  return hipGetLastError();
}

template <int D, int MC>
hipError_t launch_level(const GridArgs& a, size_t lds, const double* f, double* w, int m, int col0,
                        int lv, const int32_t* nodes, int64_t count, const double* node_xi,
                        hipStream_t s) {
  if constexpr (D >= 2) {
    auto kern = k_surplus_level_gs<D, MC>;
    const size_t lds_s = lds + (size_t)kGenWaves * 64 * MC * sizeof(double);
    if (lds_s > 65536) {
      hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds_s);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)((count + 63) / 64)), dim3(64 * kGenWaves), lds_s, s, a, f, w, m,
                       col0, lv, nodes, count, node_xi, gen_bounds(D, lv - 1));
    return hipGetLastError();
  }
  auto kern = k_surplus_level<D, MC>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  const int64_t blocks = (count + 63) / 64;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64), lds, s, a, f, w, m, col0, lv, nodes,
                     count, node_xi);
  return hipGetLastError();
}

template <int D>
hipError_t dispatch_mc_eval(int mc, const GridArgs& a, size_t lds, const double* w, int m, int col0,
                            int64_t nq, const double* xq, double* uq, hipStream_t s) {
  switch (mc) {
    case 1: return launch_eval<D, 1>(a, lds, w, m, col0, nq, xq, uq, s);
    case 2: return launch_eval<D, 2>(a, lds, w, m, col0, nq, xq, uq, s);
    default: return launch_eval<D, 3>(a, lds, w, m, col0, nq, xq, uq, s);
  }
}

template <int D>
hipError_t dispatch_mc_level(int mc, const GridArgs& a, size_t lds, const double* f, double* w, int m,
                             int col0, int lv, const int32_t* nodes, int64_t count,
                             const double* node_xi, hipStream_t s) {
  switch (mc) {
    case 1: return launch_level<D, 1>(a, lds, f, w, m, col0, lv, nodes, count, node_xi, s);
    case 2: return launch_level<D, 2>(a, lds, f, w, m, col0, lv, nodes, count, node_xi, s);
    default: return launch_level<D, 3>(a, lds, f, w, m, col0, lv, nodes, count, node_xi, s);
  }
}

#define SGCM_DIM_SWITCH(d, CALL) \
  switch (d) {                   \
    case 1: return CALL(1);      \
    case 2: return CALL(2);      \
    case 3: return CALL(3);      \
    case 4: return CALL(4);      \
    case 5: return CALL(5);      \
    case 6: return CALL(6);      \
    case 7: return CALL(7);      \
    default: return CALL(8);     \
  }

hipError_t eval_chunk(int d, int mc, const GridArgs& a, size_t lds, const double* w, int m, int col0,
                      int64_t nq, const double* xq, double* uq, hipStream_t s) {
#define CALL_EVAL(D) dispatch_mc_eval<D>(mc, a, lds, w, m, col0, nq, xq, uq, s)
  SGCM_DIM_SWITCH(d, CALL_EVAL)
#undef CALL_EVAL
}

hipError_t level_chunk(int d, int mc, const GridArgs& a, size_t lds, const double* f, double* w, int m,
                       int col0, int lv, const int32_t* nodes, int64_t count, const double* node_xi,
                       hipStream_t s) {
#define CALL_LEVEL(D) dispatch_mc_level<D>(mc, a, lds, f, w, m, col0, lv, nodes, count, node_xi, s)
  SGCM_DIM_SWITCH(d, CALL_LEVEL)
#undef CALL_LEVEL
}

template <int L, int M, typename F>
hipError_t launch_fast(const GridArgs& a, int64_t nq, const F* w, const F* xq, F* uq, hipStream_t s) {
  constexpr int D = 6;
  // the outer dimensions' basis values; with LOW0, dimension 0's of the
  // finest level only (see owalk)
  const size_t lds = (eval_low0<L, F>() ? (size_t)((D - 5) * upto(L) + upto(L) - upto(L - 1))
                                        : (size_t)(D - 4) * upto(L)) * 64 * sizeof(F);
  const int64_t blocks = (nq + 63) / 64;
  if constexpr (eval_fine<L, F>()) {
    const size_t lds_f = (size_t)(D - 5) * upto(L - 1) * 64 * sizeof(F);  // see owalk_f
    hipLaunchKernelGGL((k_eval_fine<D, L, M, F>), dim3((unsigned)blocks), dim3(64), lds_f, s, a, w, nq, xq, uq);
  } else {
    hipLaunchKernelGGL((k_eval_fast<D, L, M, F>), dim3((unsigned)blocks), dim3(64), lds, s, a, w, nq, xq, uq);
  }
  return hipGetLastError();
}

template <int L, typename F>
hipError_t fast_m(int m, const GridArgs& a, int64_t nq, const F* w, const F* xq, F* uq, hipStream_t s) {
  switch (m) {
    case 1: return launch_fast<L, 1, F>(a, nq, w, xq, uq, s);
    case 2: return launch_fast<L, 2, F>(a, nq, w, xq, uq, s);
    default: return launch_fast<L, 3, F>(a, nq, w, xq, uq, s);
  }
}

// The unrolled kernel covers d = 6, levels 1..5, m <= 3 (the rigid-body feedback).
bool fast_eval_applies(const Grid& G, int m) { return G.d == 6 && G.level >= 1 && G.level <= 5 && m <= 3; }

template <typename F>
hipError_t eval_fast(const Grid& G, int m, const GridArgs& a, int64_t nq, const F* w, const F* xq, F* uq,
                     hipStream_t s) {
  switch (G.level) {
    case 1: return fast_m<1, F>(m, a, nq, w, xq, uq, s);
    case 2: return fast_m<2, F>(m, a, nq, w, xq, uq, s);
    case 3: return fast_m<3, F>(m, a, nq, w, xq, uq, s);
    case 4: return fast_m<4, F>(m, a, nq, w, xq, uq, s);
    default: return fast_m<5, F>(m, a, nq, w, xq, uq, s);
  }
}

template <int L, int M>
hipError_t launch_surplus_fast(const GridArgs& a, const double* wsub, int64_t n, const int32_t* nodes,
                               const double* node_xi, const double* f, double* w, hipStream_t s) {
  constexpr int D = 6;
  const size_t lds = (size_t)(D - 4) * upto(L) * 64 * sizeof(double);
  const int64_t blocks = (n + 63) / 64;
  hipLaunchKernelGGL((k_surplus_fast<D, L, M>), dim3((unsigned)blocks), dim3(64), lds, s, a, wsub, n, nodes,
                     node_xi, f, w);
  return hipGetLastError();
}

constexpr int kSplitWaves = 4;  // wavefronts per group of 64 nodes in k_surplus_split

// The owners of the (e0, e1) subtrees of a level-L grid (d = 6) among S
// wavefronts: longest first (the inner nodes below the pair), each to the
// least loaded wavefront (ties: the lower index, then the canonical order).
SplitOwners split_owners(int L, int S) {
  SplitOwners r;
  for (int i = 0; i < 17 * 17; ++i) r.o[i] = -1;
  struct Item {
    int size, e0, e1;
  };
  std::vector<Item> items;
  for (int e0 = 0; e0 < upto(L); ++e0)
    for (int e1 = 0; e1 < upto(L - excess_of(e0)); ++e1)
      items.push_back({subgrid(4, L - excess_of(e0) - excess_of(e1)), e0, e1});
  std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.size > b.size; });
  std::vector<int> load(S, 0);
  for (const Item& it : items) {
    int best = 0;
    for (int k = 1; k < S; ++k)
      if (load[k] < load[best]) best = k;
    load[best] += it.size;
    r.o[it.e0 * 17 + it.e1] = (int8_t)best;
  }
  return r;
}

template <int L, int M>
hipError_t launch_surplus_split(const GridArgs& a, const double* wsub, int64_t n, const int32_t* nodes,
                                const double* node_xi, const double* f, double* w, hipStream_t s) {
  constexpr int D = 6, S = kSplitWaves;
  static const SplitOwners own = split_owners(L, S);
  const size_t lds = ((size_t)S * (D - 4) * upto(L) * 64 + (size_t)S * 64 * M) * sizeof(double);
  const int64_t blocks = (n + 63) / 64;
  hipLaunchKernelGGL((k_surplus_split<D, L, M, S>), dim3((unsigned)blocks), dim3(64 * S), lds, s, a, wsub, n,
                     nodes, node_xi, f, w, own);
  return hipGetLastError();
}

// Level 1 (13 nodes walked per node) keeps the one-wavefront kernel.
template <int L>
hipError_t surplus_fast_m(int m, const GridArgs& a, const double* wsub, int64_t n, const int32_t* nodes,
                          const double* node_xi, const double* f, double* w, hipStream_t s) {
  if constexpr (L >= 2) {
    switch (m) {
      case 1: return launch_surplus_split<L, 1>(a, wsub, n, nodes, node_xi, f, w, s);
      case 2: return launch_surplus_split<L, 2>(a, wsub, n, nodes, node_xi, f, w, s);
      default: return launch_surplus_split<L, 3>(a, wsub, n, nodes, node_xi, f, w, s);
    }
  } else {
    switch (m) {
      case 1: return launch_surplus_fast<L, 1>(a, wsub, n, nodes, node_xi, f, w, s);
      case 2: return launch_surplus_fast<L, 2>(a, wsub, n, nodes, node_xi, f, w, s);
      default: return launch_surplus_fast<L, 3>(a, wsub, n, nodes, node_xi, f, w, s);
    }
  }
}

// The unrolled build covers d = 6, levels 0..5, m <= 3 (the lower-level grids
// it evaluates have levels 1..4).
bool fast_build_applies(const Grid& G, int m) {
  return G.d == 6 && G.level <= 5 && m <= 3 && (int)G.sub.size() == G.level;
}

hipError_t build_fast(Grid& G, int dev, int m, const double* f, double* w, hipStream_t s) {
  const GridDevice& gd = G.dev[dev];
  const int64_t n01 = G.level >= 1 ? G.level_start[2] : 1;
  hipLaunchKernelGGL(k_surplus_low, dim3((unsigned)((n01 * m + 63) / 64)), dim3(64), 0, s, gd.by_level, n01, m, f,
                     w);
  hipError_t e = hipGetLastError();
  for (int lv = 2; lv <= G.level && e == hipSuccess; ++lv) {
    const Grid& S = *G.sub[lv - 1];
    const int64_t ms = S.M, start = G.level_start[lv], count = G.level_start[lv + 1] - start;
    const int32_t* map = gd.sub_map + G.sub_map_off[lv - 1];
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((ms * m + 255) / 256)), dim3(256), 0, s, map, ms, m, w,
                       gd.scratch);
    e = hipGetLastError();
    if (e != hipSuccess || count == 0) continue;
    const GridArgs sa = make_args(S, S.dev[dev]);
    const int32_t* nodes = gd.by_level + start;
    switch (lv - 1) {
      case 1: e = surplus_fast_m<1>(m, sa, gd.scratch, count, nodes, gd.node_xi, f, w, s); break;
      case 2: e = surplus_fast_m<2>(m, sa, gd.scratch, count, nodes, gd.node_xi, f, w, s); break;
      case 3: e = surplus_fast_m<3>(m, sa, gd.scratch, count, nodes, gd.node_xi, f, w, s); break;
      default: e = surplus_fast_m<4>(m, sa, gd.scratch, count, nodes, gd.node_xi, f, w, s); break;
    }
  }
  return e;
}

int current_device(int* dev) {
  if (hipGetDevice(dev) != hipSuccess) return SGCM_EDEVICE;
  if (*dev < 0 || *dev >= kMaxDevices) return SGCM_EUNSUPPORTED;
  return SGCM_OK;
}

}  // namespace

void free_device_tables(Grid& G) {
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) cur = -1;
  for (int dv = 0; dv < kMaxDevices; ++dv) {
    GridDevice& gd = G.dev[dv];
    if (!gd.ready.load()) continue;
    if (hipSetDevice(dv) == hipSuccess) release(gd);
    gd.ready.store(false);
  }
  if (cur >= 0) (void)hipSetDevice(cur);
  for (auto& sg : G.sub) free_device_tables(*sg);
}

int upload_device_tables(Grid& G, int dev, void* stream) {
  for (auto& sg : G.sub) {
    const int rc = upload_device_tables(*sg, dev, stream);
    if (rc != SGCM_OK) return rc;
  }
  std::lock_guard<std::mutex> lock(G.mu);
  GridDevice& gd = G.dev[dev];
  if (gd.ready.load()) return SGCM_OK;
  hipStream_t s = (hipStream_t)stream;
  bool dev_err = false;
  // the host tables belong to the grid and outlive the asynchronous copies
  auto up = [&](void** dst, const void* src, size_t bytes) -> bool {
    if (bytes == 0) bytes = 8;
    if (hipMalloc(dst, bytes) != hipSuccess) return false;
    if (src != nullptr && hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, s) != hipSuccess) {
      dev_err = true;
      return false;
    }
    return true;
  };
  const bool ok = up((void**)&gd.node_xi, G.xi.data(), G.xi.size() * sizeof(double)) &&
                  up((void**)&gd.by_level, G.by_level.data(), G.by_level.size() * sizeof(int32_t)) &&
                  up((void**)&gd.tables, G.itab.data(), G.itab.size() * sizeof(int32_t)) &&
                  up((void**)&gd.dtab, G.dtab.data(), G.dtab.size() * sizeof(double)) &&
                  up((void**)&gd.sub_map, G.sub_map.data(), G.sub_map.size() * sizeof(int32_t)) &&
                  up((void**)&gd.scratch, nullptr, (size_t)G.M * 3 * sizeof(double));
  if (!ok) {
    (void)hipGetLastError();
    if (dev_err) (void)hipStreamSynchronize(s);  // no copy may still read a freed table
    release(gd);
    return dev_err ? SGCM_EDEVICE : SGCM_ENOMEM;
  }
  gd.ready.store(true, std::memory_order_release);
  return SGCM_OK;
}

}  // namespace sgcm

using namespace sgcm;

extern "C" int sgcm_build_interpolant(const sgcm_grid* gh, int32_t m, const double* values,
                                      double* surplus, void* stream) {
  sgcm::CallRange range("sgcm_build_interpolant");
  if (!gh || m < 1 || m > 64 || !values || !surplus || values == surplus) return SGCM_EINVAL;
  Grid& G = const_cast<Grid&>(gh->g);
  int dev = 0;
  int rc = current_device(&dev);
  if (rc != SGCM_OK) return rc;
  if (!tables_ready(G, dev)) return SGCM_EINVAL;  // sgcm_grid_upload first
  const GridDevice& gd = G.dev[dev];
  hipStream_t s = (hipStream_t)stream;
  if (fast_build_applies(G, m)) return build_fast(G, dev, m, values, surplus, s) == hipSuccess ? SGCM_OK : SGCM_EDEVICE;
  GridArgs a = make_args(G, gd);
  const size_t lds = lds_bytes(G);
  for (int lv = 0; lv <= G.level; ++lv) {
    const int64_t start = G.level_start[lv], count = G.level_start[lv + 1] - start;
    if (count == 0) continue;
    for (int col0 = 0; col0 < m; col0 += 3) {
      const int mc = (m - col0) < 3 ? (m - col0) : 3;
      hipError_t e = level_chunk(G.d, mc, a, lds, values, surplus, m, col0, lv, gd.by_level + start,
                                 count, gd.node_xi, s);
      if (e != hipSuccess) return SGCM_EDEVICE;
    }
  }
  return SGCM_OK;
}

extern "C" int sgcm_eval_feedback(const sgcm_grid* gh, int32_t m, const double* surplus, int64_t n_q,
                                  const double* xq, double* uq, int32_t precision, void* stream) {
  sgcm::CallRange range("sgcm_eval_feedback");
  if (!gh || m < 1 || m > 64 || n_q < 0) return SGCM_EINVAL;
  if (precision != SGCM_FP64 && precision != SGCM_FP32) return SGCM_EINVAL;
  if (precision != SGCM_FP64) return SGCM_EUNSUPPORTED;
  if (n_q == 0) return SGCM_OK;
  if (!surplus || !xq || !uq) return SGCM_EINVAL;
  if ((n_q + 63) / 64 > 0x7fffffffLL) return SGCM_EUNSUPPORTED;
  Grid& G = const_cast<Grid&>(gh->g);
  int dev = 0;
  int rc = current_device(&dev);
  if (rc != SGCM_OK) return rc;
  if (!tables_ready(G, dev)) return SGCM_EINVAL;  // sgcm_grid_upload first
  GridArgs a = make_args(G, G.dev[dev]);
  const size_t lds = lds_bytes(G);
  hipStream_t s = (hipStream_t)stream;
  if (fast_eval_applies(G, m)) return eval_fast(G, m, a, n_q, surplus, xq, uq, s) == hipSuccess ? SGCM_OK : SGCM_EDEVICE;
  for (int col0 = 0; col0 < m; col0 += 3) {
    const int mc = (m - col0) < 3 ? (m - col0) : 3;
    if (eval_chunk(G.d, mc, a, lds, surplus, m, col0, n_q, xq, uq, s) != hipSuccess) return SGCM_EDEVICE;
  }
  return SGCM_OK;
}

extern "C" int sgcm_eval_feedback_f32(const sgcm_grid* gh, int32_t m, const float* surplus, int64_t n_q,
                                      const float* xq, float* uq, void* stream) {
  sgcm::CallRange range("sgcm_eval_feedback_f32");
  if (!gh || m < 1 || m > 64 || n_q < 0) return SGCM_EINVAL;
  if (n_q == 0) return SGCM_OK;
  if (!surplus || !xq || !uq) return SGCM_EINVAL;
  if ((n_q + 63) / 64 > 0x7fffffffLL) return SGCM_EUNSUPPORTED;
  Grid& G = const_cast<Grid&>(gh->g);
  if (!fast_eval_applies(G, m)) return SGCM_EUNSUPPORTED;
  int dev = 0;
  int rc = current_device(&dev);
  if (rc != SGCM_OK) return rc;
  if (!tables_ready(G, dev)) return SGCM_EINVAL;  // sgcm_grid_upload first
  GridArgs a = make_args(G, G.dev[dev]);
  return eval_fast<float>(G, m, a, n_q, surplus, xq, uq, (hipStream_t)stream) == hipSuccess ? SGCM_OK
                                                                                              : SGCM_EDEVICE;
}

extern "C" int sgcm_grid_upload(sgcm_grid* gh, void* stream) {
  sgcm::CallRange range("sgcm_grid_upload");
  if (!gh) return SGCM_EINVAL;
  int dev = 0;
  const int rc = current_device(&dev);
  if (rc != SGCM_OK) return rc;
  return upload_device_tables(gh->g, dev, stream);
}

// Example III of the paper (Sec. 5.3): three states, one control, and the
// time variable as a dimension of the sparse grid.
//
//   x1' = -x1 + x2,   x2' = -x2 + g,   x3' = (q + 2 x2 g) g + s u,
//   cost 0.5 * integral of (g^2 + u^2), no final cost,
// with s = 1 + x1^2 + x2^2, g = x3 / s, q = -2 x1^2 + 2 x1 x2 - 2 x2^2.
// The model is autonomous, so the value at (t, x) is that of the horizon
// T - t from x: the characteristic BVP of a grid node (t0, x0) runs over
// [t0, T] (eq. hamchar with x(t0) = x0, lambda(T) = 0), and V(t0, x0) and
// u*(t0, x0) = -s(x0) lambda3(t0) (eq. optuv) are the values the (t, x)
// interpolant is built from.
//
// The solver is the library's trapezoidal collocation with Newton's method
// and its rules (the first step from Y = 0 in full, then the damped steps
// with the sufficient-decrease test), in its own kernel: one wavefront per
// BVP, the residual and the Jacobian blocks lane-parallel over mesh points,
// and the linear solve a backward Riccati sweep over the intervals.  Each
// interval's equations, written as an affine map of (dx_{k-1}, dlambda_k) to
// (dx_k, dlambda_{k-1}), come from one 6 x 6 elimination (one matrix column
// per lane, four intervals at a time: they do not depend on the sweep); the
// 3 x 3 Riccati step dlambda_k = P_k dx_k + p_k then runs in every lane alike,
// and a forward pass recovers dx_k and dlambda_k.
#include <cmath>
#include <cstdint>

#include "model.h"
#include "sgcm_internal.h"
#include "trace.h"
#include "wave_la.h"

namespace sgcm {
namespace {

// Forward-mode dual number (value, one directional derivative).
struct Dual {
  double v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  const double r = a.v / b.v;
  return {r, (a.d - r * b.d) / b.v};
}

template <class T>
__device__ __forceinline__ T cst(double a) {
  if constexpr (sizeof(T) == sizeof(double)) {
    return a;
  } else {
    return T{a, 0.0};
  }
}

// Phi(y) = [dH/dlambda; -dH/dx] at u* = -s lambda3 (H = L + lambda^T f),
// y = (x1, x2, x3, lambda1, lambda2, lambda3).  By the envelope property
// (dH/du = 0 at u*), dH/dx at u* is the partial derivative at fixed u:
//   dH/dx_i = g g_i + l1 (d_i2 - d_i1) + l2 (g_i - d_i2) + l3 (phi_i + s_i u),
// phi = (q + 2 x2 g) g, g_i = dg/dx_i, s_i = ds/dx_i.
template <class T>
__device__ __forceinline__ void ex3_phi(const T* y, T* out) {
  const T x1 = y[0], x2 = y[1], x3 = y[2], l1 = y[3], l2 = y[4], l3 = y[5];
  const T s = cst<T>(1.0) + x1 * x1 + x2 * x2;
  const T g = x3 / s;
  const T q = cst<T>(-2.0) * x1 * x1 + cst<T>(2.0) * x1 * x2 - cst<T>(2.0) * x2 * x2;
  const T u = -(s * l3);
  const T w = q + cst<T>(2.0) * x2 * g;  // phi = w g
  out[0] = x2 - x1;
  out[1] = g - x2;
  out[2] = w * g + s * u;
  // partial derivatives of g, s, q
  const T g1 = cst<T>(-2.0) * x1 * g / s, g2 = cst<T>(-2.0) * x2 * g / s, g3 = cst<T>(1.0) / s;
  const T s1 = cst<T>(2.0) * x1, s2 = cst<T>(2.0) * x2;
  const T q1 = cst<T>(-4.0) * x1 + cst<T>(2.0) * x2, q2 = cst<T>(2.0) * x1 - cst<T>(4.0) * x2;
  // phi_i = w_i g + w g_i with w_i = q_i + 2 d_i2 g + 2 x2 g_i
  const T ph1 = (q1 + cst<T>(2.0) * x2 * g1) * g + w * g1;
  const T ph2 = (q2 + cst<T>(2.0) * g + cst<T>(2.0) * x2 * g2) * g + w * g2;
  const T ph3 = (cst<T>(2.0) * x2 * g3) * g + w * g3;
  const T H1 = g * g1 - l1 + l2 * g1 + l3 * (ph1 + s1 * u);
  const T H2 = g * g2 + l1 + l2 * (g2 - cst<T>(1.0)) + l3 * (ph2 + s2 * u);
  const T H3 = g * g3 + l2 * g3 + l3 * ph3;
  out[3] = -H1;
  out[4] = -H2;
  out[5] = -H3;
}

// Phi and its Jacobian (row-major, dJ[i * 6 + j] = dPhi_i / dy_j) at y: the
// columns by six forward-mode evaluations.
__device__ __forceinline__ void ex3_phi_jac(const double* y, double* phi, double* dJ) {
  ex3_phi<double>(y, phi);
#pragma unroll 1
  for (int j = 0; j < 6; ++j) {
    Dual yd[6], o[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) yd[i] = Dual{y[i], i == j ? 1.0 : 0.0};
    ex3_phi<Dual>(yd, o);
#pragma unroll
    for (int i = 0; i < 6; ++i) dJ[i * 6 + j] = o[i].d;
  }
}

// Running cost L at u*: 0.5 (g^2 + u^2).
__device__ __forceinline__ double ex3_running_cost(const double* y) {
  const double s = 1.0 + y[0] * y[0] + y[1] * y[1];
  const double g = y[2] / s, u = -(s * y[5]);
  return 0.5 * (g * g + u * u);
}

struct Ex3Args {
  int N, max_iter, max_halvings;
  int K;  // continuation stages in the initial state (0: none)
  double T, tol;
  int64_t per_bvp;  // doubles of workspace per BVP
  int tx;           // 1: the rows are (t0, x0) (4 values), 0: x0 only (t0 = 0)
};

// Workspace of one BVP, in doubles: Y, the trial point, the Newton step and
// the residual ((N + 1) x 6 each), Phi and its Jacobian at the mesh points
// ((N + 1) x 6 and (N + 1) x 36), and per interval a slot of 42 doubles (its
// 6 x 7 element, then its sweep values).
__host__ __device__ inline int64_t ex3_doubles(int N) {
  const int64_t NP = (int64_t)N + 1;
  const int64_t d = NP * 6 * 4 + NP * 6 + NP * 36 + (int64_t)N * 42;
  return (d + 31) / 32 * 32;
}

constexpr double kSigma = 1e-4;  // sufficient-decrease constant (as the main solver)

// Meshes of up to this many intervals keep the interval elements (and then
// the forward pass's values, in the same slots) in LDS: 42 N doubles, 21.5 KB
// at N = 64, so seven BVPs still share a compute unit; the serial Riccati and
// forward steps then wait on LDS instead of on the memory hierarchy.  Larger
// meshes keep them in the workspace.
constexpr int kEx3LdsMaxN = 64;

// Launches of up to this many BVPs run them in decreasing order of |x0|_1
// (k_ex3_order; the order, n int32, behind the BVP workspaces): a BVP from
// the zero state converges at once, so the nontrivial ones come first and
// take the first wavefront slots (on the level-5 grid in (t, x), 552 of 1105
// BVPs, against 1024 SIMDs), instead of sharing a SIMD with a neighbour in
// the grid's order.
constexpr int kEx3OrderMax = 8192;

size_t ex3_order_bytes(int64_t n) { return n <= kEx3OrderMax ? ((size_t)n * 4 + 255) / 256 * 256 : 0; }

// The launch order: a bucket sort of |x0|_1 (largest first; 256 buckets over
// [0, max]) in one workgroup.  rows: n rows of rs doubles, x0 from column c0.
__global__ __launch_bounds__(1024) void k_ex3_order(const double* __restrict__ rows, int rs, int c0, int n,
                                                    int32_t* __restrict__ order) {
  __shared__ float key[kEx3OrderMax];
  __shared__ float wmax[16];
  __shared__ int32_t cnt[256];
  const int t = threadIdx.x;
  float m = 0.0f;
  for (int i = t; i < n; i += 1024) {
    double a = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) a += fabs(rows[(int64_t)i * rs + c0 + j]);
    const float f = (float)a;
    key[i] = isfinite(f) ? f : 0.0f;
    m = fmaxf(m, key[i]);
  }
  if (t < 256) cnt[t] = 0;
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) m = fmaxf(m, __shfl_xor(m, d));
  if ((t & 63) == 0) wmax[t >> 6] = m;
  __syncthreads();
  float kmax = 0.0f;
#pragma unroll
  for (int w = 0; w < 16; ++w) kmax = fmaxf(kmax, wmax[w]);
  const float scale = kmax > 0.0f ? 255.5f / kmax : 0.0f;
  auto bucket = [&](int i) { return 255 - min(255, (int)(key[i] * scale)); };
  for (int i = t; i < n; i += 1024) atomicAdd(&cnt[bucket(i)], 1);
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int b = 0; b < 256; ++b) {
      const int c = cnt[b];
      cnt[b] = acc;
      acc += c;
    }
  }
  __syncthreads();
  for (int i = t; i < n; i += 1024) order[atomicAdd(&cnt[bucket(i)], 1)] = i;
}

// Residual F of point Z (N + 1 points of 6) into F; Phi at Z in PH (and the
// Jacobian blocks in DJ when jac); returns max|F|, or NaN when a value is not
// finite.  Lane-parallel over mesh points.
__device__ double ex3_residual(const Ex3Args& A, double alpha, const double* xbar, const double* Z, double* PH,
                               double* DJ, bool jac, double* F) {
  const int lane = threadIdx.x, NP = A.N + 1;
  for (int k = lane; k < NP; k += 64) {
    if (jac) ex3_phi_jac(Z + 6 * k, PH + 6 * k, DJ + 36 * k);
    else ex3_phi<double>(Z + 6 * k, PH + 6 * k);
  }
  wave_mem_sync();
  double m = 0.0;
  bool fin = true;
  for (int k = lane; k < NP; k += 64) {
    // F rows: x_0 - xbar (3), the N interval residuals (6 each), lambda_N (3)
    if (k == 0) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double f = Z[i] - xbar[i];
        F[i] = f;
        fin = fin && isfinite(f);
        m = fmax(m, fabs(f));
      }
    } else {
      const double* y0 = Z + 6 * (k - 1);
      const double* y1 = Z + 6 * k;
      const double* p0 = PH + 6 * (k - 1);
      const double* p1 = PH + 6 * k;
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const double f = y1[i] - y0[i] - alpha * (p0[i] + p1[i]);
        F[3 + 6 * (k - 1) + i] = f;
        fin = fin && isfinite(f);
        m = fmax(m, fabs(f));
      }
    }
    if (k == A.N) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double f = Z[6 * k + 3 + i];  // lambda_N - grad h = lambda_N
        F[3 + 6 * A.N + i] = f;
        fin = fin && isfinite(f);
        m = fmax(m, fabs(f));
      }
    }
  }
  wave_mem_sync();
  const bool all = __all(fin);
  m = wave_max(m);
  return all ? m : NAN;
}

// The Newton step d solving F'(Z) d = -F (F, PH, DJ at Z), by the backward
// Riccati sweep and the forward pass; false on a zero pivot.  Interval k's
// slot of 42 doubles (in LDS with LDSE, else at SWEg) holds its element until
// the sweep has used it, then the forward pass's values of the interval.
template <bool LDSE>
__device__ bool ex3_newton_step(const Ex3Args& A, double alpha, const double* DJ, const double* F, double* SWEg,
                                double* d) {
  extern __shared__ double ex3_lds[];
  double* const SWE = LDSE ? ex3_lds : SWEg;
  const int lane = threadIdx.x, N = A.N;
  bool regular = true;
  // The interval elements do not depend on the Riccati matrix: all of them
  // first, four intervals at a time (one per group of 16 lanes).  Interval
  // k's augmented matrix [Q | R_x | -L_lambda | -r], L = I - alpha J_k,
  // R = I + alpha J_{k-1}: column l in the group's lane l (l < 13).
  const int grp = lane >> 4, l0 = lane & 15;
  const int l = l0 < 13 ? l0 : 12;
  // every lane loads both Jacobians' column and selects (no divergent
  // branches, whose loads would each wait in turn): with c = l mod 6,
  // L_k[:, c] = e_c - alpha J_k[:, c] and R_k[:, c] = e_c + alpha J_{k-1}[:, c];
  // the next round's values are loaded while this round is eliminated
  const int c = l < 6 ? l : (l < 12 ? l - 6 : 0);
  auto fetch = [&](int kb, double (&j1)[6], double (&j0)[6], double (&fr)[6]) {
    const int k = kb + grp <= N ? kb + grp : N;  // groups past N repeat interval N
    const double* J1 = DJ + 36 * k;
    const double* J0 = DJ + 36 * (k - 1);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      j1[i] = J1[i * 6 + c];
      j0[i] = J0[i * 6 + c];
      fr[i] = F[3 + 6 * (k - 1) + i];
    }
  };
  double cj1[6], cj0[6], cfr[6];
  fetch(1, cj1, cj0, cfr);
  for (int kb = 1; kb <= N; kb += 4) {
    const int k = kb + grp <= N ? kb + grp : N;
    double nj1[6], nj0[6], nfr[6];
    if (kb + 4 <= N) fetch(kb + 4, nj1, nj0, nfr);
    double v[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const double e = i == c ? 1.0 : 0.0;
      const double lk = e - alpha * cj1[i];
      const double rk = e + alpha * cj0[i];
      const double fk = -cfr[i];
      v[i] = l < 3 ? lk : (l < 6 ? -rk : (l < 9 ? rk : (l < 12 ? -lk : fk)));
    }
    regular = gauss_jordan<6, 16>(v) && regular;
    // the element (6 x 7, row-major): the group's lanes 6..8 hold [A; C],
    // 9..11 [B; D], 12 [a; c]
    if (kb + grp <= N && l0 >= 6 && l0 < 13) {
      double* E = SWE + 42 * (int64_t)(k - 1);
#pragma unroll
      for (int i = 0; i < 6; ++i) E[i * 7 + (l0 - 6)] = v[i];
    }
    if (kb + 4 <= N) {
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        cj1[i] = nj1[i];
        cj0[i] = nj0[i];
        cfr[i] = nfr[i];
      }
    }
  }
  wave_mem_sync();
  regular = __all(regular);
  // P and p at the right end: dlambda_N = 0 dx_N - F_N
  double P[9], p[3];
#pragma unroll
  for (int e = 0; e < 9; ++e) P[e] = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) p[i] = -F[3 + 6 * N + i];
  for (int k = N; k >= 1; --k) {
    // element blocks, read where used: A, B (rows 0..2), C, D (rows 3..5),
    // a, c (column 6)
    double* E = SWE + 42 * (int64_t)(k - 1);
#define EA(i, j) E[(i) * 7 + (j)]
#define EB(i, j) E[(i) * 7 + 3 + (j)]
#define EC(i, j) E[(3 + (i)) * 7 + (j)]
#define ED(i, j) E[(3 + (i)) * 7 + 3 + (j)]
    // M = (I - B P)^{-1} by the adjugate
    double G[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double t = (i == j ? 1.0 : 0.0);
#pragma unroll
        for (int r = 0; r < 3; ++r) t = fma(-EB(i, r), P[r * 3 + j], t);
        G[i * 3 + j] = t;
      }
    double M[9];
    const double det = inv3(G, M);
    regular = regular && det != 0.0;
    // MA = M A, Mb = M (B p + a)
    double MA[9], bp[3], Mb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double t = E[i * 7 + 6];
#pragma unroll
      for (int r = 0; r < 3; ++r) t = fma(EB(i, r), p[r], t);
      bp[i] = t;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double t = 0.0;
#pragma unroll
      for (int r = 0; r < 3; ++r) t = fma(M[i * 3 + r], bp[r], t);
      Mb[i] = t;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double u = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) u = fma(M[i * 3 + r], EA(r, j), u);
        MA[i * 3 + j] = u;
      }
    }
    // P_{k-1} = C + D P MA,  p_{k-1} = D (P Mb + p) + c
    double DP[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double t = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) t = fma(ED(i, r), P[r * 3 + j], t);
        DP[i * 3 + j] = t;
      }
    double Pn[9], pn[3], PMb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double t = p[i];
#pragma unroll
      for (int r = 0; r < 3; ++r) t = fma(P[i * 3 + r], Mb[r], t);
      PMb[i] = t;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double t = E[(3 + i) * 7 + 6];
#pragma unroll
      for (int r = 0; r < 3; ++r) t = fma(ED(i, r), PMb[r], t);
      pn[i] = t;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double u = EC(i, j);
#pragma unroll
        for (int r = 0; r < 3; ++r) u = fma(DP[i * 3 + r], MA[r * 3 + j], u);
        Pn[i * 3 + j] = u;
      }
    }
    // the element is used: the slot takes the forward pass's values of
    // interval k (MA, Mb, P_k, p_k; the same in every lane)
    if (lane == 0) {
      double* sw = E;
#pragma unroll
      for (int e = 0; e < 9; ++e) {
        sw[e] = MA[e];
        sw[12 + e] = P[e];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        sw[9 + i] = Mb[i];
        sw[21 + i] = p[i];
      }
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) P[e] = Pn[e];
#pragma unroll
    for (int i = 0; i < 3; ++i) p[i] = pn[i];
#undef EA
#undef EB
#undef EC
#undef ED
  }
  wave_mem_sync();
  // forward: dx_0 = -F_0, dlambda_k = P_k dx_k + p_k, dx_k = MA_k dx_{k-1} + Mb_k
  double dx[3], dl[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) dx[i] = -F[i];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double t = p[i];
#pragma unroll
    for (int r = 0; r < 3; ++r) t = fma(P[i * 3 + r], dx[r], t);
    dl[i] = t;
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      d[i] = dx[i];
      d[3 + i] = dl[i];
    }
  }
  for (int k = 1; k <= N; ++k) {
    const double* sw = SWE + 42 * (int64_t)(k - 1);
    double nx[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double t = sw[9 + i];
#pragma unroll
      for (int r = 0; r < 3; ++r) t = fma(sw[i * 3 + r], dx[r], t);
      nx[i] = t;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      dx[i] = nx[i];
      double t = sw[21 + i];
#pragma unroll
      for (int r = 0; r < 3; ++r) t = fma(sw[12 + i * 3 + r], nx[r], t);
      dl[i] = t;
    }
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        d[6 * k + i] = dx[i];
        d[6 * k + 3 + i] = dl[i];
      }
    }
  }
  wave_mem_sync();
  return regular;
}

// Newton's iteration on the collocation equations from xbar: from Y = 0 with
// the first step in full (from_zero), else from Y with its test.  Returns the
// status and writes the iteration count.
template <bool LDSE>
__device__ int ex3_newton(const Ex3Args& A, double alpha, const double* xbar, bool from_zero, double* Y,
                          double* Yt, double* D, double* F, double* PH, double* DJ, double* SWE, int* iters) {
  const int lane = threadIdx.x, NP = A.N + 1;
  *iters = 0;
  if (from_zero) {
    for (int i = lane; i < 6 * NP; i += 64) Y[i] = 0.0;
    wave_mem_sync();
    (void)ex3_residual(A, alpha, xbar, Y, PH, DJ, true, F);
    if (!ex3_newton_step<LDSE>(A, alpha, DJ, F, SWE, D)) return SGCM_BVP_SINGULAR;
    for (int i = lane; i < 6 * NP; i += 64) Y[i] += D[i];
    wave_mem_sync();
  }
  for (int it = 0;; ++it) {
    *iters = it;
    const double fn = ex3_residual(A, alpha, xbar, Y, PH, DJ, false, F);
    if (isnan(fn)) return SGCM_BVP_NONFINITE;
    if (fn <= A.tol) return SGCM_BVP_CONVERGED;
    if (it == A.max_iter) return SGCM_BVP_MAXITER;
    (void)ex3_residual(A, alpha, xbar, Y, PH, DJ, true, F);
    if (!ex3_newton_step<LDSE>(A, alpha, DJ, F, SWE, D)) return SGCM_BVP_SINGULAR;
    double t = 1.0;
    for (int j = 0;; ++j) {
      for (int i = lane; i < 6 * NP; i += 64) Yt[i] = Y[i] + t * D[i];
      wave_mem_sync();
      if (j == A.max_halvings) break;  // the last trial is taken
      const double ft = ex3_residual(A, alpha, xbar, Yt, PH, DJ, false, F);
      if (!isnan(ft) && ft <= (1.0 - kSigma * t) * fn) break;
      t *= 0.5;
    }
    for (int i = lane; i < 6 * NP; i += 64) Y[i] = Yt[i];
    wave_mem_sync();
  }
}

// One BVP per 64-lane workgroup (BVP order[blockIdx.x], or blockIdx.x without
// an order); with LDSE, 42 N doubles of dynamic LDS (N <= kEx3LdsMaxN).
template <bool LDSE>
__global__ __launch_bounds__(64) void k_ex3_newton(Ex3Args A, const double* __restrict__ rows,
                                                   double* __restrict__ lam0, double* __restrict__ u0,
                                                   double* __restrict__ Vout, double* __restrict__ traj,
                                                   int32_t* __restrict__ status, int32_t* __restrict__ iters,
                                                   double* __restrict__ ws, const int32_t* __restrict__ order) {
  const int lane = threadIdx.x;
  const int64_t b = order ? order[blockIdx.x] : blockIdx.x;
  const int N = A.N, NP = N + 1;
  double* Y = ws + b * A.per_bvp;
  double* Yt = Y + 6 * (int64_t)NP;
  double* D = Yt + 6 * (int64_t)NP;
  double* F = D + 6 * (int64_t)NP;
  double* PH = F + 6 * (int64_t)NP;
  double* DJ = PH + 6 * (int64_t)NP;
  double* SWE = DJ + 36 * (int64_t)NP;
  const int rs = A.tx ? 4 : 3;
  const double t0 = A.tx ? rows[b * rs] : 0.0;
  double xbar[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) xbar[i] = rows[b * rs + (A.tx ? 1 : 0) + i];
  const double horizon = A.T - t0;
  int st = SGCM_BVP_MAXITER, it = 0;
  if (!(horizon >= 0.0) || !isfinite(horizon)) {
    st = SGCM_BVP_NONFINITE;  // a start time after T (or not finite)
    for (int i = lane; i < 6 * NP; i += 64) Y[i] = NAN;
    wave_mem_sync();
  } else {
    const double alpha = 0.5 * (horizon / N);
    // without continuation one stage from x0; with K stages, stage k from
    // (k / K) x0, the first from Y = 0 and each later one from the last
    const int stages = A.K > 0 ? A.K : 1;
    for (int k = 1; k <= stages; ++k) {
      double xk[3];
      const double sk = A.K > 0 ? (double)k / A.K : 1.0;
#pragma unroll
      for (int i = 0; i < 3; ++i) xk[i] = A.K > 0 ? sk * xbar[i] : xbar[i];
      int its = 0;
      st = ex3_newton<LDSE>(A, alpha, xk, k == 1, Y, Yt, D, F, PH, DJ, SWE, &its);
      it += its;
      if (st != SGCM_BVP_CONVERGED) break;
    }
  }
  // outputs: lambda(t0), u*(t0, x0), V by the trapezoidal rule, the mesh values
  if (lane == 0) {
    status[b] = st;
    iters[b] = it;
  }
  if (lane < 3) lam0[b * 3 + lane] = Y[3 + lane];
  if (lane == 0) {
    const double s = 1.0 + Y[0] * Y[0] + Y[1] * Y[1];
    u0[b] = -(s * Y[5]);
  }
  if (Vout) {
    const double alpha = 0.5 * ((A.T - t0) / N);
    double part = 0.0;
    for (int k = lane; k < NP; k += 64) {
      const double Lk = ex3_running_cost(Y + 6 * k);
      part += (k == 0 || k == N) ? Lk : 2.0 * Lk;
    }
    part = wave_sum(part);
    if (lane == 0) Vout[b] = alpha * part;
  }
  if (traj) {
    double* out = traj + b * 6 * (int64_t)NP;
    for (int i = lane; i < 6 * NP; i += 64) out[i] = Y[i];
  }
}

// Phi and its Jacobian at n points (one per thread).
__global__ __launch_bounds__(256) void k_ex3_rhs(int64_t n, const double* __restrict__ y, double* __restrict__ phi,
                                                 double* __restrict__ dphi) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double yy[6], ph[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) yy[e] = y[i * 6 + e];
  if (dphi) {
    ex3_phi_jac(yy, ph, dphi + i * 36);
  } else {
    ex3_phi<double>(yy, ph);
  }
#pragma unroll
  for (int e = 0; e < 6; ++e) phi[i * 6 + e] = ph[e];
}

int ex3_args(const sgcm_problem* p, Ex3Args* a) {
  if (!p || p->model != SGCM_MODEL_EXAMPLE3) return SGCM_EINVAL;
  if (p->n != 3 || p->m != 1) return SGCM_EINVAL;
  if (!(std::isfinite(p->T) && p->T > 0.0)) return SGCM_EINVAL;
  if (p->N < 1 || p->N > 65536) return SGCM_EINVAL;
  if (!(p->tol >= 0.0) || p->max_iter < 0 || p->max_iter > 1000) return SGCM_EINVAL;
  if (p->max_halvings < 0 || p->max_halvings > 60) return SGCM_EINVAL;
  if (p->precision != SGCM_FP64 && p->precision != SGCM_FP32) return SGCM_EINVAL;
  if (p->scheme != SGCM_TRAPEZOID && p->scheme != SGCM_LOBATTO4) return SGCM_EINVAL;
  if (p->precision != SGCM_FP64 || p->scheme != SGCM_TRAPEZOID) return SGCM_EUNSUPPORTED;
  a->N = p->N;
  a->max_iter = p->max_iter;
  a->max_halvings = p->max_halvings;
  a->T = p->T;
  a->tol = p->tol;
  if (p->continuation < 0 || p->continuation > 64) return SGCM_EINVAL;
  a->K = p->continuation;
  a->per_bvp = ex3_doubles(p->N);
  a->tx = 0;
  return SGCM_OK;
}

}  // namespace

int ex3_workspace(const sgcm_problem* p, int64_t n_bvps, size_t* bytes) {
  Ex3Args a;
  if (!bytes || n_bvps < 0) return SGCM_EINVAL;
  const int rc = ex3_args(p, &a);
  if (rc != SGCM_OK) return rc;
  *bytes = (size_t)a.per_bvp * sizeof(double) * (size_t)n_bvps + ex3_order_bytes(n_bvps);
  return SGCM_OK;
}

int ex3_solve(const sgcm_problem* p, int64_t n_bvps, const double* rows, int tx, double* lambda0, double* u0,
              double* V, double* traj, int32_t* status, int32_t* iters, void* workspace, size_t ws_bytes,
              void* stream) {
  Ex3Args a;
  if (n_bvps < 0) return SGCM_EINVAL;
  int rc = ex3_args(p, &a);
  if (rc != SGCM_OK) return rc;
  a.tx = tx;
  if (n_bvps == 0) return SGCM_OK;
  if (n_bvps > 0x7fffffffLL) return SGCM_EUNSUPPORTED;
  if (!rows || !lambda0 || !u0 || !status || !iters || !workspace) return SGCM_EINVAL;
  if (((uintptr_t)workspace & 255u) != 0) return SGCM_EINVAL;
  const size_t bvp_bytes = (size_t)a.per_bvp * sizeof(double) * (size_t)n_bvps;
  if (ws_bytes < bvp_bytes + ex3_order_bytes(n_bvps)) return SGCM_EINVAL;
  int32_t* order = nullptr;
  if (n_bvps <= kEx3OrderMax) {
    order = reinterpret_cast<int32_t*>(static_cast<char*>(workspace) + bvp_bytes);
    hipLaunchKernelGGL(k_ex3_order, dim3(1), dim3(1024), 0, (hipStream_t)stream, rows, tx ? 4 : 3, tx ? 1 : 0,
                       (int)n_bvps, order);
  }
  if (a.N <= kEx3LdsMaxN) {
    hipLaunchKernelGGL(k_ex3_newton<true>, dim3((unsigned)n_bvps), dim3(64), (size_t)42 * a.N * sizeof(double),
                       (hipStream_t)stream, a, rows, lambda0, u0, V, traj, status, iters, (double*)workspace, order);
  } else {
    hipLaunchKernelGGL(k_ex3_newton<false>, dim3((unsigned)n_bvps), dim3(64), 0, (hipStream_t)stream, a, rows,
                       lambda0, u0, V, traj, status, iters, (double*)workspace, order);
  }
  return hipGetLastError() == hipSuccess ? SGCM_OK : SGCM_EDEVICE;
}

int ex3_characteristic_rhs(const sgcm_problem* p, int64_t n_points, const double* y, double* phi, double* dphi,
                           void* stream) {
  Ex3Args a;
  if (n_points < 0) return SGCM_EINVAL;
  const int rc = ex3_args(p, &a);
  if (rc != SGCM_OK && rc != SGCM_EUNSUPPORTED) return rc;
  if (n_points == 0) return SGCM_OK;
  if (!y || !phi) return SGCM_EINVAL;
  const int64_t blocks = (n_points + 255) / 256;
  if (blocks > 0x7fffffffLL) return SGCM_EUNSUPPORTED;
  hipLaunchKernelGGL(k_ex3_rhs, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, n_points, y, phi, dphi);
  return hipGetLastError() == hipSuccess ? SGCM_OK : SGCM_EDEVICE;
}

}  // namespace sgcm

extern "C" int sgcm_solve_bvps_tx(const sgcm_problem* p, int64_t n_bvps, const double* tx, double* lambda0,
                                  double* u0, double* V, double* traj, int32_t* status, int32_t* iters,
                                  void* workspace, size_t ws_bytes, void* stream) {
  sgcm::CallRange range("sgcm_solve_bvps_tx");
  if (!p) return SGCM_EINVAL;
  if (p->model != SGCM_MODEL_EXAMPLE3) return SGCM_EUNSUPPORTED;
  return sgcm::ex3_solve(p, n_bvps, tx, 1, lambda0, u0, V, traj, status, iters, workspace, ws_bytes, stream);
}

// The first Newton step of the trapezoidal solve from Y = 0 for the six unit
// initial states, by doubling.
//
// At Y = 0 every interval of the trapezoidal collocation (Sec. 3.1) has the
// same equations: with G = Phi'(0) = [A, -S; W, -A^T] (the characteristic
// right-hand side of eq. hamchar linearised about the origin) and alpha = h/2,
//   (I - alpha G) y_k = (I + alpha G) y_{k-1},   k = 1..N,
// with x_0 = xbar and lambda_N = p_w x_N; the step d from Y = 0 solves these
// linear equations (the residual at Y = 0 is [-xbar; 0; 0]).  Written as a
// map of (x_{k-1}, lambda_k) to (x_k, lambda_{k-1}), one interval is the
// element
//   x_k = A0 x_{k-1} + B0 lambda_k,   lambda_{k-1} = C0 x_{k-1} + D0 lambda_k,
// and the element of two adjacent spans is the star product of theirs
// (eliminating the shared x and lambda); all spans of 2^b intervals share
// one element E_b, made by b doublings.  Then for every mesh point k, with
// the spans [k, N] and [0, k] written as sums of powers of two:
//   lambda_k = P_k x_k,  P_N = p_w I,  P at the left end of a span E with P_c
//   at its right end:  C + D P_c (I - B P_c)^{-1} A;
//   x_k = (I - B P_k)^{-1} A xbar  with (A, B) of the element of [0, k].
// This is the solution of the same linear equations (up to rounding) that
// each BVP's first sweep would compute, in about log2(N) dependent steps of
// 6 x 6 algebra instead of N.  The forms avoid powers of the interval map,
// whose growth over long horizons would ruin them.
//
// One workgroup of three wavefronts per mesh point: the first makes the
// elements E_b one level after the other, the second applies each level to
// P and the third to the element of [0, k] as soon as it is made.  In the
// 6 x 6 algebra a lane holds one column of a matrix: a product is a
// matrix-vector product per lane (the other matrix read from LDS), and the
// elimination broadcasts the pivot column from its lane (readlane), so no
// step waits on a barrier.
#include "model.h"
#include "wave_la.h"

namespace sgcm {
namespace {

constexpr int kEl = 4 * 36;     // doubles of one element: A, B, C, D (6 x 6 row-major each)
constexpr int kMaxLevels = 17;  // 2^16 intervals, the largest mesh

// Levels b of the elements E_b a mesh of N intervals needs (2^b <= N).
__host__ __device__ inline int first_step_levels(int N) {
  int l = 0;
  while (l < 31 && (1 << l) <= N) ++l;
  return l;
}

// E = E1 * E2, the element of span 1 followed by span 2 (E may be E1, not
// E2), by one wavefront: with Z = (I - B1 C2)^{-1},
//   A = A2 Z A1,  B = B2 + A2 Z B1 D2,  C = C1 + D1 C2 Z A1,
//   D = D1 (D2 + C2 Z B1 D2).
// Lanes 0..5 hold the columns of I - B1 C2, lanes 6..11 those of A1 (then
// of Z A1), lanes 12..17 those of B1 D2 (then of Z B1 D2).
__device__ __forceinline__ void star(const double* E1, const double* E2, double* E) {
  const double *A1 = E1, *B1 = E1 + 36, *C1 = E1 + 72, *D1 = E1 + 108;
  const double *A2 = E2, *B2 = E2 + 36, *C2 = E2 + 72, *D2 = E2 + 108;
  const int lane = threadIdx.x & 63;
  const int g = lane < 6 ? 0 : (lane < 12 ? 1 : 2);  // lanes from 18 on repeat group 2
  const int j = lane < 18 ? lane - 6 * g : 0;
  double v[6], t[6];
  if (g == 1) {
    load_col(A1, j, v);
  } else {
    load_col(g == 0 ? C2 : D2, j, t);
    matvec(B1, t, v);
    if (g == 0) {
#pragma unroll
      for (int i = 0; i < 6; ++i) v[i] = (i == j ? 1.0 : 0.0) - v[i];
    }
  }
  gauss_jordan<6>(v);
  if (lane >= 6 && lane < 18) {
    double a[6], c[6], d[6];
    matvec(A2, v, a);
    matvec(C2, v, c);
    if (g == 2) {
      double d2[6];
      load_col(D2, j, d2);
#pragma unroll
      for (int i = 0; i < 6; ++i) c[i] += d2[i];
    }
    matvec(D1, c, d);
    double o[6];
    load_col(g == 1 ? C1 : B2, j, o);
    if (g == 1) {
#pragma unroll
      for (int i = 0; i < 6; ++i) o[i] += d[i];
      store_col(E, j, a);       // A
      store_col(E + 72, j, o);  // C
    } else {
#pragma unroll
      for (int i = 0; i < 6; ++i) o[i] += a[i];
      store_col(E + 36, j, o);   // B
      store_col(E + 108, j, d);  // D
    }
  }
  wave_lds_sync();
}

// P <- C + D P (I - B P)^{-1} A, the Riccati matrix at the left end of the
// span of element E from P at its right end, by one wavefront; DP: LDS
// scratch of 36 doubles.  Lanes 0..5 hold the columns of I - B P, lanes 6..11
// those of A (then of X = (I - B P)^{-1} A), lanes 12..17 form D P.
__device__ __forceinline__ void terminal(const double* E, double* P, double* DP) {
  const double *A = E, *B = E + 36, *C = E + 72, *D = E + 108;
  const int lane = threadIdx.x & 63;
  const int g = lane < 6 ? 0 : (lane < 12 ? 1 : 2);
  const int j = lane < 18 ? lane - 6 * g : 0;
  double v[6], t[6];
  if (g == 1) {
    load_col(A, j, v);
  } else {
    load_col(P, j, t);
    matvec(g == 0 ? B : D, t, v);
    if (g == 0) {
#pragma unroll
      for (int i = 0; i < 6; ++i) v[i] = (i == j ? 1.0 : 0.0) - v[i];
    } else if (lane < 18) {
      store_col(DP, j, v);
    }
  }
  lds_handoff();
  gauss_jordan<6>(v);
  if (g == 1) {
    double o[6], c[6];
    matvec(DP, v, o);
    load_col(C, j, c);
#pragma unroll
    for (int i = 0; i < 6; ++i) c[i] += o[i];
    store_col(P, j, c);
  }
  wave_lds_sync();
}

// The element E_0 of one interval at Y = 0 into E, by one wavefront: from
// the interval equations, Q [x_k; lambda_{k-1}] = R [x_{k-1}; lambda_k] with
//   Q = [I - aA, aS; -aW, -(I - aA^T)],  R = [I + aA, -aS; aW, -(I + aA^T)],
// so [A0 B0; C0 D0] = Q^{-1} R.  Lane l < 24 holds column l of [Q | R].
__device__ __forceinline__ void interval_element(const BvpArgs& P, const double* GA, const double* GW, double* E) {
  const int lane = threadIdx.x & 63;
  const int c = lane < 24 ? lane : 0;
  const int cc = c < 12 ? c : c - 12;
  const bool cx = cc < 6;
  const int j = cx ? cc : cc - 6;
  const double sg = c < 12 ? -1.0 : 1.0;  // the sign of a in Q, R
  const double a = P.alpha;
  double v[12];
#pragma unroll
  for (int r = 0; r < 12; ++r) {
    const bool rx = r < 6;
    const int i = rx ? r : r - 6;
    const double id = i == j ? 1.0 : 0.0;
    double x;
    if (rx && cx) x = id + sg * a * GA[i * 6 + j];
    else if (rx) x = -sg * a * ((i >= 3 && j >= 3) ? P.Sw[(i - 3) * 3 + (j - 3)] : 0.0);
    else if (cx) x = sg * a * GW[i * 6 + j];
    else x = -(id + sg * a * GA[j * 6 + i]);
    v[r] = x;
  }
  gauss_jordan<12>(v);
  if (lane >= 12 && lane < 24) {
    const int q = lane - 12, jj = q < 6 ? q : q - 6;
    double* top = E + (q < 6 ? 0 : 36);    // A0 or B0
    double* bot = E + (q < 6 ? 72 : 108);  // C0 or D0
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      top[i * 6 + jj] = v[i];
      bot[i * 6 + jj] = v[6 + i];
    }
  }
  wave_lds_sync();
}

// Statuses and iteration counts of the six steps as a solve with
// max_iter = 0 reports them when they are finite.
__global__ void k_first_check(int32_t* __restrict__ chk) {
  const int t = threadIdx.x;
  if (t < 12) chk[t] = t < 6 ? SGCM_BVP_MAXITER : 0;
}

// Mesh point k = blockIdx.x of the six steps, y1[j][k] = [X_k e_j; P_k X_k
// e_j] (y1 is 6 x (N + 1) x 12); a non-finite value marks the steps invalid
// in chk.  Three wavefronts: the elements, the P chain, the [0, k] chain.
__global__ void __launch_bounds__(192) k_first_steps(const BvpArgs P, int N, int levels, double* __restrict__ y1,
                                                     int32_t* __restrict__ chk) {
  __shared__ double E[kMaxLevels * kEl];
  __shared__ double GA[36], GW[36], Pk[36], DP[36], El[kEl];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int k = blockIdx.x;
  const int L = N - k;
  if (t == 0) {
    double y[12] = {};
    double phi[12], A[36], W[36];
    point_eval(P, y, phi, A, W);
#pragma unroll
    for (int e = 0; e < 36; ++e) {
      GA[e] = A[e];
      GW[e] = W[e];
    }
  }
  if (wave == 1 && lane < 36) Pk[lane] = (lane / 6 == lane - 6 * (lane / 6)) ? P.pw : 0.0;
  __syncthreads();
  bool have = false;  // the [0, k] chain has an element
  for (int b = 0; b < levels; ++b) {
    if (wave == 0) {
      if (b == 0) interval_element(P, GA, GW, E);
      else star(E + (b - 1) * kEl, E + (b - 1) * kEl, E + b * kEl);
    }
    __syncthreads();  // E_b is made; the chains apply it while E_{b+1} is made
    if (wave == 1 && ((L >> b) & 1)) terminal(E + b * kEl, Pk, DP);
    if (wave == 2 && ((k >> b) & 1)) {
      if (!have) {
        for (int e = lane; e < kEl; e += 64) El[e] = E[b * kEl + e];
        wave_lds_sync();
      } else {
        star(El, E + b * kEl, El);
      }
      have = true;
    }
  }
  __syncthreads();
  if (wave != 1) return;
  // X = (I - B P)^{-1} A for the element (A, B) of [0, k] (the identity at
  // k = 0), then P X: lanes 0..5 hold the columns of I - B P, lanes 6..11
  // those of A (then of X).
  const int g = lane < 6 ? 0 : 1;
  const int j = lane < 12 ? lane - 6 * g : 0;
  double v[6];
  if (g == 0) {
    double pc[6];
    load_col(Pk, j, pc);
    if (k > 0) matvec(El + 36, pc, v);
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] = (i == j ? 1.0 : 0.0) - (k > 0 ? v[i] : 0.0);
  } else if (k > 0) {
    load_col(El, j, v);
  } else {
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] = i == j ? 1.0 : 0.0;
  }
  gauss_jordan<6>(v);
  bool fin = true;
  if (lane >= 6 && lane < 12) {
    double px[6];
    matvec(Pk, v, px);
    double* out = y1 + (int64_t)j * 12 * (N + 1) + (int64_t)k * 12;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      out[i] = v[i];
      out[6 + i] = px[i];
      fin = fin && isfinite(v[i]) && isfinite(px[i]);
    }
  }
  if (!__all(fin) && lane < 6) chk[lane] = SGCM_BVP_NONFINITE;
}

}  // namespace

int launch_first_steps(const BvpArgs& a, int N, double* y1, int32_t* chk, hipStream_t s) {
  const int levels = first_step_levels(N);
  if (N < 1 || levels > kMaxLevels) return SGCM_EINVAL;
  hipLaunchKernelGGL(k_first_check, dim3(1), dim3(64), 0, s, chk);
  hipLaunchKernelGGL(k_first_steps, dim3((unsigned)N + 1), dim3(192), 0, s, a, N, levels, y1, chk);
  return hipGetLastError() == hipSuccess ? SGCM_OK : SGCM_EDEVICE;
}

}  // namespace sgcm

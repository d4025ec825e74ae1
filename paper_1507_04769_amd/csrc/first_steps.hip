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
#include "model.h"

namespace sgcm {
namespace {

constexpr int kEl = 4 * 36;  // doubles of one element: A, B, C, D (6 x 6 row-major each)
constexpr int kMaxLevels = 17;  // 2^16 intervals, the largest mesh

// Levels b of the elements E_b a mesh of N intervals needs (2^b <= N).
__host__ __device__ inline int first_step_levels(int N) {
  int l = 0;
  while (l < 31 && (1 << l) <= N) ++l;
  return l;
}

// Entry t (row t / 6, column t % 6) of the product of two 6 x 6 matrices in
// LDS with row strides la and lb.
__device__ __forceinline__ double mm6(const double* A, int la, const double* B, int lb, int t) {
  const int i = t / 6, j = t - 6 * (t / 6);
  double s = A[i * la] * B[j];
#pragma unroll
  for (int l = 1; l < 6; ++l) s = fma(A[i * la + l], B[l * lb + j], s);
  return s;
}

// Gauss-Jordan elimination with partial pivoting of the n x w matrix M in
// LDS (row-major): afterwards its first n columns hold the identity and the
// other w - n columns the solution of M_left X = M_right.  A zero pivot
// leaves non-finite values.  Every thread of the (one-wave) workgroup takes
// part.
template <int n, int w>
__device__ void gauss_jordan(double* M) {
  constexpr int kPer = (n * w + 63) / 64;
  const int lane = threadIdx.x;
  for (int c = 0; c < n; ++c) {
    int p = c;
    double best = fabs(M[c * w + c]);
    for (int r = c + 1; r < n; ++r) {
      const double v = fabs(M[r * w + c]);
      if (v > best) {
        best = v;
        p = r;
      }
    }
    const double rp = 1.0 / M[p * w + c];
    double out[kPer];
#pragma unroll
    for (int s = 0; s < kPer; ++s) {
      const int e = lane + 64 * s;
      out[s] = 0.0;
      if (e < n * w) {
        const int i = e / w, j = e - w * (e / w);
        const double pr = M[p * w + j] * rp;  // row c after the swap, scaled
        const int src = i == p ? c : i;       // rows c and p trade places
        out[s] = i == c ? pr : fma(-M[src * w + c], pr, M[src * w + j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kPer; ++s) {
      const int e = lane + 64 * s;
      if (e < n * w) M[e] = out[s];
    }
    __syncthreads();
  }
}

// LDS scratch of the element algebra.
struct ElemScratch {
  double aug[6 * 18];  // augmented systems
  double s1[36], s2[36];
};

// E = E1 * E2, the element of span 1 followed by span 2 (E may be E1, not
// E2): with Z = (I - B1 C2)^{-1},
//   A = A2 Z A1,  B = B2 + A2 Z B1 D2,  C = C1 + D1 C2 Z A1,
//   D = D1 (D2 + C2 Z B1 D2).
__device__ void star(const double* E1, const double* E2, double* E, ElemScratch& w) {
  const double *A1 = E1, *B1 = E1 + 36, *C1 = E1 + 72, *D1 = E1 + 108;
  const double *A2 = E2, *B2 = E2 + 36, *C2 = E2 + 72, *D2 = E2 + 108;
  const int t = threadIdx.x;
  if (t < 36) {
    const int i = t / 6, j = t - 6 * (t / 6);
    const double bc = mm6(B1, 6, C2, 6, t), bd = mm6(B1, 6, D2, 6, t);
    w.aug[i * 18 + j] = (i == j ? 1.0 : 0.0) - bc;
    w.aug[i * 18 + 6 + j] = A1[t];
    w.aug[i * 18 + 12 + j] = bd;
  }
  __syncthreads();
  gauss_jordan<6, 18>(w.aug);  // columns 6..11: Z A1, 12..17: Z B1 D2
  double a2u = 0.0, a2v = 0.0, c2u = 0.0, c2v = 0.0;
  if (t < 36) {
    a2u = mm6(A2, 6, w.aug + 6, 18, t);
    a2v = mm6(A2, 6, w.aug + 12, 18, t);
    c2u = mm6(C2, 6, w.aug + 6, 18, t);
    c2v = mm6(C2, 6, w.aug + 12, 18, t);
  }
  __syncthreads();
  if (t < 36) {
    w.s1[t] = c2u;
    w.s2[t] = D2[t] + c2v;
    E[t] = a2u;
    E[36 + t] = B2[t] + a2v;
  }
  __syncthreads();
  double dc = 0.0, dd = 0.0;
  if (t < 36) {
    dc = mm6(D1, 6, w.s1, 6, t);
    dd = mm6(D1, 6, w.s2, 6, t);
  }
  __syncthreads();
  if (t < 36) {
    E[72 + t] = C1[t] + dc;
    E[108 + t] = dd;
  }
  __syncthreads();
}

// P <- C + D P (I - B P)^{-1} A: the Riccati matrix at the left end of the
// span of element E from P at its right end.
__device__ void terminal(const double* E, double* P, ElemScratch& w) {
  const double *A = E, *B = E + 36, *C = E + 72, *D = E + 108;
  const int t = threadIdx.x;
  if (t < 36) {
    const int i = t / 6, j = t - 6 * (t / 6);
    const double bp = mm6(B, 6, P, 6, t), dp = mm6(D, 6, P, 6, t);
    w.aug[i * 12 + j] = (i == j ? 1.0 : 0.0) - bp;
    w.aug[i * 12 + 6 + j] = A[t];
    w.s1[t] = dp;
  }
  __syncthreads();
  gauss_jordan<6, 12>(w.aug);
  if (t < 36) P[t] = C[t] + mm6(w.s1, 6, w.aug + 6, 12, t);
  __syncthreads();
}

// The elements E_b (b < levels) of problem P's trapezoidal intervals at
// Y = 0 into tab (levels x kEl doubles); chk (12) gets the statuses and
// iteration counts a solve with max_iter = 0 reports for the steps
// (SGCM_BVP_MAXITER, 0), or SGCM_BVP_NONFINITE if the table is not finite.
// One 64-thread workgroup.
__global__ void __launch_bounds__(64) k_first_table(const BvpArgs P, int levels, double* __restrict__ tab,
                                                     int32_t* __restrict__ chk) {
  __shared__ double aug[12 * 24];
  __shared__ double GA[36], GW[36];
  __shared__ double E[kMaxLevels * kEl];
  __shared__ ElemScratch w;
  const int t = threadIdx.x;
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
  __syncthreads();
  // [Q | R]: Q [x_k; lambda_{k-1}] = R [x_{k-1}; lambda_k], from the
  // interval equations, with
  //   Q = [I - aA, aS; -aW, -(I - aA^T)],  R = [I + aA, -aS; aW, -(I + aA^T)].
  const double a = P.alpha;
  for (int e = t; e < 12 * 24; e += 64) {
    const int r = e / 24, c = e - 24 * (e / 24);
    const int cc = c < 12 ? c : c - 12;
    const bool rx = r < 6, cx = cc < 6;
    const int i = rx ? r : r - 6, j = cx ? cc : cc - 6;
    const double id = i == j ? 1.0 : 0.0;
    const double sg = c < 12 ? -1.0 : 1.0;  // the sign of a in Q, R
    double v;
    if (rx && cx) v = id + sg * a * GA[i * 6 + j];
    else if (rx) v = -sg * a * ((i >= 3 && j >= 3) ? P.Sw[(i - 3) * 3 + (j - 3)] : 0.0);
    else if (cx) v = sg * a * GW[i * 6 + j];
    else v = -(id + sg * a * GA[j * 6 + i]);
    aug[e] = v;
  }
  __syncthreads();
  gauss_jordan<12, 24>(aug);
  for (int e = t; e < kEl; e += 64) {
    const int blk = e / 36, q = e - 36 * (e / 36);
    const int i = q / 6, j = q - 6 * (q / 6);
    const int r = (blk >= 2 ? 6 : 0) + i, c = 12 + (blk & 1 ? 6 : 0) + j;
    E[e] = aug[r * 24 + c];
  }
  __syncthreads();
  for (int b = 1; b < levels; ++b) star(E + (b - 1) * kEl, E + (b - 1) * kEl, E + b * kEl, w);
  bool fin = true;
  for (int e = t; e < levels * kEl; e += 64) {
    tab[e] = E[e];
    fin &= isfinite(E[e]);
  }
  const bool all = __syncthreads_and(fin);
  if (t < 12) chk[t] = t < 6 ? (all ? SGCM_BVP_MAXITER : SGCM_BVP_NONFINITE) : 0;
}

// Mesh point k = blockIdx.x of the six steps: y1[j][k] = [X_k e_j; P_k X_k
// e_j] (y1 is 6 x (N + 1) x 12); a non-finite value marks the steps invalid
// in chk.  One 64-thread workgroup per point.
__global__ void __launch_bounds__(64) k_first_points(int N, double pw, int levels, const double* __restrict__ tab,
                                                      double* __restrict__ y1, int32_t* __restrict__ chk) {
  __shared__ double E[kMaxLevels * kEl];
  __shared__ double Pk[36], El[kEl];
  __shared__ ElemScratch w;
  const int t = threadIdx.x;
  const int k = blockIdx.x;
  for (int e = t; e < levels * kEl; e += 64) E[e] = tab[e];
  if (t < 36) Pk[t] = (t / 6 == t - 6 * (t / 6)) ? pw : 0.0;
  __syncthreads();
  const int L = N - k;
  for (int b = 0; b < levels; ++b)
    if ((L >> b) & 1) terminal(E + b * kEl, Pk, w);
  // the element of [0, k]
  bool have = false;
  for (int b = 0; b < levels; ++b) {
    if (!((k >> b) & 1)) continue;
    if (!have) {
      for (int e = t; e < kEl; e += 64) El[e] = E[b * kEl + e];
      __syncthreads();
      have = true;
    } else {
      star(El, E + b * kEl, El, w);
    }
  }
  // X = (I - B P)^{-1} A (the identity at k = 0), then P X
  if (t < 36) {
    const int i = t / 6, j = t - 6 * (t / 6);
    const double id = i == j ? 1.0 : 0.0;
    w.aug[i * 12 + j] = have ? id - mm6(El + 36, 6, Pk, 6, t) : id;
    w.aug[i * 12 + 6 + j] = have ? El[t] : id;
  }
  __syncthreads();
  gauss_jordan<6, 12>(w.aug);
  double px = 0.0;
  if (t < 36) px = mm6(Pk, 6, w.aug + 6, 12, t);
  bool fin = true;
  if (t < 36) {
    const int i = t / 6, j = t - 6 * (t / 6);  // entry (i, j): component i of step j
    const double x = w.aug[i * 12 + 6 + j];
    const int64_t o = (int64_t)j * 12 * (N + 1) + (int64_t)k * 12;
    y1[o + i] = x;
    y1[o + 6 + i] = px;
    fin = isfinite(x) && isfinite(px);
  }
  const bool all = __syncthreads_and(fin);
  if (!all && t < 6) chk[t] = SGCM_BVP_NONFINITE;
}

}  // namespace

int64_t first_step_table_doubles(int N) { return (int64_t)first_step_levels(N) * kEl; }

int launch_first_steps(const BvpArgs& a, int N, double* table, double* y1, int32_t* chk, hipStream_t s) {
  const int levels = first_step_levels(N);
  if (N < 1 || levels > kMaxLevels) return SGCM_EINVAL;
  hipLaunchKernelGGL(k_first_table, dim3(1), dim3(64), 0, s, a, levels, table, chk);
  hipLaunchKernelGGL(k_first_points, dim3((unsigned)N + 1), dim3(64), 0, s, N, a.pw, levels, table, y1, chk);
  return hipGetLastError() == hipSuccess ? SGCM_OK : SGCM_EDEVICE;
}

}  // namespace sgcm

// Characteristic BVPs on gfx950 (Sec. 3.1, eq. hamchar and eq. optuv).
//
// One 64-lane workgroup (one wavefront) owns one BVP.  The discretisation is
// trapezoidal collocation on N uniform intervals; the unknowns are
// y_k = (x_k, lambda_k), k = 0..N, and the residual is
//   F = [ x_0 - xbar ; r_k = y_k - y_{k-1} - a (Phi_{k-1} + Phi_k), k=1..N ;
//         lambda_N - p_w x_N ],   a = h/2,
// with Phi = [ f(x, u*) ; -q_w x - A^T lambda ], A = df/dx, u* = argmin_u H.
// Newton's linear system is block bidiagonal:
//   (I - a Phi'_k) dy_k = (I + a Phi'_{k-1}) dy_{k-1} - r_k,
//   Phi' = [[A, -S], [W, -A^T]],  S = (1/r_w) Bt Bt^T,  W = -q_w I - sum_i lambda_i f_i''.
//
// Linear solve: a backward Riccati sweep dlambda_k = P_k dx_k + c_k from
// P_N = p_w I, c_N = -F_N.  The controls act on the body rates only, so S has
// rank <= 3 and lives in the rate block; eliminating dlambda_{k-1} with
// D^{-1} = (I - a A_{k-1}^T)^{-1} and dx_k with L_k = (I - a A_k)^{-1} leaves,
// on the serial path, one 3 x 3 system per interval (a Woodbury-type step):
//   EM1 = F P_k - H,  Psi = P_k + EM1,
//   Z3  = I + S_w Psi_w B_k,   [M | m] = Z3^{-1} S_w [Psi_w R_k - Gam_w | Psi_w rho + phi_w],
//   P_{k-1} = (EM1 R_k - Gam) - (EM1 B_k) M,   c_{k-1} = EM1 rho - (EM1 B_k) m + F c_k + D^{-1} r^l,
//   G_k = R_k - B_k M,  g_k = rho - B_k m   (dx_k = G_k dx_{k-1} + g_k),
// with F = D^{-1}(I + a A_k^T), H = a D^{-1} W_k, Gam = a D^{-1} W_{k-1},
// R_k = L_k (I + a A_{k-1}), B_k = a L_k[:, rates], rho = -L_k r^x,
// phi = (I + F) c_k + D^{-1} r^l.  D and I - a A_k are block triangular (the
// rates do not depend on the angles), so L_k comes from two 3 x 3 inverses and
// D^{-1} = L_{k-1}^T.
//
// Per-point blocks (A, W, L) are derived in batches of 8 points into an LDS
// ring ahead of the sweep (the trigonometric factors come from the residual
// pass); each interval is four LDS-synchronised stages (interval products,
// then three chain stages), each of which issues all of its LDS reads before
// its first product.  The interval solutions [G_k g_k ; P_{k-1} c_{k-1}] go
// to global memory and come back, staged through LDS 8 intervals at a time
// with a register prefetch, for the forward pass dx_0 = -F_0,
// dx_k = G_k dx_{k-1} + g_k, dlambda_{k-1} = P_{k-1} dx_{k-1} + c_{k-1}.
// Mesh-point work and the residual are lane-parallel over k.
#include <hip/hip_runtime.h>

#include <cstddef>

#include "sgcm_internal.h"

namespace sgcm {
namespace {

struct BvpArgs {
  int model, m, N, max_iter;
  double J[3];
  double a[3];   // gyroscopic coefficients: w_i' gets a_i w_j w_k
  double Sw[9];  // (1/r_w) J^{-1} B B^T J^{-1}, row-major 3 x 3
  double U[9];   // u* = U lambda_w, U[j][i] = -B[i][j] / (r_w J_i), row-major m x 3
  double q, r, pw, T, h, alpha, tol;
  int64_t per_bvp;  // doubles of workspace per BVP
};

// Phi, A = df/dx and W = -q I - Hessian_x(lambda^T f) at one mesh point.
__device__ __forceinline__ void point_eval(const BvpArgs& P, const double* __restrict__ y,
                                           double (&phi)[12], double (&A)[36], double (&W)[36],
                                           double* trig = nullptr) {
  const double w1 = y[3], w2 = y[4], w3 = y[5];
  const double l1 = y[6], l2 = y[7], l3 = y[8], l4 = y[9], l5 = y[10], l6 = y[11];
#pragma unroll
  for (int i = 0; i < 36; ++i) {
    A[i] = 0.0;
    W[i] = 0.0;
  }
  // J^{-1} B u* = -S_w lambda_w
  const double bu0 = -(P.Sw[0] * l4 + P.Sw[1] * l5 + P.Sw[2] * l6);
  const double bu1 = -(P.Sw[3] * l4 + P.Sw[4] * l5 + P.Sw[5] * l6);
  const double bu2 = -(P.Sw[6] * l4 + P.Sw[7] * l5 + P.Sw[8] * l6);
  double f[6];
  if (P.model == SGCM_MODEL_RIGID_BODY) {
    double s, c, st, ct;
    sincos(y[0], &s, &c);
    sincos(y[1], &st, &ct);
    const double k = 1.0 / ct, t = st * k;
    if (trig) {
      trig[0] = s;
      trig[1] = c;
      trig[2] = t;
      trig[3] = k;
    }
    const double al = s * w2 + c * w3;  // phi-rotated rates
    const double be = c * w2 - s * w3;  // d al / d phi
    f[0] = w1 + t * al;
    f[1] = be;
    f[2] = k * al;
    f[3] = P.a[0] * w2 * w3 + bu0;
    f[4] = P.a[1] * w3 * w1 + bu1;
    f[5] = P.a[2] * w1 * w2 + bu2;
    A[0 * 6 + 0] = t * be;
    A[0 * 6 + 1] = k * k * al;
    A[0 * 6 + 3] = 1.0;
    A[0 * 6 + 4] = t * s;
    A[0 * 6 + 5] = t * c;
    A[1 * 6 + 0] = -al;
    A[1 * 6 + 4] = c;
    A[1 * 6 + 5] = -s;
    A[2 * 6 + 0] = k * be;
    A[2 * 6 + 1] = k * t * al;
    A[2 * 6 + 4] = k * s;
    A[2 * 6 + 5] = k * c;
    A[3 * 6 + 4] = P.a[0] * w3;
    A[3 * 6 + 5] = P.a[0] * w2;
    A[4 * 6 + 3] = P.a[1] * w3;
    A[4 * 6 + 5] = P.a[1] * w1;
    A[5 * 6 + 3] = P.a[2] * w2;
    A[5 * 6 + 4] = P.a[2] * w1;
    // Hessian of g = lambda^T f = l1 w1 + Pc al + l2 be + (gyroscopic terms),
    // Pc = l1 t + l3 k depends on theta only.
    const double Pc = l1 * t + l3 * k;
    const double Pt = l1 * k * k + l3 * k * t;
    const double Ptt = 2.0 * l1 * k * k * t + l3 * k * (t * t + k * k);
    const double H00 = -Pc * al - l2 * be, H01 = Pt * be;
    const double H04 = Pc * c - l2 * s, H05 = -Pc * s - l2 * c;
    const double H11 = Ptt * al, H14 = Pt * s, H15 = Pt * c;
    const double H34 = l6 * P.a[2], H35 = l5 * P.a[1], H45 = l4 * P.a[0];
    W[0 * 6 + 0] = -H00;
    W[0 * 6 + 1] = W[1 * 6 + 0] = -H01;
    W[0 * 6 + 4] = W[4 * 6 + 0] = -H04;
    W[0 * 6 + 5] = W[5 * 6 + 0] = -H05;
    W[1 * 6 + 1] = -H11;
    W[1 * 6 + 4] = W[4 * 6 + 1] = -H14;
    W[1 * 6 + 5] = W[5 * 6 + 1] = -H15;
    W[3 * 6 + 4] = W[4 * 6 + 3] = -H34;
    W[3 * 6 + 5] = W[5 * 6 + 3] = -H35;
    W[4 * 6 + 5] = W[5 * 6 + 4] = -H45;
  } else {
    f[0] = w1;
    f[1] = w2;
    f[2] = w3;
    f[3] = bu0;
    f[4] = bu1;
    f[5] = bu2;
    A[0 * 6 + 3] = A[1 * 6 + 4] = A[2 * 6 + 5] = 1.0;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) W[i * 6 + i] -= P.q;
#pragma unroll
  for (int i = 0; i < 6; ++i) phi[i] = f[i];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double s = -P.q * y[j];
#pragma unroll
    for (int i = 0; i < 6; ++i) s -= A[i * 6 + j] * y[6 + i];
    phi[6 + j] = s;
  }
}

__device__ __forceinline__ double S_at(const BvpArgs& P, int r, int m) {
  return (r >= 3 && m >= 3) ? P.Sw[(r - 3) * 3 + (m - 3)] : 0.0;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Inverse of a 3 x 3 matrix (row-major) by the adjugate; returns the
// determinant (0 means singular; out is then not finite).
__device__ __forceinline__ double inv3(const double (&m)[9], double (&out)[9]) {
  const double c00 = m[4] * m[8] - m[5] * m[7];
  const double c01 = m[5] * m[6] - m[3] * m[8];
  const double c02 = m[3] * m[7] - m[4] * m[6];
  const double det = m[0] * c00 + m[1] * c01 + m[2] * c02;
  const double r = 1.0 / det;
  out[0] = c00 * r;
  out[1] = (m[2] * m[7] - m[1] * m[8]) * r;
  out[2] = (m[1] * m[5] - m[2] * m[4]) * r;
  out[3] = c01 * r;
  out[4] = (m[0] * m[8] - m[2] * m[6]) * r;
  out[5] = (m[2] * m[3] - m[0] * m[5]) * r;
  out[6] = c02 * r;
  out[7] = (m[1] * m[6] - m[0] * m[7]) * r;
  out[8] = (m[0] * m[4] - m[1] * m[3]) * r;
  return det;
}

// The Newton kernel runs one wavefront per workgroup.  LDS operations of a
// wavefront are executed in program order, so lanes exchange data through LDS
// with only a wait on the LDS counter and a compiler barrier (no s_barrier and,
// unlike a workgroup barrier with its release fence, no wait for outstanding
// global loads and stores: prefetches stay in flight).  Global-memory hand-offs
// between lanes (a few per Newton iteration) wait for the vector memory counter.
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void wave_mem_sync() { asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory"); }
// The lane id as a value the compiler cannot prove loop invariant: index
// arithmetic derived from it is then recomputed where it is used instead of
// being hoisted out of the Newton and sweep loops, where it would hold
// registers for the whole kernel.
__device__ __forceinline__ int opaque_lane(int lane) {
  asm volatile("" : "+v"(lane));
  return lane;
}

constexpr int kRing = 16;    // point slots in the LDS ring (power of two)
constexpr int kBatch = 8;    // points derived per refill
constexpr int kSlot = 120;   // per point: A (36), W (36), L (36), r_k (12)
constexpr int kChunk = 8;    // intervals staged per forward-pass chunk
constexpr int kZRow = 8;     // padded row of a staged interval solution
constexpr int kZInt = 12 * kZRow;
constexpr int kZPer = (kChunk * 84 + 63) / 64;  // prefetch registers per lane

struct SweepShared {
  union {
    double ring[kRing * kSlot];
    double zst[kChunk * kZInt];
    double pa[2 * 64 * 12];  // phase A: Phi and y of one 64-point chunk
  } u;
  double carry_phi[12], carry_y[12];
  double F[36], H[36], Gam[36], Rk[36], rho[6], Dr[6];
  double Pt[36], c[6];  // P_k column-major (Pt[j*6+m] = P[m][j]), c_k
  double EM1[36], Psi[18], phi[6], phic[6];
  double T1[9], T2[18], t3[3];
  double X1[36], X2[18], X3[6];
  double dx[2][8];
  double zsw[kBatch * 84];               // interval solutions of the last kBatch steps
  double dxs[kChunk * 6], dls[kChunk * 6]; // forward pass: dx and dlambda of one chunk
  double F0[6], FN[6], xb[6];
  double zero[2];  // a zero operand for uniform (branch-free) stage code
  int flag;
};

// Flat double offsets into SweepShared: the sweep stages address LDS as one
// array so that every lane runs the same instructions with per-lane offsets.
#define SGCM_OFF(field) ((int)(offsetof(SweepShared, field) / sizeof(double)))

// A = df/dx, W and L = (I - a A)^{-1} of one mesh point into an LDS slot
// (row-major 6 x 6 each).  Entries are stored as soon as they are formed so
// that few values stay live; the structural zeros of A and W are written too.
__device__ __forceinline__ void point_blocks(const BvpArgs& P, const double (&y)[12], const double (&tr)[4],
                                             double* slot, int* flag) {
  const double w1 = y[3], w2 = y[4], w3 = y[5];
  const double l1 = y[6], l2 = y[7], l3 = y[8], l4 = y[9], l5 = y[10], l6 = y[11];
  double* A = slot;
  double* W = slot + 36;
  double* L = slot + 72;
#pragma unroll
  for (int e = 0; e < 36; ++e) {
    A[e] = 0.0;
    W[e] = 0.0;
  }
  // the entries of A that the inverse needs: angle block (A00 A01 A10 A20 A21),
  // kinematic coupling E = A[0:3, 3:6], rate block Omega = A[3:6, 3:6]
  double a00 = 0.0, a01 = 0.0, a10 = 0.0, a20 = 0.0, a21 = 0.0;
  double E[9], Om[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    E[e] = 0.0;
    Om[e] = 0.0;
  }
  if (P.model == SGCM_MODEL_RIGID_BODY) {
    const double s = tr[0], c = tr[1], t = tr[2], k = tr[3];
    const double al = s * w2 + c * w3;
    const double be = c * w2 - s * w3;
    a00 = t * be;
    a01 = k * k * al;
    a10 = -al;
    a20 = k * be;
    a21 = k * t * al;
    E[0] = 1.0; E[1] = t * s; E[2] = t * c;
    E[3] = 0.0; E[4] = c;     E[5] = -s;
    E[6] = 0.0; E[7] = k * s; E[8] = k * c;
    Om[1] = P.a[0] * w3; Om[2] = P.a[0] * w2;
    Om[3] = P.a[1] * w3; Om[5] = P.a[1] * w1;
    Om[6] = P.a[2] * w2; Om[7] = P.a[2] * w1;
    const double Pc = l1 * t + l3 * k;
    const double Pt = l1 * k * k + l3 * k * t;
    const double Ptt = 2.0 * l1 * k * k * t + l3 * k * (t * t + k * k);
    W[0 * 6 + 0] = Pc * al + l2 * be - P.q;
    W[0 * 6 + 1] = W[1 * 6 + 0] = -Pt * be;
    W[0 * 6 + 4] = W[4 * 6 + 0] = l2 * s - Pc * c;
    W[0 * 6 + 5] = W[5 * 6 + 0] = Pc * s + l2 * c;
    W[1 * 6 + 1] = -Ptt * al - P.q;
    W[1 * 6 + 4] = W[4 * 6 + 1] = -Pt * s;
    W[1 * 6 + 5] = W[5 * 6 + 1] = -Pt * c;
    W[3 * 6 + 4] = W[4 * 6 + 3] = -l6 * P.a[2];
    W[3 * 6 + 5] = W[5 * 6 + 3] = -l5 * P.a[1];
    W[4 * 6 + 5] = W[5 * 6 + 4] = -l4 * P.a[0];
    W[2 * 6 + 2] = W[3 * 6 + 3] = W[4 * 6 + 4] = W[5 * 6 + 5] = -P.q;
  } else {
    E[0] = E[4] = E[8] = 1.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) W[i * 6 + i] = -P.q;
  }
  A[0 * 6 + 0] = a00;
  A[0 * 6 + 1] = a01;
  A[1 * 6 + 0] = a10;
  A[2 * 6 + 0] = a20;
  A[2 * 6 + 1] = a21;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      A[i * 6 + 3 + j] = E[i * 3 + j];
      A[(3 + i) * 6 + 3 + j] = Om[i * 3 + j];
    }
  const double a = P.alpha;
  double M1[9] = {1.0 - a * a00, -a * a01, 0.0, -a * a10, 1.0, 0.0, -a * a20, -a * a21, 1.0};
  double M2[9], Xb[9], Yb[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) M2[e] = ((e % 4) == 0 ? 1.0 : 0.0) - a * Om[e];
  const double d1 = inv3(M1, Xb);
  const double d2 = inv3(M2, Yb);
  if (d1 == 0.0 || d2 == 0.0) *flag = 1;
  // L = [[Xb, Xb (a E) Yb], [0, Yb]]
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double xe[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      xe[j] = a * (Xb[i * 3 + 0] * E[0 * 3 + j] + Xb[i * 3 + 1] * E[1 * 3 + j] + Xb[i * 3 + 2] * E[2 * 3 + j]);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      L[i * 6 + j] = Xb[i * 3 + j];
      L[i * 6 + 3 + j] = xe[0] * Yb[0 * 3 + j] + xe[1] * Yb[1 * 3 + j] + xe[2] * Yb[2 * 3 + j];
      L[(3 + i) * 6 + j] = 0.0;
      L[(3 + i) * 6 + 3 + j] = Yb[i * 3 + j];
    }
  }
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_newton(BvpArgs P, const double* __restrict__ x0,
                                               double* __restrict__ lam0, double* __restrict__ u0,
                                               double* __restrict__ Vout, double* __restrict__ traj,
                                               int32_t* __restrict__ status, int32_t* __restrict__ iters,
                                               double* __restrict__ ws) {
  const int lane0 = threadIdx.x;
  const int lane = lane0;
  const int64_t b = blockIdx.x;
  const int N = P.N, NP = N + 1;
  const double alpha = P.alpha;
  double* Y = ws + b * P.per_bvp;      // NP x 12: the iterate
  double* R = Y + 12 * (int64_t)NP;    // NP x 12: residuals (row 0 = [F_0, F_N]), then the step
  double* TR = R + 12 * (int64_t)NP;   // NP x 4: sin phi, cos phi, tan theta, sec theta
  double* Zg = TR + 4 * (int64_t)NP;   // N x 84: interval solutions, row-major 12 x 7

  __shared__ SweepShared sh;
  if (lane < 6) sh.xb[lane] = x0[b * 6 + lane];
  if (lane < 2) sh.zero[lane] = 0.0;
  for (int i = lane; i < 12 * NP; i += 64) Y[i] = 0.0;
  wave_mem_sync();

  int it = -1, st = SGCM_BVP_MAXITER;
  while (true) {
    // ---- residual F(Y) and its max norm (lane-parallel over mesh points) ----
    double lmax = 0.0;
    int bad = 0;
    for (int base = 0; base < NP; base += 64) {
      const int lane = opaque_lane(lane0);
      const int k = base + lane;
      const bool valid = k < NP;
      double yk[12], ph[12];
      if (valid) {
#pragma unroll
        for (int i = 0; i < 12; ++i) yk[i] = Y[12 * (int64_t)k + i];
        double A[36], W[36], tr[4] = {0.0, 0.0, 0.0, 0.0};
        point_eval(P, yk, ph, A, W, tr);
#pragma unroll
        for (int i = 0; i < 4; ++i) TR[4 * (int64_t)k + i] = tr[i];
#pragma unroll
        for (int i = 0; i < 12; ++i) {
          sh.u.pa[lane * 12 + i] = ph[i];
          sh.u.pa[768 + lane * 12 + i] = yk[i];
        }
      }
      wave_lds_sync();
      if (valid) {
        if (k == 0) {
#pragma unroll
          for (int i = 0; i < 6; ++i) {
            const double v = yk[i] - sh.xb[i];
            R[i] = v;
            bad |= !isfinite(v);
            lmax = fmax(lmax, fabs(v));
          }
        } else {
          const double* pp = lane > 0 ? &sh.u.pa[(lane - 1) * 12] : sh.carry_phi;
          const double* yp = lane > 0 ? &sh.u.pa[768 + (lane - 1) * 12] : sh.carry_y;
#pragma unroll
          for (int i = 0; i < 12; ++i) {
            const double v = yk[i] - yp[i] - alpha * (pp[i] + ph[i]);
            R[12 * (int64_t)k + i] = v;
            bad |= !isfinite(v);
            lmax = fmax(lmax, fabs(v));
          }
        }
        if (k == N) {
#pragma unroll
          for (int i = 0; i < 6; ++i) {
            const double v = yk[6 + i] - P.pw * yk[i];
            R[6 + i] = v;
            bad |= !isfinite(v);
            lmax = fmax(lmax, fabs(v));
          }
        }
      }
      wave_lds_sync();
      if (lane == 63 && valid) {
#pragma unroll
        for (int i = 0; i < 12; ++i) {
          sh.carry_phi[i] = ph[i];
          sh.carry_y[i] = yk[i];
        }
      }
      wave_lds_sync();
    }
    wave_mem_sync();  // residuals R visible to every lane
    const bool nonfinite = __any(bad);
    lmax = wave_max(lmax);
    if (it >= 0) {
      if (nonfinite) { st = SGCM_BVP_NONFINITE; break; }
      if (lmax <= P.tol) { st = SGCM_BVP_CONVERGED; break; }
      if (it == P.max_iter) { st = SGCM_BVP_MAXITER; break; }
    }

    // ---- backward Riccati sweep ----
    if (lane < 6) {
      sh.F0[lane] = R[lane];
      sh.FN[lane] = R[6 + lane];
      sh.c[lane] = -R[6 + lane];
    }
    if (lane < 36) {
      const int j = lane / 6, m = lane % 6;
      sh.Pt[lane] = (j == m) ? P.pw : 0.0;
    }
    if (lane == 0) sh.flag = 0;
    int pf_lo = N + 1;  // lowest point already in the ring
    int zhi = N;        // highest interval staged in zsw and not yet written out
    // write the staged interval solutions of intervals [klo, zhi] to global memory
    auto flush_z = [&](int klo) {
      const int lane = opaque_lane(lane0);
      const int cnt = (zhi - klo + 1) * 84;
      for (int e = lane; e < cnt; e += 64) {
        const int kk = klo + e / 84, r = e % 84;
        Zg[(int64_t)(kk - 1) * 84 + r] = sh.zsw[(kk & (kBatch - 1)) * 84 + r];
      }
      zhi = klo - 1;
    };
    wave_lds_sync();
    bool singular = false;
    for (int k = N; k >= 1; --k) {
      if (k - 1 < pf_lo) {
        // refill the ring with points [lo, hi]: issue the loads first, then
        // write out the staged solutions, so that the wait for the loads does
        // not include the stores
        const int lane = opaque_lane(lane0);
        const int hi = pf_lo - 1;
        const int lo = hi - (kBatch - 1) < 0 ? 0 : hi - (kBatch - 1);
        const int p = lo + lane;
        double py[12], pr[12], pt[4];
        if (lane < kBatch && p <= hi) {
          const int64_t pp = p >= 1 ? p : 1;  // r_0 does not exist; row 0 holds F_0, F_N
#pragma unroll
          for (int i = 0; i < 12; ++i) {
            py[i] = Y[12 * (int64_t)p + i];
            pr[i] = R[12 * pp + i];
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) pt[i] = TR[4 * (int64_t)p + i];
        }
        if (zhi > k) flush_z(k + 1);
        if (lane < kBatch && p <= hi) {
          double* slot = sh.u.ring + (p & (kRing - 1)) * kSlot;
#pragma unroll
          for (int i = 0; i < 12; ++i) slot[108 + i] = pr[i];
          point_blocks(P, py, pt, slot, &sh.flag);
        }
        pf_lo = lo;
        wave_lds_sync();
        if (sh.flag) {
          singular = true;
          break;
        }
      }
      double* const Bs = reinterpret_cast<double*>(&sh);
      const int ra = ((k - 1) & (kRing - 1)) * kSlot;  // point k-1 in the ring
      const int rb = (k & (kRing - 1)) * kSlot;        // point k
      // stage 0: interval products (independent of P_k).  Lane (i, j):
      //   F = L_a^T (I + a A_b^T), H = a L_a^T W_b, Gam = a L_a^T W_a share
      //   column i of L_a; R_k = L_b (I + a A_a); lanes j = 0, 1 also form
      //   rho = -L_b r^x and D^{-1} r^l = L_a^T r^l.
      if (opaque_lane(lane0) < 36) {
        const int lane = opaque_lane(lane0);
        const int i = lane / 6, j = lane % 6;
        const int r5 = rb + 108 + (j == 0 ? 0 : 6);
        // every LDS read of the stage is issued before the first product, so
        // the stage waits for LDS once
        double la[6], lb[6], ab[6], wb[6], wa[6], aa[6], rv[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
          la[m] = Bs[ra + 72 + m * 6 + i];
          lb[m] = Bs[rb + 72 + i * 6 + m];
          ab[m] = Bs[rb + j * 6 + m];
          wb[m] = Bs[rb + 36 + m * 6 + j];
          wa[m] = Bs[ra + 36 + m * 6 + j];
          aa[m] = Bs[ra + m * 6 + j];
          rv[m] = Bs[r5 + m];
        }
        const double cF = Bs[ra + 72 + j * 6 + i], cR = Bs[rb + 72 + i * 6 + j];
        __builtin_amdgcn_sched_barrier(0);
        double sF = 0.0, sH = 0.0, sG = 0.0, sR = 0.0, s5 = 0.0;
#pragma unroll
        for (int m = 0; m < 6; ++m) {
          sF = fma(la[m], ab[m], sF);
          sH = fma(la[m], wb[m], sH);
          sG = fma(la[m], wa[m], sG);
          sR = fma(lb[m], aa[m], sR);
          s5 = fma(j == 0 ? lb[m] : la[m], rv[m], s5);
        }
        sh.F[lane] = fma(alpha, sF, cF);
        sh.H[lane] = alpha * sH;
        sh.Gam[lane] = alpha * sG;
        sh.Rk[lane] = fma(alpha, sR, cR);
        if (j == 0) sh.rho[i] = -s5;
        if (j == 1) sh.Dr[i] = s5;
      }
      wave_lds_sync();
      // stage 1: EM1 = F P_k - H; Psi_w = (P_k + EM1) rate rows; lanes j = 0:
      // phic = F c_k + D^{-1} r^l and phi = c_k + phic
      if (opaque_lane(lane0) < 36) {
        const int lane = opaque_lane(lane0);
        const int i = lane / 6, j = lane % 6;
        double f[6], pt[6], cc[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
          f[m] = sh.F[i * 6 + m];
          pt[m] = sh.Pt[j * 6 + m];
          cc[m] = sh.c[m];
        }
        const double h = sh.H[lane], dr = sh.Dr[i], pji = sh.Pt[j * 6 + i], ci = sh.c[i];
        __builtin_amdgcn_sched_barrier(0);
        double e = -h, q = dr;
#pragma unroll
        for (int m = 0; m < 6; ++m) {
          e = fma(f[m], pt[m], e);
          q = fma(f[m], cc[m], q);
        }
        sh.EM1[lane] = e;
        if (i >= 3) sh.Psi[(i - 3) * 6 + j] = pji + e;
        if (j == 0) {
          sh.phic[i] = q;
          sh.phi[i] = q + ci;
        }
      }
      wave_lds_sync();
      // stage 2: rows r = 0..2 are Psi_w rows -> T2 = Psi_w R_k - Gam_w,
      // T1 = Psi_w B_k, t3 = Psi_w rho + phi_w; rows r = 3..8 are EM1 rows ->
      // X1 = EM1 R_k - Gam, X2 = EM1 B_k, X3 = EM1 rho.  Column o = 0..5: R_k
      // column, 6..8: B_k column (a L_b rate columns), 9: rho.  Each lane forms
      // two outputs of one row.
      if (opaque_lane(lane0) < 45) {
        const int lane = opaque_lane(lane0);
        const int r = lane / 5, o0 = 2 * (lane % 5);
        const int lrow = (r < 3) ? SGCM_OFF(Psi) + r * 6 : SGCM_OFF(EM1) + (r - 3) * 6;
        const int grow = (r < 3) ? 3 + r : r - 3;
        double lv[6], rc[2][6], cv[2], coef[2], csgn[2];
        int dst[2];
#pragma unroll
        for (int m = 0; m < 6; ++m) lv[m] = Bs[lrow + m];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int o = o0 + h;
          const int rbase = (o < 6) ? SGCM_OFF(Rk) + o : (o < 9) ? rb + 72 + 3 + (o - 6) : SGCM_OFF(rho);
          const int rs = (o < 9) ? 6 : 1;
          const int cidx = (o < 6) ? SGCM_OFF(Gam) + grow * 6 + o
                                   : (o == 9 && r < 3) ? SGCM_OFF(phi) + 3 + r : SGCM_OFF(zero);
          csgn[h] = (o < 6) ? -1.0 : 1.0;
          coef[h] = (o >= 6 && o < 9) ? alpha : 1.0;
          dst[h] = (r < 3) ? ((o < 6) ? SGCM_OFF(T2) + r * 6 + o
                                      : (o < 9) ? SGCM_OFF(T1) + r * 3 + (o - 6) : SGCM_OFF(t3) + r)
                           : ((o < 6) ? SGCM_OFF(X1) + (r - 3) * 6 + o
                                      : (o < 9) ? SGCM_OFF(X2) + (r - 3) * 3 + (o - 6)
                                                : SGCM_OFF(X3) + (r - 3));
#pragma unroll
          for (int m = 0; m < 6; ++m) rc[h][m] = Bs[rbase + m * rs];
          cv[h] = Bs[cidx];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          double acc = 0.0;
#pragma unroll
          for (int m = 0; m < 6; ++m) acc = fma(lv[m], rc[h][m], acc);
          Bs[dst[h]] = fma(coef[h], acc, csgn[h] * cv[h]);
        }
      }
      wave_lds_sync();
      // stage 3: Z3 = I + S_w T1 and its inverse (every lane), then lane (i, j):
      // M = Z3^{-1} S_w [T2 | t3], P_{k-1} = X1 - X2 M, c_{k-1} = X3 + phic - X2 m,
      // G_k = R_k - B_k M, g_k = rho - B_k m
      {
        const int lane = opaque_lane(lane0);
        const int ll = lane < 42 ? lane : 41;
        const int i = ll / 7, j = ll % 7;
        const bool col = j < 6;
        double t1[9], v[3], x2[3], lb[3];
#pragma unroll
        for (int e = 0; e < 9; ++e) t1[e] = sh.T1[e];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          v[m] = Bs[col ? SGCM_OFF(T2) + m * 6 + j : SGCM_OFF(t3) + m];
          x2[m] = sh.X2[i * 3 + m];
          lb[m] = Bs[rb + 72 + i * 6 + 3 + m];
        }
        const double p0 = Bs[col ? SGCM_OFF(X1) + i * 6 + j : SGCM_OFF(X3) + i];
        const double p1 = Bs[col ? SGCM_OFF(zero) : SGCM_OFF(phic) + i];
        const double g0 = Bs[col ? SGCM_OFF(Rk) + i * 6 + j : SGCM_OFF(rho) + i];
        __builtin_amdgcn_sched_barrier(0);
        double Z3[9], Zi[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            double t = (a == c) ? 1.0 : 0.0;
#pragma unroll
            for (int m = 0; m < 3; ++m) t = fma(P.Sw[a * 3 + m], t1[m * 3 + c], t);
            Z3[a * 3 + c] = t;
          }
        const double det = inv3(Z3, Zi);
        if (det == 0.0) singular = true;
        if (lane < 42 && !singular) {
          double w[3], mu[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) w[a] = P.Sw[a * 3 + 0] * v[0] + P.Sw[a * 3 + 1] * v[1] + P.Sw[a * 3 + 2] * v[2];
#pragma unroll
          for (int a = 0; a < 3; ++a) mu[a] = Zi[a * 3 + 0] * w[0] + Zi[a * 3 + 1] * w[1] + Zi[a * 3 + 2] * w[2];
          double pn = p0 + p1;
          double gn = g0;
#pragma unroll
          for (int m = 0; m < 3; ++m) {
            pn = fma(-x2[m], mu[m], pn);
            gn = fma(-alpha * lb[m], mu[m], gn);
          }
          Bs[col ? SGCM_OFF(Pt) + j * 6 + i : SGCM_OFF(c) + i] = pn;
          double* zk = sh.zsw + (k & (kBatch - 1)) * 84;
          zk[i * 7 + j] = gn;
          zk[(6 + i) * 7 + j] = pn;
        }
      }
      wave_lds_sync();
      if (singular) break;
    }
    if (singular) {
      st = SGCM_BVP_SINGULAR;
      if (it < 0) it = 0;
      break;
    }
    if (zhi >= 1) flush_z(1);

    // ---- forward pass; the step goes into R ----
    wave_mem_sync();  // interval solutions Z visible to every lane
    if (lane < 6) {
      const double d = -sh.F0[lane];
      sh.dx[0][lane] = d;
      R[lane] = d;
    }
    double zr[kZPer];
    auto zload = [&](int c0) {
      const int lane = opaque_lane(lane0);
#pragma unroll
      for (int t = 0; t < kZPer; ++t) {
        const int e = lane + 64 * t;
        if (e < kChunk * 84 && c0 + e / 84 <= N) zr[t] = Zg[(int64_t)(c0 - 1) * 84 + e];
      }
    };
    zload(1);
    int cur = 0;
    for (int c0 = 1; c0 <= N; c0 += kChunk) {
      const int lane = opaque_lane(lane0);
#pragma unroll
      for (int t = 0; t < kZPer; ++t) {
        const int e = lane + 64 * t;
        if (e < kChunk * 84 && c0 + e / 84 <= N) {
          const int kl = e / 84, rem = e % 84;
          sh.u.zst[kl * kZInt + (rem / 7) * kZRow + rem % 7] = zr[t];
        }
      }
      wave_lds_sync();
      if (c0 + kChunk <= N) zload(c0 + kChunk);
      const int nk = (N - c0 + 1) < kChunk ? (N - c0 + 1) : kChunk;
      for (int kl = 0; kl < nk; ++kl) {
        if (lane < 12) {
          const double* zrow = sh.u.zst + kl * kZInt + lane * kZRow;
          double v = zrow[6];
#pragma unroll
          for (int j = 0; j < 6; ++j) v = fma(zrow[j], sh.dx[cur][j], v);
          if (lane < 6) {
            sh.dx[cur ^ 1][lane] = v;
            sh.dxs[kl * 6 + lane] = v;        // dx_k
          } else {
            sh.dls[kl * 6 + lane - 6] = v;    // dlambda_{k-1}
          }
        }
        wave_lds_sync();
        cur ^= 1;
      }
      // write out the chunk: dx of points c0..c0+nk-1, dlambda of points c0-1..c0+nk-2
      for (int e = lane; e < 12 * nk; e += 64) {
        const int half = e / (6 * nk), q = e % (6 * nk), kl = q / 6, i = q % 6;
        if (half == 0) R[12 * (int64_t)(c0 + kl) + i] = sh.dxs[kl * 6 + i];
        else R[12 * (int64_t)(c0 - 1 + kl) + 6 + i] = sh.dls[kl * 6 + i];
      }
    }
    if (lane < 6) R[12 * (int64_t)N + 6 + lane] = P.pw * sh.dx[cur][lane] - sh.FN[lane];
    wave_mem_sync();
    for (int i = lane; i < 12 * NP; i += 64) Y[i] += R[i];
    wave_mem_sync();
    ++it;
  }
  // ---- outputs (eq. optuv at t = 0) ----
  if (lane < 6) lam0[b * 6 + lane] = Y[6 + lane];
  if (lane < P.m)
    u0[b * P.m + lane] = P.U[lane * 3 + 0] * Y[9] + P.U[lane * 3 + 1] * Y[10] + P.U[lane * 3 + 2] * Y[11];
  if (Vout) {
    double part = 0.0;
    for (int k = lane; k < NP; k += 64) {
      const double* yk = Y + 12 * (int64_t)k;
      double xx = 0.0, uu = 0.0;
#pragma unroll
      for (int i = 0; i < 6; ++i) xx += yk[i] * yk[i];
      for (int j = 0; j < P.m; ++j) {
        const double u = P.U[j * 3 + 0] * yk[9] + P.U[j * 3 + 1] * yk[10] + P.U[j * 3 + 2] * yk[11];
        uu += u * u;
      }
      const double L = 0.5 * (P.q * xx + P.r * uu);
      part += ((k == 0 || k == N) ? 0.5 : 1.0) * L;
    }
    part = wave_sum(part);
    if (lane == 0) {
      const double* yN = Y + 12 * (int64_t)N;
      double xx = 0.0;
      for (int i = 0; i < 6; ++i) xx += yN[i] * yN[i];
      Vout[b] = P.h * part + 0.5 * P.pw * xx;
    }
  }
  if (traj) {
    double* out = traj + b * 12 * (int64_t)NP;
    for (int i = lane; i < 12 * NP; i += 64) out[i] = Y[i];
  }
  if (lane == 0) {
    status[b] = st;
    iters[b] = it < 0 ? 0 : it;
  }
}

__global__ __launch_bounds__(256) void k_rhs(BvpArgs P, int64_t n, const double* __restrict__ y,
                                             double* __restrict__ phi_out, double* __restrict__ dphi) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double phi[12], A[36], W[36];
  point_eval(P, y + 12 * i, phi, A, W);
#pragma unroll
  for (int c = 0; c < 12; ++c) phi_out[12 * i + c] = phi[c];
  if (dphi) {
    double* D = dphi + 144 * i;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        D[r * 12 + c] = A[r * 6 + c];
        D[r * 12 + 6 + c] = -S_at(P, r, c);
        D[(6 + r) * 12 + c] = W[r * 6 + c];
        D[(6 + r) * 12 + 6 + c] = -A[c * 6 + r];
      }
  }
}

// Validate a problem and derive the kernel arguments.
int make_bvp_args(const sgcm_problem* p, BvpArgs* a) {
  if (!p) return SGCM_EINVAL;
  if (p->model != SGCM_MODEL_RIGID_BODY && p->model != SGCM_MODEL_LINEARISED) return SGCM_EINVAL;
  if (p->n != 6 || p->m < 1 || p->m > 3) return SGCM_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (!(std::isfinite(p->J[i]) && p->J[i] > 0.0)) return SGCM_EINVAL;
  for (int i = 0; i < 3 * p->m; ++i)
    if (!std::isfinite(p->B[i])) return SGCM_EINVAL;
  if (!(std::isfinite(p->q_w) && p->q_w >= 0.0) || !(std::isfinite(p->r_w) && p->r_w > 0.0) ||
      !(std::isfinite(p->p_w) && p->p_w >= 0.0) || !(std::isfinite(p->T) && p->T > 0.0))
    return SGCM_EINVAL;
  if (p->N < 1 || p->N > 65536) return SGCM_EINVAL;
  if (!(p->tol >= 0.0) || p->max_iter < 0 || p->max_iter > 1000) return SGCM_EINVAL;
  if (p->precision != SGCM_FP64 && p->precision != SGCM_FP32) return SGCM_EINVAL;
  if (p->precision != SGCM_FP64) return SGCM_EUNSUPPORTED;
  a->model = p->model;
  a->m = p->m;
  a->N = p->N;
  a->max_iter = p->max_iter;
  const double* J = p->J;
  for (int i = 0; i < 3; ++i) a->J[i] = J[i];
  a->a[0] = (J[1] - J[2]) / J[0];
  a->a[1] = (J[2] - J[0]) / J[1];
  a->a[2] = (J[0] - J[1]) / J[2];
  for (int i = 0; i < 3; ++i)
    for (int l = 0; l < 3; ++l) {
      double s = 0.0;
      for (int j = 0; j < p->m; ++j) s += p->B[i + 3 * j] * p->B[l + 3 * j];
      a->Sw[i * 3 + l] = s / (p->r_w * J[i] * J[l]);
    }
  for (int j = 0; j < 3; ++j)
    for (int i = 0; i < 3; ++i) a->U[j * 3 + i] = (j < p->m) ? -p->B[i + 3 * j] / (p->r_w * J[i]) : 0.0;
  a->q = p->q_w;
  a->r = p->r_w;
  a->pw = p->p_w;
  a->T = p->T;
  a->h = p->T / p->N;
  a->alpha = 0.5 * a->h;
  a->tol = p->tol;
  const int64_t NP = (int64_t)p->N + 1;
  const int64_t doubles = (12 + 12 + 4) * NP + 84 * (int64_t)p->N;
  a->per_bvp = (doubles + 31) / 32 * 32;  // 256-byte multiples
  return SGCM_OK;
}

}  // namespace
}  // namespace sgcm

using namespace sgcm;

extern "C" int sgcm_solve_bvps_workspace(const sgcm_problem* p, int64_t n_bvps, size_t* bytes) {
  BvpArgs a;
  if (!bytes || n_bvps < 0) return SGCM_EINVAL;
  int rc = make_bvp_args(p, &a);
  if (rc != SGCM_OK) return rc;
  *bytes = (size_t)a.per_bvp * sizeof(double) * (size_t)n_bvps;
  return SGCM_OK;
}

extern "C" int sgcm_solve_bvps(const sgcm_problem* p, int64_t n_bvps, const double* x0, double* lambda0,
                               double* u0, double* V, double* traj, int32_t* status, int32_t* iters,
                               void* workspace, size_t ws_bytes, void* stream) {
  BvpArgs a;
  if (n_bvps < 0) return SGCM_EINVAL;
  int rc = make_bvp_args(p, &a);
  if (rc != SGCM_OK) return rc;
  if (n_bvps == 0) return SGCM_OK;
  if (n_bvps > 0x7fffffffLL) return SGCM_EUNSUPPORTED;
  if (!x0 || !lambda0 || !u0 || !status || !iters || !workspace) return SGCM_EINVAL;
  if (((uintptr_t)workspace & 255u) != 0) return SGCM_EINVAL;
  if (ws_bytes < (size_t)a.per_bvp * sizeof(double) * (size_t)n_bvps) return SGCM_EINVAL;
  hipLaunchKernelGGL(k_newton, dim3((unsigned)n_bvps), dim3(64), 0, (hipStream_t)stream, a, x0, lambda0,
                     u0, V, traj, status, iters, (double*)workspace);
  return hipGetLastError() == hipSuccess ? SGCM_OK : SGCM_EDEVICE;
}

extern "C" int sgcm_characteristic_rhs(const sgcm_problem* p, int64_t n_points, const double* y, double* phi,
                                       double* dphi, void* stream) {
  BvpArgs a;
  if (n_points < 0) return SGCM_EINVAL;
  int rc = make_bvp_args(p, &a);
  if (rc != SGCM_OK) return rc;
  if (n_points == 0) return SGCM_OK;
  if (!y || !phi) return SGCM_EINVAL;
  const int64_t blocks = (n_points + 255) / 256;
  if (blocks > 0x7fffffffLL) return SGCM_EUNSUPPORTED;
  hipLaunchKernelGGL(k_rhs, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a, n_points, y, phi,
                     dphi);
  return hipGetLastError() == hipSuccess ? SGCM_OK : SGCM_EDEVICE;
}

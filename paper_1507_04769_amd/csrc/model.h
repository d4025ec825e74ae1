// Device-side pieces shared by the collocation solvers of libsgcm (the
// trapezoid in bvp.hip, the four-point Lobatto IIIA formula in lobatto.hip):
// the kernel arguments of a problem, the characteristic right-hand side of
// the rigid-body models and its Jacobian blocks, and wavefront helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sgcm.h"

namespace sgcm {

struct BvpArgs {
  int model, m, N, max_iter;
  double J[3];
  double a[3];   // gyroscopic coefficients: w_i' gets a_i w_j w_k
  double Sw[9];  // (1/r_w) J^{-1} B B^T J^{-1}, row-major 3 x 3
  double U[9];   // u* = U lambda_w, U[j][i] = -B[i][j] / (r_w J_i), row-major m x 3
  double q, r, pw, T, h, alpha, tol;
  int64_t per_bvp;  // doubles of workspace per BVP
  // A solve plan's first Newton steps for the six unit initial states, 6 x
  // (N + 1) x 12 (device), or null: then each BVP takes its own first step.
  const double* y1;
  // Statuses and iteration counts (6 + 6, device) of the solves that made y1
  // inside this call, or null (a plan checked on the host): y1 is used only
  // if every one took its first step and nothing more (status CONVERGED or
  // MAXITER after 0 iterations), else each BVP takes its own first step.
  const int32_t* y1_check;
  int sinv;         // 1: S_w is invertible and Si holds its inverse
  int fp32;         // 1: Newton linear solve in FP32 (inexact Newton)
  double Si[9];
  int max_halvings;  // backtracking cap H of each counted Newton step
  // Continuation stages (host-driven launches on one workspace):
  int resume;   // 1: start from the iterate the previous stage left in the
                // workspace (skipping a BVP whose previous stage failed) and
                // add this stage's iterations to iters[]
  int keep;     // 1: leave the final iterate in the workspace's first buffer
  int outputs;  // 1: write lambda0, u0, V and traj (the last stage)
  int scheme;   // sgcm_scheme of the collocation
  double lob[4][4];  // the four-point Lobatto IIIA tableau (SGCM_LOBATTO4)
  int nb, fc;   // tile sizes of the trapezoidal solve: sweep batch, forward chunk
};

// Sufficient-decrease constant of the backtracking test
// max|F(Y + t d)| <= (1 - sigma t) max|F(Y)|.
constexpr double kArmijoSigma = 1e-4;

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

// LDS hand-off inside the wavefront: a compiler-only barrier.  LDS accesses of
// one wavefront are performed in program order, so a value one lane writes is
// seen by a later read of another lane without waiting for the write.
__device__ __forceinline__ void lds_handoff() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


// ---- the first Newton steps of the unit initial states (first_steps.hip) -----

// The first Newton step from Y = 0 of the trapezoidal solve of problem a
// (FP64; mesh of N intervals of width a.h) for the six unit initial states,
// into y1 (device, 6 x (N + 1) x 12), with the statuses and iteration counts
// (device, 6 + 6) of a solve with max_iter = 0: SGCM_BVP_MAXITER and 0, or
// SGCM_BVP_NONFINITE when the steps are not finite.  Two launches on stream s.
int launch_first_steps(const BvpArgs& a, int N, double* y1, int32_t* chk, hipStream_t s);

// ---- Example III and the time dimension (example3.hip) ----------------------

// Workspace, solve and characteristic right-hand side for the model
// SGCM_MODEL_EXAMPLE3 (its own solver).  ex3_solve: rows are (t0, x0) (tx = 1)
// or x0 (tx = 0, t0 = 0); arguments and errors as for sgcm_solve_bvps.
int ex3_workspace(const sgcm_problem* p, int64_t n_bvps, size_t* bytes);
int ex3_solve(const sgcm_problem* p, int64_t n_bvps, const double* rows, int tx, double* lambda0, double* u0,
              double* V, double* traj, int32_t* status, int32_t* iters, void* workspace, size_t ws_bytes,
              void* stream);
int ex3_characteristic_rhs(const sgcm_problem* p, int64_t n_points, const double* y, double* phi, double* dphi,
                           void* stream);

// ---- four-point Lobatto IIIA collocation (lobatto.hip) ----------------------

// Workspace of one BVP of the Lobatto solver, in doubles (a multiple of 32).
int64_t lobatto_doubles(int64_t N);

// One launch of the Lobatto Newton kernel over n_bvps BVPs (workgroup g takes
// BVP order[g], or g without an order; workspace slot g of lobatto_doubles(N)).
int launch_lobatto(const BvpArgs& a, int64_t n_bvps, const double* x0, double* lambda0, double* u0, double* V,
                   double* traj, int32_t* status, int32_t* iters, double* workspace, const int32_t* order,
                   hipStream_t s);

}  // namespace sgcm

// Characteristic BVPs on gfx950 (Sec. 3.1, eq. hamchar and eq. optuv).
//
// One 64-lane workgroup (one wavefront) owns one BVP.  The discretisation is
// trapezoidal collocation on N uniform intervals; the unknowns are
// y_k = (x_k, lambda_k), k = 0..N, and the residual is
//   F = [ x_0 - xbar ; r_k = y_k - y_{k-1} - (h/2)(Phi_{k-1} + Phi_k), k=1..N ;
//         lambda_N - p_w x_N ],
// with Phi = [ f(x, u*) ; -q_w x - A^T lambda ], A = df/dx, u* = argmin_u H.
// Newton's linear system is block bidiagonal:
//   (I - (h/2) Phi'_k) dy_k = (I + (h/2) Phi'_{k-1}) dy_{k-1} - r_k,
//   Phi' = [[A, -S], [W, -A^T]],  S = (1/r_w) Bt Bt^T,  W = -q_w I - sum_i lambda_i f_i''.
// It is solved by a backward Riccati sweep: with dlambda_k = P_k dx_k + c_k
// (P_N = p_w I, c_N = -F_N) each interval gives a 12 x 12 system for
// (dx_k, dlambda_{k-1}) in terms of dx_{k-1}, solved by Gauss-Jordan with row
// partial pivoting cooperatively by the 64 lanes in LDS; its solution rows
// are dx_k = G_k dx_{k-1} + g_k and dlambda_{k-1} = P_{k-1} dx_{k-1} + c_{k-1}.
// A forward pass from dx_0 = -F_0 recovers the step.  Mesh-point work
// (Phi, A, W) and the residual are lane-parallel over k.
#include <hip/hip_runtime.h>

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

constexpr int kRows = 12, kCols = 19, kLd = 20;

// Phi, A = df/dx and W = -q I - Hessian_x(lambda^T f) at one mesh point.
__device__ __forceinline__ void point_eval(const BvpArgs& P, const double* __restrict__ y,
                                           double (&phi)[12], double (&A)[36], double (&W)[36]) {
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

__global__ __launch_bounds__(64) void k_newton(BvpArgs P, const double* __restrict__ x0,
                                               double* __restrict__ lam0, double* __restrict__ u0,
                                               double* __restrict__ Vout, double* __restrict__ traj,
                                               int32_t* __restrict__ status, int32_t* __restrict__ iters,
                                               double* __restrict__ ws) {
  const int lane = threadIdx.x;
  const int64_t b = blockIdx.x;
  const int N = P.N, NP = N + 1;
  const double alpha = P.alpha;
  double* Y = ws + b * P.per_bvp;        // NP x 12
  double* PD = Y + 12 * (int64_t)NP;     // 84 x NP: Phi (12), A (36), W (36), by component
  double* R = PD + 84 * (int64_t)NP;     // NP x 12: row 0 = [F_0, F_N], row k = r_k
  double* Z = R + 12 * (int64_t)NP;      // N x 84: solution rows of interval k at (k-1)*84

  __shared__ double Ka[kRows][kLd];
  __shared__ double AW[2][72];  // [0] = A_k, W_k   [1] = A_{k-1}, W_{k-1}
  __shared__ double Pc[6][7];   // P_k | c_k
  __shared__ double rk[12];
  __shared__ double dx[6];
  __shared__ double xb[6];
  __shared__ int prow[12];

  if (lane < 6) xb[lane] = x0[b * 6 + lane];
  for (int i = lane; i < 12 * NP; i += 64) Y[i] = 0.0;
  __syncthreads();

  int it = -1, st = SGCM_BVP_MAXITER;
  while (true) {
    // ---- mesh points: Phi, A, W ----
    for (int k = lane; k < NP; k += 64) {
      double phi[12], A[36], W[36];
      point_eval(P, Y + 12 * (int64_t)k, phi, A, W);
#pragma unroll
      for (int c = 0; c < 12; ++c) PD[c * (int64_t)NP + k] = phi[c];
#pragma unroll
      for (int c = 0; c < 36; ++c) {
        PD[(12 + c) * (int64_t)NP + k] = A[c];
        PD[(48 + c) * (int64_t)NP + k] = W[c];
      }
    }
    __syncthreads();
    // ---- residual and its max norm ----
    double lmax = 0.0;
    int bad = 0;
    for (int k = lane; k < NP; k += 64) {
      double v[12];
      if (k == 0) {
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          v[i] = Y[i] - xb[i];
          v[6 + i] = Y[12 * (int64_t)N + 6 + i] - P.pw * Y[12 * (int64_t)N + i];
        }
      } else {
#pragma unroll
        for (int i = 0; i < 12; ++i)
          v[i] = Y[12 * (int64_t)k + i] - Y[12 * (int64_t)(k - 1) + i] -
                 alpha * (PD[i * (int64_t)NP + k - 1] + PD[i * (int64_t)NP + k]);
      }
#pragma unroll
      for (int i = 0; i < 12; ++i) {
        R[12 * (int64_t)k + i] = v[i];
        bad |= !isfinite(v[i]);
        lmax = fmax(lmax, fabs(v[i]));
      }
    }
    const bool nonfinite = __any(bad);
    lmax = wave_max(lmax);
    __syncthreads();
    if (it >= 0) {
      if (nonfinite) { st = SGCM_BVP_NONFINITE; break; }
      if (lmax <= P.tol) { st = SGCM_BVP_CONVERGED; break; }
      if (it == P.max_iter) { st = SGCM_BVP_MAXITER; break; }
    }
    // ---- backward Riccati sweep ----
    if (lane < 42) {
      const int i = lane / 7, c = lane % 7;
      Pc[i][c] = (c < 6) ? ((i == c) ? P.pw : 0.0) : -R[6 + i];
    }
    bool singular = false;
    for (int k = N; k >= 1; --k) {
      for (int e = lane; e < 144; e += 64) {
        const int slot = e / 72, c = e % 72;
        AW[slot][c] = PD[(12 + c) * (int64_t)NP + (k - slot)];
      }
      if (lane < 12) rk[lane] = R[12 * (int64_t)k + lane];
      __syncthreads();
      const double* A0 = AW[0];
      const double* W0 = AW[0] + 36;
      const double* A1 = AW[1];
      const double* W1 = AW[1] + 36;
      for (int e = lane; e < kRows * kCols; e += 64) {
        const int r = e / kCols, c = e % kCols;
        double v;
        if (r < 6) {
          if (c < 6) {
            v = (r == c ? 1.0 : 0.0) - alpha * A0[r * 6 + c];
            for (int mm = 3; mm < 6; ++mm) v += alpha * S_at(P, r, mm) * Pc[mm][c];
          } else if (c < 12) {
            v = alpha * S_at(P, r, c - 6);
          } else if (c < 18) {
            v = (r == c - 12 ? 1.0 : 0.0) + alpha * A1[r * 6 + (c - 12)];
          } else {
            v = -rk[r];
            for (int mm = 3; mm < 6; ++mm) v -= alpha * S_at(P, r, mm) * Pc[mm][6];
          }
        } else {
          const int i = r - 6;
          if (c < 6) {
            v = Pc[i][c] - alpha * W0[i * 6 + c];
            for (int mm = 0; mm < 6; ++mm) v += alpha * A0[mm * 6 + i] * Pc[mm][c];
          } else if (c < 12) {
            const int j = c - 6;
            v = -((i == j ? 1.0 : 0.0) - alpha * A1[j * 6 + i]);
          } else if (c < 18) {
            v = alpha * W1[i * 6 + (c - 12)];
          } else {
            v = -rk[6 + i] - Pc[i][6];
            for (int mm = 0; mm < 6; ++mm) v -= alpha * A0[mm * 6 + i] * Pc[mm][6];
          }
        }
        Ka[r][c] = v;
      }
      __syncthreads();
      // Gauss-Jordan with row partial pivoting (first index of the largest |a|)
      unsigned used = 0;
      for (int j = 0; j < 12; ++j) {
        int p = -1;
        double best = 0.0;
        for (int r = 0; r < 12; ++r) {
          if ((used >> r) & 1u) continue;
          const double a = fabs(Ka[r][j]);
          if (a > best) {
            best = a;
            p = r;
          }
        }
        if (p < 0) {
          singular = true;
          break;
        }
        used |= 1u << p;
        if (lane == 0) prow[j] = p;
        const double inv = 1.0 / Ka[p][j];
        double av[4], mv[4], pv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int e = lane + 64 * t;
          const int r = e / kCols, c = e % kCols;
          if (e < kRows * kCols && c > j) {
            av[t] = Ka[r][c];
            mv[t] = Ka[r][j];
            pv[t] = Ka[p][c];
          }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int e = lane + 64 * t;
          const int r = e / kCols, c = e % kCols;
          if (e < kRows * kCols && c > j) Ka[r][c] = (r == p) ? av[t] * inv : av[t] - mv[t] * inv * pv[t];
        }
        __syncthreads();
      }
      if (singular) break;
      for (int e = lane; e < 84; e += 64) {
        const int j = e / 7, c = e % 7;
        const double v = Ka[prow[j]][12 + c];
        Z[(int64_t)(k - 1) * 84 + e] = v;
        if (j >= 6) Pc[j - 6][c] = v;
      }
      __syncthreads();
    }
    if (singular) {
      st = SGCM_BVP_SINGULAR;
      if (it < 0) it = 0;
      break;
    }
    // ---- forward pass and update ----
    if (lane < 6) {
      const double d = -R[lane];
      dx[lane] = d;
      Y[lane] += d;
    }
    __syncthreads();
    for (int k = 1; k <= N; ++k) {
      double v = 0.0;
      if (lane < 12) {
        const double* zr = Z + (int64_t)(k - 1) * 84 + lane * 7;
        v = zr[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) v += zr[j] * dx[j];
      }
      __syncthreads();
      if (lane < 6) {
        dx[lane] = v;
        Y[12 * (int64_t)k + lane] += v;
      } else if (lane < 12) {
        Y[12 * (int64_t)(k - 1) + lane] += v;  // dlambda_{k-1}
      }
      __syncthreads();
    }
    if (lane < 6) Y[12 * (int64_t)N + 6 + lane] += P.pw * dx[lane] - R[6 + lane];
    __syncthreads();
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
  const int64_t doubles = (12 + 84 + 12) * NP + 84 * (int64_t)p->N;
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

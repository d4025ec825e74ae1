// Four-point Lobatto IIIA collocation of the characteristic BVP on gfx950 (the
// paper's BVP formula: Sec. 3.1, and Sec. 5.1 where it is used with error
// control).
//
// On interval k of width h the collocation points are t_k + c_j h,
// c = (0, (5 - sqrt 5)/10, (5 + sqrt 5)/10, 1).  The unknowns are the mesh values
// y_k = (x_k, lambda_k) and the two interior stage values Z_{k,1}, Z_{k,2},
// stored point by point: y_0, then for every interval Z_{k,1}, Z_{k,2}, y_{k+1}
// (point 3k + j holds stage j of interval k; Z_{k,0} = y_k, Z_{k,3} = y_{k+1}).
// The equations are the boundary rows x_0 = xbar and lambda_N = p_w x_N, and
//   Z_{k,i} = y_k + h sum_j a_ij Phi(Z_{k,j}),  i = 1, 2, 3,
// with the Lobatto IIIA coefficients a_ij (closed forms; the last row is the
// Lobatto quadrature (1, 5, 5, 1) / 12).
//
// One 64-lane workgroup solves one BVP with the damped Newton iteration of the
// trapezoidal solver (same first step, statuses, stopping test, backtracking
// and continuation stages).  The Newton system is solved in three passes:
//  (1) condensation, interval by interval: the equations of the two interior
//      stages give dZ = X1 dy_k + X4 dy_{k+1} + X0 (a 24 x 24 system with 25
//      right-hand sides), and the last stage equation becomes the interval
//      relation C_k dy_k + D_k dy_{k+1} = e_k;
//  (2) a backward Riccati sweep dlambda_k = P_k dx_k + c_k from P_N = p_w I,
//      c_N = -F_N, each step a 12 x 12 system with 7 right-hand sides giving
//      dx_{k+1} = G_k dx_k + g_k as well;
//  (3) the forward pass from dx_0 = -F_0, the interior stages recovered from
//      (1).
// The dense systems are solved in LDS by Gauss-Jordan elimination with row
// partial pivoting, one lane per column.  This solver is the paper's formula
// and the accurate reference of the total-error estimate, not the throughput
// path: its intervals are condensed one after the other by the whole wave.
#include <hip/hip_runtime.h>

#include <cmath>

#include "model.h"
#include "wave_la.h"

namespace sgcm {
namespace {

constexpr int kLd = 50;  // LDS row stride of the dense systems, in doubles

struct LobShared {
  double A[24 * kLd];  // the dense system of the step
  double v[32];        // small vectors: dx, dlambda, dy_k, dy_{k+1}
  double xb[6];
  double P[36], c[6];  // the sweep's [P | c] of the next interval
};

// Gauss-Jordan elimination with row partial pivoting (the first row of
// largest |a| in the pivot column) of the n x ncols system held in LDS
// (row-major, stride kLd, ncols <= 64): lane j takes column j into
// registers, the elimination runs there (gauss_jordan: the pivot column
// broadcast by readlane, no LDS traffic per row), and the columns n..ncols-1
// go back: A[:, :n]^{-1} A[:, n:].  Returns false on a zero or non-finite
// pivot.  (Row by row in LDS, the elimination waited on LDS once per row and
// pivot: about four fifths of the four-point solve.)
template <int n, int ncols>
__device__ bool wave_gauss_jordan(double* A) {
  static_assert(ncols <= 64 && n <= ncols, "one column per lane");
  const int lane = threadIdx.x;
  double v[n];
#pragma unroll
  for (int i = 0; i < n; ++i) v[i] = lane < ncols ? A[i * kLd + lane] : 0.0;
  const bool ok = gauss_jordan<n, 64, true>(v);
  if (lane >= n && lane < ncols) {
#pragma unroll
    for (int i = 0; i < n; ++i) A[i * kLd + lane] = v[i];
  }
  lds_handoff();
  return ok;
}

// Entry (r, c) of the 12 x 12 Jacobian of Phi from A and W of point_eval:
// Phi' = [[A, -S], [W, -A^T]].
__device__ __forceinline__ double phi_jac(const BvpArgs& P, const double (&A)[36], const double (&W)[36], int r,
                                          int c) {
  if (r < 6) return c < 6 ? A[r * 6 + c] : -S_at(P, r, c - 6);
  return c < 6 ? W[(r - 6) * 6 + c] : -A[(c - 6) * 6 + (r - 6)];
}

// Workspace of one BVP (doubles, from the start of its slot).
struct LobLayout {
  int64_t npt, ny;  // collocation points 3N + 1, unknowns 12 npt
  int64_t Y, Yt, D, F, Phi, Jp, X, CDe, Z, total;
  __host__ __device__ explicit LobLayout(int64_t N) {
    npt = 3 * N + 1;
    ny = 12 * npt;
    Y = 0;
    Yt = Y + ny;
    D = Yt + ny;
    F = D + ny;
    Phi = F + ny;
    Jp = Phi + ny;              // 144 per point: Phi' row-major
    X = Jp + 144 * npt;         // 24 x 25 per interval: the condensation [X1 X4 X0]
    CDe = X + 600 * N;          // per interval: C (12 x 12), D (12 x 12), e (12)
    Z = CDe + 300 * N;          // per interval: [G g ; P c], 12 x 7 row-major
    total = (Z + 84 * N + 31) / 32 * 32;
  }
};

// Outputs of one BVP from its unknowns Y (eq. optuv at t = 0): lambda(0),
// u(0), V = z(T) + h(x(T)) with z by the Lobatto quadrature of each
// interval, and the mesh values.
__device__ void lob_outputs(const BvpArgs& P, const int N, const double h, const int64_t b,
                            const double* __restrict__ Y, double* __restrict__ lam0, double* __restrict__ u0,
                            double* __restrict__ Vout, double* __restrict__ traj) {
  const int lane = threadIdx.x;
  if (lane < 6) lam0[b * 6 + lane] = Y[6 + lane];
  if (lane < P.m)
    u0[b * P.m + lane] = P.U[lane * 3 + 0] * Y[9] + P.U[lane * 3 + 1] * Y[10] + P.U[lane * 3 + 2] * Y[11];
  if (Vout) {
    double part = 0.0;
    for (int q = lane; q < 3 * N + 1; q += 64) {
      const double* yq = Y + 12 * (int64_t)q;
      double xx = 0.0, uu = 0.0;
      for (int i = 0; i < 6; ++i) xx += yq[i] * yq[i];
      for (int j = 0; j < P.m; ++j) {
        const double u = P.U[j * 3 + 0] * yq[9] + P.U[j * 3 + 1] * yq[10] + P.U[j * 3 + 2] * yq[11];
        uu += u * u;
      }
      const double L = 0.5 * (P.q * xx + P.r * uu);
      // quadrature weight of point q: b_j of its interval(s); a mesh point
      // inside the interval range belongs to two intervals
      const int j = q % 3;
      const double w = q == 0 ? P.lob[3][0]
                       : q == 3 * N ? P.lob[3][3]
                       : j == 0 ? P.lob[3][0] + P.lob[3][3]
                                : P.lob[3][j];
      part += w * L;
    }
    part = wave_sum(part);
    if (lane == 0) {
      const double* yN = Y + 12 * (int64_t)(3 * N);
      double xx = 0.0;
      for (int i = 0; i < 6; ++i) xx += yN[i] * yN[i];
      Vout[b] = h * part + 0.5 * P.pw * xx;
    }
  }
  if (traj) {
    double* out = traj + b * 12 * (int64_t)(N + 1);
    for (int i = lane; i < 12 * (N + 1); i += 64) out[i] = Y[36 * (int64_t)(i / 12) + i % 12];
  }
}

__global__ __launch_bounds__(64) void k_lobatto(BvpArgs P, const double* __restrict__ x0, double* __restrict__ lam0,
                                                double* __restrict__ u0, double* __restrict__ Vout,
                                                double* __restrict__ traj, int32_t* __restrict__ status,
                                                int32_t* __restrict__ iters, double* __restrict__ ws,
                                                const int32_t* __restrict__ order) {
  __shared__ LobShared sh;
  const int64_t b = order ? order[blockIdx.x] : blockIdx.x;
  const int lane = threadIdx.x;
  const int N = P.N;
  const double h = P.h;
  const LobLayout Lw(N);
  double* ws_b = ws + (int64_t)blockIdx.x * P.per_bvp;
  double* Y = ws_b + Lw.Y;
  double* Yt = ws_b + Lw.Yt;
  double* D = ws_b + Lw.D;
  double* F = ws_b + Lw.F;
  double* Phi = ws_b + Lw.Phi;
  double* Jp = ws_b + Lw.Jp;
  double* Xg = ws_b + Lw.X;
  double* CDe = ws_b + Lw.CDe;
  double* Zs = ws_b + Lw.Z;
  const int64_t npt = Lw.npt, ny = Lw.ny;

  if (P.resume && status[b] != SGCM_BVP_CONVERGED) {
    if (P.outputs) lob_outputs(P, N, h, b, ws_b, lam0, u0, Vout, traj);
    return;
  }
  if (lane < 6) sh.xb[lane] = x0[b * 6 + lane];
  int it = -1, st = SGCM_BVP_MAXITER;
  if (P.resume) {
    it = 0;
  } else {
    for (int64_t i = lane; i < ny; i += 64) Y[i] = 0.0;
  }
  wave_mem_sync();

  // the damped iteration of the trapezoidal solver (see bvp.hip)
  bool trial = false, full = false;
  int halvings = 0;
  double t = 1.0, fn0 = 0.0;
  bool lin = it < 0;
  while (true) {
    const bool blend = trial && halvings > 0;
    const double* src = trial ? Yt : Y;
    // ---- Phi and Phi' at every collocation point ----
    for (int64_t q = lane; q < npt; q += 64) {
      double y[12];
      if (blend) {
#pragma unroll
        for (int i = 0; i < 12; ++i) {
          y[i] = fma(t, D[12 * q + i], Y[12 * q + i]);
          Yt[12 * q + i] = y[i];
        }
      } else {
#pragma unroll
        for (int i = 0; i < 12; ++i) y[i] = src[12 * q + i];
      }
      double ph[12], A[36], W[36];
      point_eval(P, y, ph, A, W);
#pragma unroll
      for (int i = 0; i < 12; ++i) Phi[12 * q + i] = ph[i];
      double* jq = Jp + 144 * q;
#pragma unroll
      for (int r = 0; r < 12; ++r)
#pragma unroll
        for (int c = 0; c < 12; ++c) jq[r * 12 + c] = phi_jac(P, A, W, r, c);
    }
    wave_mem_sync();
    // ---- residual F and its max norm ----
    const double* yv = trial ? Yt : Y;  // the point evaluated (blend stored it to Yt)
    double lmax = 0.0;
    int bad = 0;
    for (int k = lane; k < N; k += 64) {
      const double* yk = yv + 36 * (int64_t)k;
      for (int i = 1; i < 4; ++i) {
        const double* zi = yk + 12 * i;
        double* Fi = F + 6 + 12 * (3 * (int64_t)k + i - 1);
#pragma unroll
        for (int r = 0; r < 12; ++r) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < 4; ++j) s = fma(P.lob[i][j], Phi[12 * (3 * (int64_t)k + j) + r], s);
          const double v = zi[r] - yk[r] - h * s;
          Fi[r] = v;
          bad |= !isfinite(v);
          lmax = fmax(lmax, fabs(v));
        }
      }
    }
    if (lane < 6) {
      const double v0 = yv[lane] - sh.xb[lane];
      const double* yN = yv + 12 * (npt - 1);
      const double vN = yN[6 + lane] - P.pw * yN[lane];
      F[lane] = v0;
      F[ny - 6 + lane] = vN;
      bad |= !isfinite(v0) || !isfinite(vN);
      lmax = fmax(lmax, fmax(fabs(v0), fabs(vN)));
    }
    wave_mem_sync();
    const bool nonfinite = __any(bad);
    lmax = wave_max(lmax);
    if (trial) {
      const bool take = full || halvings == P.max_halvings || (!nonfinite && lmax <= (1.0 - kArmijoSigma * t) * fn0);
      if (!take) {
        t *= 0.5;
        ++halvings;
        continue;
      }
      double* y = Y;
      Y = Yt;
      Yt = y;
      ++it;
      trial = false;
    }
    if (it >= 0) {
      if (nonfinite) { st = SGCM_BVP_NONFINITE; break; }
      if (lmax <= P.tol) { st = SGCM_BVP_CONVERGED; break; }
      if (it == P.max_iter) { st = SGCM_BVP_MAXITER; break; }
    }
    fn0 = lmax;
    bool regular = true;

    // ---- (1) condensation of the interior stages, interval by interval ----
    for (int k = 0; k < N && regular; ++k) {
      const double* J0 = Jp + 144 * (3 * (int64_t)k);
      const double* Fk = F + 6 + 36 * (int64_t)k;
      // [M | B1 | B4 | -F_{1,2}], 24 x 49: stage rows i = 1, 2
      // one load and one fma per entry in every lane (no divergent branches,
      // whose loads would each wait in turn): entry = ident + coef J0[off],
      // with ident -0 where there is none (so that it adds nothing, sign of
      // zero included), or -F in the last column
      for (int e = lane; e < 24 * 49; e += 64) {
        const int r = e / 49, c = e - 49 * r;
        const int i = 1 + r / 12, rr = r % 12;
        const int jj = c < 24 ? 1 + c / 12 : (c < 36 ? 0 : 3);  // stage of the Jacobian block
        const int cc = c < 24 ? c % 12 : (c < 36 ? c - 24 : (c < 48 ? c - 36 : 0));
        const double t = h * P.lob[i][jj];
        const double coef = c < 24 ? -t : t;
        const double ident = c < 24 ? (r == c ? 1.0 : 0.0) : (c < 36 ? (rr == cc ? 1.0 : 0.0) : -0.0);
        const double x = fma(coef, J0[144 * jj + rr * 12 + cc], ident);
        const double f = -Fk[12 * (i - 1) + rr];
        sh.A[r * kLd + c] = c < 48 ? x : f;
      }
      lds_handoff();
      regular = wave_gauss_jordan<24, 49>(sh.A);
      double* Xk = Xg + 600 * (int64_t)k;
      for (int e = lane; e < 600; e += 64) Xk[e] = sh.A[(e / 25) * kLd + 24 + e % 25];
      // T = h [a_31 Phi'_1 | a_32 Phi'_2] (12 x 24);
      // C = -(I + h a_30 Phi'_0 + T X1), D = I - h a_33 Phi'_3 - T X4, e = -F_3 + T X0
      double* Ck = CDe + 300 * (int64_t)k;
      for (int e = lane; e < 300; e += 64) {
        const int r = e / 25, col = e - 25 * r;
        double s = 0.0;
        for (int q = 0; q < 24; ++q)
          s = fma(h * P.lob[3][1 + q / 12] * J0[144 * (1 + q / 12) + r * 12 + q % 12], sh.A[q * kLd + 24 + col], s);
        // the three kinds of entry from one selected load (no divergent branches)
        const bool cl = col < 12, dl = !cl && col < 24;
        const int cj = cl ? col : (dl ? col - 12 : 0);
        const double jv = J0[(cl ? 0 : 144 * 3) + r * 12 + cj];
        const double id = r == cj ? 1.0 : 0.0;
        const double cv = -(id + h * P.lob[3][0] * jv + s);
        const double dv = id - h * P.lob[3][3] * jv - s;
        const double ev = -Fk[24 + r] + s;
        Ck[cl ? r * 12 + col : (dl ? 144 + r * 12 + col - 12 : 288 + r)] = cl ? cv : (dl ? dv : ev);
      }
      wave_mem_sync();
      lds_handoff();
    }
    // ---- (2) backward Riccati sweep ----
    if (lane < 36) sh.P[lane] = (lane / 6 == lane % 6) ? P.pw : 0.0;
    if (lane < 6) sh.c[lane] = -F[ny - 6 + lane];
    lds_handoff();
    for (int k = N - 1; k >= 0 && regular; --k) {
      const double* Ck = CDe + 300 * (int64_t)k;
      const double* Dk = Ck + 144;
      const double* ek = Ck + 288;
      // [Dx + Dl P | Cl | -Cx | e - Dl c], 12 x 19
      // one selected load per entry, and one shared sum for the columns
      // that have one (0..5: + Dl P, 18: - Dl c); no four-way branch, whose
      // loads would each wait in turn
      for (int e = lane; e < 12 * 19; e += 64) {
        const int r = e / 19, col = e - 19 * r;
        const bool px = col < 6, ce = col >= 18;
        const int off = px ? 144 + r * 12 + col : (col < 12 ? r * 12 + col : (col < 18 ? r * 12 + col - 12 : 288 + r));
        const double b0 = Ck[off];
        double v = (col >= 12 && col < 18) ? -b0 : b0;
        if (px || ce) {
#pragma unroll
          for (int m = 0; m < 6; ++m) {
            const double dm = Dk[r * 12 + 6 + m];
            v = px ? fma(dm, sh.P[m * 6 + col], v) : fma(-dm, sh.c[m], v);
          }
        }
        sh.A[r * kLd + col] = v;
      }
      lds_handoff();
      regular = wave_gauss_jordan<12, 19>(sh.A);
      // rows 0..5: [G g] (dx_{k+1} = G dx_k + g); rows 6..11: [P c] at k
      double* Zk = Zs + 84 * (int64_t)k;
      for (int e = lane; e < 84; e += 64) Zk[e] = sh.A[(e / 7) * kLd + 12 + e % 7];
      if (lane < 36) sh.P[lane] = sh.A[(6 + lane / 6) * kLd + 12 + lane % 6];
      if (lane < 6) sh.c[lane] = sh.A[(6 + lane) * kLd + 18];
      wave_mem_sync();
      lds_handoff();
    }
    if (!regular) {
      st = SGCM_BVP_SINGULAR;
      if (it < 0) it = 0;
      break;
    }
    // ---- (3) forward pass: the step D and the full-step point Yt = Y + D ----
    // sh.v: [0, 6) dx_k, [6, 12) dlambda_k, [12, 18) dx_{k+1}, [18, 24) dlambda_{k+1}
    if (lane < 6) sh.v[lane] = -F[lane];
    lds_handoff();
    for (int k = 0; k < N; ++k) {
      const double* Zk = Zs + 84 * (int64_t)k;
      if (k == 0 && lane >= 6 && lane < 12) {  // dlambda_0 = P_0 dx_0 + c_0
        double s = Zk[lane * 7 + 6];
        for (int j = 0; j < 6; ++j) s = fma(Zk[lane * 7 + j], sh.v[j], s);
        sh.v[lane] = s;
      }
      lds_handoff();
      if (lane < 6) {  // dx_{k+1} = G_k dx_k + g_k
        double s = Zk[lane * 7 + 6];
        for (int j = 0; j < 6; ++j) s = fma(Zk[lane * 7 + j], sh.v[j], s);
        sh.v[12 + lane] = s;
      }
      lds_handoff();
      if (lane < 6) {  // dlambda_{k+1} = P_{k+1} dx_{k+1} + c_{k+1}, or p_w dx_N - F_N
        double s;
        if (k + 1 < N) {
          const double* Zn = Zs + 84 * (int64_t)(k + 1);
          s = Zn[(6 + lane) * 7 + 6];
          for (int j = 0; j < 6; ++j) s = fma(Zn[(6 + lane) * 7 + j], sh.v[12 + j], s);
        } else {
          s = P.pw * sh.v[12 + lane] - F[ny - 6 + lane];
        }
        sh.v[18 + lane] = s;
      }
      lds_handoff();
      // the interior stages dZ = X1 dy_k + X4 dy_{k+1} + X0, and the step's
      // entries of points 3k (dy_k), 3k + 1, 3k + 2
      const double* Xk = Xg + 600 * (int64_t)k;
      const int64_t base = 36 * (int64_t)k;
      if (lane < 24) {
        double s = Xk[lane * 25 + 24];
        for (int j = 0; j < 12; ++j) s = fma(Xk[lane * 25 + j], sh.v[j], s);
        for (int j = 0; j < 12; ++j) s = fma(Xk[lane * 25 + 12 + j], sh.v[12 + j], s);
        D[base + 12 + lane] = s;
        Yt[base + 12 + lane] = Y[base + 12 + lane] + s;
      } else if (lane < 36) {
        const double d = sh.v[lane - 24];
        D[base + lane - 24] = d;
        Yt[base + lane - 24] = Y[base + lane - 24] + d;
      }
      lds_handoff();
      if (lane < 12) sh.v[lane] = sh.v[12 + lane];  // dy_{k+1} becomes dy_k
      lds_handoff();
    }
    if (lane < 12) {  // dy_N
      const double d = sh.v[lane];
      D[ny - 12 + lane] = d;
      Yt[ny - 12 + lane] = Y[ny - 12 + lane] + d;
    }
    wave_mem_sync();
    trial = true;
    full = lin;
    t = 1.0;
    halvings = 0;
    lin = false;
  }
  if (P.keep && Y != ws_b) {
    for (int64_t i = lane; i < ny; i += 64) ws_b[i] = Y[i];
    wave_mem_sync();
  }
  if (P.outputs) lob_outputs(P, N, h, b, Y, lam0, u0, Vout, traj);
  if (lane == 0) {
    status[b] = st;
    const int n_it = it < 0 ? 0 : it;
    iters[b] = P.resume ? iters[b] + n_it : n_it;
  }
}

}  // namespace

int64_t lobatto_doubles(int64_t N) { return LobLayout(N).total; }

int launch_lobatto(const BvpArgs& a, int64_t n_bvps, const double* x0, double* lambda0, double* u0, double* V,
                   double* traj, int32_t* status, int32_t* iters, double* workspace, const int32_t* order,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_lobatto, dim3((unsigned)n_bvps), dim3(64), 0, s, a, x0, lambda0, u0, V, traj, status, iters,
                     workspace, order);
  return hipGetLastError() == hipSuccess ? SGCM_OK : SGCM_EDEVICE;
}

}  // namespace sgcm

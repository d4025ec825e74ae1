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
// P_N = p_w I, c_N = -F_N, and a forward pass dx_0 = -F_0,
// dx_k = G_k dx_{k-1} + g_k, dlambda_{k-1} = P_{k-1} dx_{k-1} + c_{k-1}.
// With L = (I - a A)^{-1} at each point (two 3 x 3 inverses: the rates do not
// depend on the angles) and, per interval k,
//   K = L_k [I + a A_{k-1} | a e_rates | -r^x_k]   (6 x 10),
//   F = L_{k-1}^T (I + a A_k^T),  H = a L_{k-1}^T W_k,
//   C = H K + [a L_{k-1}^T W_{k-1} | 0 | -L_{k-1}^T r^l_k],
// one sweep step is
//   Q = [P_k | c_k] [K ; e_9],  E = F Q - C,  T = Q + E on the rate rows,
//   (S_w^{-1} + T[:, 6..8]) M = T   (or (I + S_w T[:, 6..8]) M = S_w T),
//   [P_{k-1} | c_{k-1}] = E[:, state] - E[:, 6..8] M,
//   [G_k | g_k] = K[:, state] - K[:, 6..8] M:
// the elimination of dlambda_{k-1} and dx_k from the interval equations.  The
// controls act on the rates only (S has rank <= 3), so the only inverse on the
// serial path is 3 x 3.
//
// Per Newton iteration: (1) the residual pass, one lane per mesh point:
// Phi, the residual and its norm, and the point blocks (nonzeros of A and W,
// L, r_k) stored entry-major in the workspace; (2) the sweep in batches of 8
// intervals from k = N down: the batch's window of point blocks comes to LDS
// by direct global-to-LDS loads (issued a batch ahead), the interval
// constants K, F, H, Gam' are formed lane-parallel, and the serial chain runs
// one lane per entry of the 6 x 10 step with three LDS exchanges per interval;
// the interval solutions [G_k g_k ; P_{k-1} c_{k-1}] go to the workspace;
// (3) the forward pass, 12 rows per 16-lane row with dx broadcast by DPP,
// the interval solutions staged through LDS 12 at a time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <new>
#include <type_traits>
#include <vector>

#include "model.h"
#include "sgcm_internal.h"
#include "trace.h"

namespace sgcm {
namespace {

// s_waitcnt lgkmcnt(n), the other counters left alone (gfx9 encoding: vmcnt
// in bits 3:0 and 15:14, expcnt in 6:4, lgkmcnt in 11:8): with only LDS
// operations in flight, which complete in order, every one but the n most
// recent has completed.  The compiler's own wait insertion takes this wait
// into account and still adds whatever a later use needs, so n sets how long
// the wave waits, never what it reads.
template <int n>
__device__ __forceinline__ void lds_wait_all_but() {
  static_assert(n >= 0 && n < 16, "lgkmcnt has 4 bits");
  __builtin_amdgcn_s_waitcnt(0xC07F | (n << 8));
}

// Value of v in lane J of each 16-lane row, to every lane of that row (DPP
// row_newbcast): no SGPR round trip, the result lands in VGPRs.  gfx950 moves
// a 64-bit value with one row_newbcast (v_mov_b64_dpp).
template <int J>
__device__ __forceinline__ double row_bcast(double v) {
  const long long bits = __builtin_amdgcn_mov_dpp(__double_as_longlong(v), 0x150 + J, 0xf, 0xf, false);
  return __longlong_as_double(bits);
}

template <int J>
__device__ __forceinline__ float row_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + J, 0xf, 0xf, false));
}

typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef float flt2 __attribute__((ext_vector_type(2)));
template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
  using type = dbl2;
};
template <>
struct Vec2<float> {
  using type = flt2;
};

// Hardware reciprocal estimate (refined by the caller).
__device__ __forceinline__ double hw_rcp(double x) { return __builtin_amdgcn_rcp(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// 16 bytes from src (per lane) into LDS at dst + 16 * lane, without passing
// through registers (gfx950 global_load_lds_dwordx4); dst is wave-uniform.
// Completion is tracked by the vector memory counter.
__device__ __forceinline__ void g2lds16(const double* src, double* dst) {
  __builtin_amdgcn_global_load_lds((const void*)src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
}

// LDS strides are skewed so that the lanes of one access fall on distinct
// banks (32 banks of 4 bytes): columns of K and Q 12 banks apart, rows of
// [F | H | Gam'] 12 banks apart; point blocks are entry-major, so lanes that
// read one entry of consecutive points read consecutive words.
constexpr int kKc = 60;            // K = [R | B | rho], column-major, 6 per column
constexpr int kFHr = 22;           // row of F (6), H (6), Gam' (7), pad
constexpr int kCst = kKc + 6 * kFHr + 2;  // per interval, 4 banks apart
constexpr int kZI = 84;            // interval solution [G g ; P c], row-major 12 x 7

// Tile sizes of the solve (a launch-time choice; results do not depend on
// them): NB intervals per sweep batch (the interval constants of a batch are
// formed together, one lane per (interval, row pair)), FC intervals per
// forward-pass chunk (two chunk buffers; even).  Instantiated for NB in
// {8, 10, 12, 16} and FC in {8, 12}.
template <int NB, int FC>
struct Tile {
  static_assert(NB >= 1 && 3 * NB <= 64, "sweep batch");
  static_assert(FC >= 2 && FC % 2 == 0, "forward chunk");
  static constexpr int kNB = NB;
  static constexpr int kFwd = FC;
  static constexpr int kFwdY = 12 * (FC + 1);        // rows of Y a chunk updates
  static constexpr int kFwdBuf = FC * kZI + kFwdY;
};

// Structural zeros of A = df/dx and W at a mesh point (both models): the
// rates do not depend on the angles, yaw does not enter the kinematics, and
// the gyroscopic terms couple distinct rates only.  A point block stores the
// structurally nonzero entries of A (row-major), those of the symmetric W on
// and above the diagonal, L without its zero block L[3..5][0..2] (rows 0..2,
// then columns 3..5 of rows 3..5) and the interval residual r.
__host__ __device__ constexpr bool a_nz(int r, int c) {
  return (r == 0 && c != 2) || (r == 1 && (c == 0 || c >= 4)) || (r == 2 && c != 3 && c != 2) ||
         (r >= 3 && c >= 3 && c != r);
}
__host__ __device__ constexpr bool w_nz(int r, int c) {
  return r == c || ((r == 0 || r == 1) && (c == 0 || c == 1 || c == 4 || c == 5)) ||
         ((c == 0 || c == 1) && (r == 4 || r == 5)) || (r >= 3 && c >= 3);
}
__host__ __device__ constexpr int a_idx(int r, int c) {
  int n = 0;
  for (int e = 0; e < r * 6 + c; ++e) n += a_nz(e / 6, e % 6) ? 1 : 0;
  return n;
}
// slot of W[r][c], r <= c, among the stored entries of W
__host__ __device__ constexpr int w_idx(int r, int c) {
  int n = 0;
  for (int e = 0; e < r * 6 + c; ++e) n += (w_nz(e / 6, e % 6) && e / 6 <= e % 6) ? 1 : 0;
  return n;
}
constexpr int kPbW = a_idx(6, 0);        // W entries start after the 18 of A
constexpr int kPbL = kPbW + w_idx(6, 0);  // L (27) after the 14 of W
constexpr int kPbR = kPbL + 27;           // r (12)
constexpr int kPB = kPbR + 12;            // entries per point block
static_assert(kPbW == 18 && kPbL == 32 && kPB == 71, "point-block layout");
// slot of L[r][c] (r < 3, or r >= 3 and c >= 3) relative to kPbL
__host__ __device__ constexpr int l_slot(int r, int c) { return r < 3 ? r * 6 + c : 18 + (r - 3) * 3 + (c - 3); }
// Entry of A[r][c] and of W[r][c] in a point block (-1: structural zero), as
// tables so that an index known at compile time folds to a constant.
struct PbIndex {
  int a[36], w[36];
};
__host__ __device__ constexpr PbIndex make_pb_index() {
  PbIndex t{};
  for (int e = 0; e < 36; ++e) {
    const int r = e / 6, c = e % 6;
    t.a[e] = a_nz(r, c) ? a_idx(r, c) : -1;
    t.w[e] = w_nz(r, c) ? kPbW + (r <= c ? w_idx(r, c) : w_idx(c, r)) : -1;
  }
  return t;
}
__device__ constexpr PbIndex kPbIdx = make_pb_index();

// Point blocks of a batch in LDS: entry e of point p0 + s at [e][s], kSP
// points per entry (16-byte units, so p0 is a multiple of kU = 16 / sizeof(T)
// and the NB + 1 points klo - 1 .. klo + NB - 1, which start less than kU
// points after p0, always fit).
template <typename T, int NB>
struct PointBlockLayout {
  static constexpr int kU = 16 / (int)sizeof(T);                 // points per 16-byte unit
  static constexpr int kSP = (NB + kU + kU - 1) / kU * kU;       // points per entry in LDS
};

// Points per entry of a BVP's global point-block array: a multiple of 4
// that holds the N + 1 mesh points and every batch's 16-byte-aligned window
// for all instantiated tiles (a window starts at most N - NB and spans kSP
// <= NB + 2 kU - 1 points, so it ends before N + 2 kU <= N + 8).
__host__ __device__ inline int64_t pb_stride(int64_t N) {
  const int64_t n = N + 8 > 16 ? N + 8 : 16;
  return (n + 3) / 4 * 4;
}

// T is the arithmetic type of the Newton linear solve (double, or float for
// the FP32 inexact Newton); the residual pass and the Y rows of the forward
// pass are FP64 in both.
template <typename T, int NB, int FC>
struct __align__(16) SweepShared {
  union {
    struct {
      T pts[kPB * PointBlockLayout<T, NB>::kSP];  // point blocks of one batch, entry-major
      T cst[NB * kCst];                          // interval constants of one batch
    } b;
    double fwd[2 * Tile<NB, FC>::kFwdBuf];  // forward pass: two chunks of [Z | Y rows]
    double pa[2 * 64 * 12];         // residual pass: Phi and y of one 64-point chunk
  } u;
  // chain exchange buffers, one entry per lane: lane 10 i + o holds entry
  // (i, o) of [P | c] (c in column 9), of Q, of T = (Q + E) and of E
  T PL[64];
  T QL[64];
  T TL[64];
  T EL[64];
  double carry_phi[12], carry_y[12];
  double xb[6], F0[6], FN[6];
  double zero[8];
};


// L = (I - a A)^{-1} of one mesh point from its A (row-major 6 x 6), and
// the stored entries of A, W and L (see the point-block layout) as entries
// 0 .. kPbR - 1 of the point's column of a point-block array (entry e at
// dst[e * stride]).  I - a A is block upper triangular (the
// rates do not depend on the angles) with an angle block that has a zero
// column, so L = [[X, X (a E) Y], [0, Y]] from two 3 x 3 inverses, X of the
// angle block and Y of the rate block, E = A[0:3, 3:6].  Returns false when
// either inverse is singular.
template <typename T>
__device__ __forceinline__ bool point_block_store(const double a, const double (&A)[36], const double (&W)[36],
                                                  T* __restrict__ dst, const int64_t stride) {
  double M1[9], M2[9], E[9], Xb[9], Yb[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      M1[i * 3 + j] = (i == j ? 1.0 : 0.0) - a * A[i * 6 + j];
      M2[i * 3 + j] = (i == j ? 1.0 : 0.0) - a * A[(3 + i) * 6 + 3 + j];
      E[i * 3 + j] = A[i * 6 + 3 + j];
    }
  const double d1 = inv3(M1, Xb);
  const double d2 = inv3(M2, Yb);
#pragma unroll
  for (int e = 0; e < 36; ++e) {
    if (kPbIdx.a[e] >= 0) dst[kPbIdx.a[e] * stride] = (T)A[e];
    if (kPbIdx.w[e] >= 0 && e / 6 <= e % 6) dst[kPbIdx.w[e] * stride] = (T)W[e];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double xe[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      xe[j] = a * (Xb[i * 3 + 0] * E[0 * 3 + j] + Xb[i * 3 + 1] * E[1 * 3 + j] + Xb[i * 3 + 2] * E[2 * 3 + j]);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      dst[(kPbL + l_slot(i, j)) * stride] = (T)Xb[i * 3 + j];
      dst[(kPbL + l_slot(i, 3 + j)) * stride] = (T)(xe[0] * Yb[0 * 3 + j] + xe[1] * Yb[1 * 3 + j] + xe[2] * Yb[2 * 3 + j]);
      dst[(kPbL + l_slot(3 + i, 3 + j)) * stride] = (T)Yb[i * 3 + j];
    }
  }
  return d1 != 0.0 && d2 != 0.0;
}

// Outputs of one BVP from its iterate Y (eq. optuv at t = 0): lambda(0),
// u(0) = u*(x0, lambda(0)), V = z(T) + h(x(T)) with z by the trapezoidal rule
// on the mesh, and the trajectory.
__device__ __forceinline__ void bvp_outputs(const BvpArgs& P, const int N, const double h, const int64_t b,
                                            const double* __restrict__ Y, double* __restrict__ lam0,
                                            double* __restrict__ u0, double* __restrict__ Vout,
                                            double* __restrict__ traj) {
  const int lane = threadIdx.x;
  const int NP = N + 1;
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
      Vout[b] = h * part + 0.5 * P.pw * xx;
    }
  }
  if (traj) {
    double* out = traj + b * 12 * (int64_t)NP;
    for (int i = lane; i < 12 * NP; i += 64) out[i] = Y[i];
  }
}

// Whether the first steps of the unit initial states made inside the call
// may be combined (the rule sgcm_plan_create checks on the host); a null
// check stands for a plan that was checked there.
__device__ __forceinline__ bool plan_steps_valid(const int32_t* __restrict__ chk) {
  if (!chk) return true;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 6; ++j)
    ok &= (chk[j] == SGCM_BVP_CONVERGED || chk[j] == SGCM_BVP_MAXITER) && chk[6 + j] == 0;
  return ok;
}

// Newton's method for one BVP (index b, mesh of N intervals of width h,
// workspace ws_b) by one 64-lane workgroup.
template <typename T, int NB, int FC>
__device__ __forceinline__ void newton_bvp(const BvpArgs& P, const int N, const double h, const int64_t b,
                                           const double* __restrict__ y1, double* ws_b,
                                           const double* __restrict__ x0, double* __restrict__ lam0,
                                           double* __restrict__ u0, double* __restrict__ Vout,
                                           double* __restrict__ traj, int32_t* __restrict__ status,
                                           int32_t* __restrict__ iters, SweepShared<T, NB, FC>& sh) {
  using V2 = typename Vec2<T>::type;
  constexpr int kNB = Tile<NB, FC>::kNB, kFwd = Tile<NB, FC>::kFwd;
  constexpr int kFwdY = Tile<NB, FC>::kFwdY, kFwdBuf = Tile<NB, FC>::kFwdBuf;
  const int lane0 = threadIdx.x;
  const int lane = lane0;
  const int NP = N + 1;
  const double alpha = 0.5 * h;
  const T at = (T)alpha;
  // two NP x 12 buffers: the iterate Y and the trial point Yt (swapped when a
  // trial is taken)
  double* Y = ws_b;
  double* Yt = ws_b + 12 * (int64_t)NP;
  double* R = ws_b + 24 * (int64_t)NP;  // 16: F_0 (6), F_N (6), pad
  T* Zg = reinterpret_cast<T*>(R + 16);  // N x 84: interval solutions, 12 x 7 rows
  // point blocks [A | W | L | r_k] of every mesh point, entry-major: entry e
  // of point k at PBg[e * pbs + k]
  T* PBg = reinterpret_cast<T*>(R + 16 + (int64_t)kZI * N);
  const int64_t pbs = pb_stride(N);

  if (P.resume && status[b] != SGCM_BVP_CONVERGED) {
    // an earlier continuation stage failed: that status stands, and the last
    // stage writes the outputs of the iterate it left
    if (P.outputs) bvp_outputs(P, N, h, b, ws_b, lam0, u0, Vout, traj);
    return;
  }
  if (lane < 6) sh.xb[lane] = x0[b * 6 + lane];
  if (lane < 8) sh.zero[lane] = 0.0;
  // it = -1: the first Newton step from Y = 0 (the discrete LQR guess) is
  // still to be taken.  At Y = 0 the residual is [-xbar; 0; 0] and the
  // Jacobian does not depend on xbar, so that step is linear in xbar; with a
  // plan it is the combination of the plan's steps for the unit initial
  // states, and the loop starts with its test (it = 0).  A resumed stage
  // starts from the iterate in the workspace with its test.
  int it = -1, st = SGCM_BVP_MAXITER;
  if (P.resume) {
    it = 0;
  } else if (y1 && plan_steps_valid(P.y1_check)) {
    double xb[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) xb[j] = x0[b * 6 + j];
    const int64_t n12 = 12 * (int64_t)NP;
#pragma unroll 4
    for (int64_t i = lane; i < n12; i += 64) {
      double y = xb[0] * y1[i];
#pragma unroll
      for (int j = 1; j < 6; ++j) y = fma(xb[j], y1[j * n12 + i], y);
      Y[i] = y;
    }
    it = 0;
  } else {
    for (int i = lane; i < 12 * NP; i += 64) Y[i] = 0.0;
  }
  wave_mem_sync();

  // Damping of the counted steps: after a linear solve the forward pass has
  // written the full-step point Yt = Y + d; the residual pass then evaluates
  // the trial point Y + t d (t = 1: Yt as written; each halving of t moves Yt
  // halfway back to Y in place, Yt <- Y + (Yt - Y) / 2, which is Y + t d up to
  // rounding), which is taken when its residual is finite and
  // max|F| <= (1 - sigma t) max|F(Y)|, or when it is the last allowed trial
  // (t = 2^-H); else t is halved.  The first step from Y = 0 (the initial
  // guess) is taken in full.
  bool trial = false;  // the pass evaluates a trial point
  bool full = false;   // ... that is taken without a test (the first step)
  int halvings = 0;    // trials rejected so far in this step
  double t = 1.0, fn0 = 0.0;
  bool lin = it < 0;   // the pass at Y = 0 before the first (linearised) step
  while (true) {
    // ---- residual F and its max norm at the pass's point (lane-parallel
    //      over mesh points) ----
    double lmax = 0.0;
    int bad = 0;
    bool regular = true;
    const bool blend = trial && halvings > 0;  // the point is Y + t d, formed here from Yt
    const double* src = trial ? Yt : Y;
    // In the first (linearised) step Y = 0, and the sweep forms its interval
    // constants from the first batch alone (every interval has the same
    // ones).  The pass then covers only the last 64 points, which hold that
    // batch's window of point blocks, and sets F_0 = 0 - xbar and
    // F_N = 0 - p_w 0 directly (the values the pass would compute); nothing
    // is tested in that step.
    int base0 = 0;
    if (lin && NP > 64) {
      base0 = NP - 64;
      if (lane < 6) {
        R[lane] = 0.0 - sh.xb[lane];
        R[6 + lane] = 0.0 - P.pw * 0.0;
      }
    }
    for (int base = base0; base < NP; base += 64) {
      const int lane = opaque_lane(lane0);
      const int k = base + lane;
      const bool valid = k < NP;
      double yk[12], ph[12];
      if (valid) {
        if (blend) {
#pragma unroll
          for (int i = 0; i < 12; ++i) {
            const double y0 = Y[12 * (int64_t)k + i];
            yk[i] = fma(0.5, Yt[12 * (int64_t)k + i] - y0, y0);
            Yt[12 * (int64_t)k + i] = yk[i];
          }
        } else {
#pragma unroll
          for (int i = 0; i < 12; ++i) yk[i] = src[12 * (int64_t)k + i];
        }
        double A[36], W[36];
        point_eval(P, yk, ph, A, W);
        regular &= point_block_store(alpha, A, W, PBg + k, pbs);
#pragma unroll
        for (int i = 0; i < 12; ++i) {
          sh.u.pa[lane * 12 + i] = ph[i];
          sh.u.pa[768 + lane * 12 + i] = yk[i];
        }
      }
      lds_handoff();
      if (valid) {
        if (k == 0) {
#pragma unroll
          for (int i = 0; i < 6; ++i) {
            const double v = yk[i] - sh.xb[i];
            R[i] = v;
            bad |= !isfinite(v);
            lmax = fmax(lmax, fabs(v));
          }
#pragma unroll
          for (int i = 0; i < 12; ++i) PBg[(kPbR + i) * pbs] = T(0);  // point 0 has no interval
        } else {
          const double* pp = lane > 0 ? &sh.u.pa[(lane - 1) * 12] : sh.carry_phi;
          const double* yp = lane > 0 ? &sh.u.pa[768 + (lane - 1) * 12] : sh.carry_y;
#pragma unroll
          for (int i = 0; i < 12; ++i) {
            const double v = yk[i] - yp[i] - alpha * (pp[i] + ph[i]);
            PBg[(kPbR + i) * pbs + k] = (T)v;
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
      lds_handoff();
      if (lane == 63 && valid) {
#pragma unroll
        for (int i = 0; i < 12; ++i) {
          sh.carry_phi[i] = ph[i];
          sh.carry_y[i] = yk[i];
        }
      }
      lds_handoff();
    }
    wave_mem_sync();  // residuals and point blocks visible to every lane
    const bool nonfinite = __any(bad);
    const bool singular_point = __any(!regular);
    lmax = wave_max(lmax);
    if (trial) {
      const bool take = full || halvings == P.max_halvings || (!nonfinite && lmax <= (1.0 - kArmijoSigma * t) * fn0);
      if (!take) {
        t *= 0.5;
        ++halvings;
        continue;
      }
      double* y = Y;  // the trial point becomes the iterate
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
    if (singular_point) {  // I - a A is singular at a mesh point
      st = SGCM_BVP_SINGULAR;
      if (it < 0) it = 0;
      break;
    }
    fn0 = lmax;

    // ---- backward Riccati sweep, batches of kNB intervals from k = N down ----
    if (lane < 6) {
      sh.F0[lane] = R[lane];
      sh.FN[lane] = R[6 + lane];
    }
    lds_handoff();
    // chain state: lane (i, o), o in 0..5 and 9, holds [P_k | c_k][i][o];
    // P_N = p_w I, c_N = -F_N
    T pv;
    {
      const int l = opaque_lane(lane0);
      const int i = l < 60 ? l / 10 : 5, o = l < 60 ? l - 10 * i : 0;
      pv = (T)((o < 6) ? (o == i ? P.pw : 0.0) : -sh.FN[i]);
    }
    // point blocks of the window of kSP points from p0 = (lo - 1) rounded
    // down to a 16-byte unit (it covers points lo - 1 .. lo + kNB - 1) into LDS,
    // entry-major, by direct global-to-LDS loads: 16-byte unit u of the
    // window (entry u / (kSP / kU), part u % (kSP / kU)) to LDS unit u
    constexpr int kU = PointBlockLayout<T, NB>::kU, kSP = PointBlockLayout<T, NB>::kSP;
    auto load_points = [&](int lo) {
      const int l = opaque_lane(lane0);
      const int64_t p0 = (lo - 1) / kU * kU;
      constexpr int upe = kSP / kU, units = kPB * upe;
      double* dst = reinterpret_cast<double*>(sh.u.b.pts);
#pragma unroll
      for (int j = 0; j < (units + 63) / 64; ++j) {
        const int u = 64 * j + l;
        if (u < units) {
          const int e = u / upe, q = u - e * upe;
          g2lds16(reinterpret_cast<const double*>(PBg + e * pbs + p0 + q * kU), dst + 128 * j);
        }
      }
    };
    int khi = N;
    int klo = khi - (kNB - 1) < 1 ? 1 : khi - (kNB - 1);
    load_points(klo);
    bool singular = false;
    while (true) {
      const int nb = khi - klo + 1;
      // In the first (linearised) step Y = 0: every mesh point has the same
      // y, trigonometric factors and interval residual (zero), so every
      // interval has the same constants.  They are formed in the first batch
      // and the later batches reuse them from LDS.
      const bool reuse = lin && khi != N;
      if (!reuse) {
        wave_mem_sync();  // the point blocks of points klo - 1 .. khi have landed
        lds_handoff();
        const int p0b = (klo - 1) / kU * kU;
        // interval constants of interval k = khi - tl, lane (tl, rows i and i + 3):
        // rows of K = L_k [I + a A_{k-1} | a e_rates | -r^x], F = L_{k-1}^T (I + a A_k^T),
        // H = a L_{k-1}^T W_k, Gam = a L_{k-1}^T W_{k-1} and -D^{-1} r^l = -L_{k-1}^T r^l.
        // Every LDS access is an immediate offset from a per-lane base.  Terms
        // with a structural zero are skipped at compile time: those of A and
        // W, and L[3..5][0..2] = 0 (row i + 3 of L_k, column i of L_{k-1}).
        {
          const unsigned l = (unsigned)opaque_lane(lane0);
          const int tl = (int)(l % kNB), ip = (int)(l / kNB);
          if (ip < 3 && tl < nb) {
            const int k = khi - tl;
            const T* pa = sh.u.b.pts + (k - 1 - p0b);  // point k - 1: entry e at pa[e * kSP]
            const T* pb = pa + 1;                      // point k
            T* cst = sh.u.b.cst + tl * kCst;
            T lb[2][6], la[2][6];  // rows i, i + 3 of L_k and of L_{k-1}^T
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
              for (int m = 0; m < 6; ++m) {
                // L_k[ip + 3h][m] and L_{k-1}[m][ip + 3h]; the slot is linear
                // in ip (row ip: ip * 6 + m; row 3 + ip: 18 + ip * 3 + m - 3;
                // column ip + 3h of row m < 3: m * 6 + 3h + ip; of row m >= 3:
                // 18 + (m - 3) * 3 + ip)
                lb[h][m] = (h == 1 && m < 3) ? T(0)
                           : pb[(kPbL + (h == 0 ? ip * 6 + m : 18 + ip * 3 + m - 3)) * kSP];
                la[h][m] = (h == 0 && m >= 3) ? T(0)
                           : pa[(kPbL + (m < 3 ? m * 6 + 3 * h + ip : 18 + (m - 3) * 3 + ip)) * kSP];
              }
            T* kc = cst + ip;              // K[i][o] at kc[o * 6 + 3 h]
            T* fh = cst + kKc + ip * kFHr;  // row i of [F | H | Gam'] at fh[3 h kFHr + j]
#pragma unroll
            for (int o = 0; o < 6; ++o) {
              T v[6];
#pragma unroll
              for (int m = 0; m < 6; ++m) v[m] = kPbIdx.a[m * 6 + o] >= 0 ? pa[kPbIdx.a[m * 6 + o] * kSP] : T(0);  // A_{k-1}[m][o]
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                T q = T(0);
#pragma unroll
                for (int m = 0; m < 6; ++m)
                  if (kPbIdx.a[m * 6 + o] >= 0 && !(h == 1 && m < 3)) q = fma(lb[h][m], v[m], q);
                kc[o * 6 + 3 * h] = fma(at, q, lb[h][o]);
              }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
              for (int c = 0; c < 3; ++c) kc[(6 + c) * 6 + 3 * h] = at * lb[h][3 + c];
            {
              T v[6];
#pragma unroll
              for (int m = 0; m < 6; ++m) v[m] = pb[(kPbR + m) * kSP];
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                T q = T(0);
#pragma unroll
                for (int m = 0; m < 6; ++m)
                  if (!(h == 1 && m < 3)) q = fma(lb[h][m], v[m], q);
                kc[54 + 3 * h] = -q;
              }
            }
#pragma unroll
            for (int j = 0; j < 6; ++j) {
              T vf[6], vh[6], vg[6];
#pragma unroll
              for (int m = 0; m < 6; ++m) {
                const int ia = kPbIdx.a[j * 6 + m], iw = kPbIdx.w[m * 6 + j];
                vf[m] = ia >= 0 ? pb[ia * kSP] : T(0);  // A_k[j][m]
                vh[m] = iw >= 0 ? pb[iw * kSP] : T(0);  // W_k[m][j]
                vg[m] = iw >= 0 ? pa[iw * kSP] : T(0);  // W_{k-1}[m][j]
              }
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                T qf = T(0), qh = T(0), qg = T(0);
#pragma unroll
                for (int m = 0; m < 6; ++m) {
                  if (h == 0 && m >= 3) continue;
                  if (kPbIdx.a[j * 6 + m] >= 0) qf = fma(la[h][m], vf[m], qf);
                  if (kPbIdx.w[m * 6 + j] >= 0) {
                    qh = fma(la[h][m], vh[m], qh);
                    qg = fma(la[h][m], vg[m], qg);
                  }
                }
                fh[3 * h * kFHr + j] = fma(at, qf, la[h][j]);
                fh[3 * h * kFHr + 6 + j] = at * qh;
                fh[3 * h * kFHr + 12 + j] = at * qg;
              }
            }
            {
              T v[6];
#pragma unroll
              for (int m = 0; m < 6; ++m) v[m] = pb[(kPbR + 6 + m) * kSP];
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                T q = T(0);
#pragma unroll
                for (int m = 0; m < 6; ++m)
                  if (!(h == 0 && m >= 3)) q = fma(la[h][m], v[m], q);
                fh[3 * h * kFHr + 18] = -q;
              }
            }
          }
        }
        lds_handoff();
      }  // !reuse
      // inputs of the next batch, in flight during the chain
      const int nhi = klo - 1;
      const int nlo = nhi - (kNB - 1) < 1 ? 1 : nhi - (kNB - 1);
      if (nhi >= 1 && !lin) load_points(nlo);
      // the serial chain: three LDS exchanges per interval.  Lane (i, o),
      // 60 lanes, owns entry (i, o) of the step; columns o = 0..5 (R), 6..8
      // (B) and 9 (rho) of [K ; e_9]; the state columns 0..5 and 9 carry
      // [P | c] (slot 6 for column 9).  The constants of interval t + 1 are
      // read while interval t finishes.
      int ci, co, cs;
      bool cv, cst_lane;
      {
        const int l = opaque_lane(lane0);
        cv = l < 60;
        ci = cv ? l / 10 : 5;
        co = cv ? l - 10 * ci : 0;
        cst_lane = cv && (co < 6 || co == 9);
        cs = co < 6 ? co : 6;
      }
      T kcol[6], fh[12], kb[3], gam, kio;
      auto load_consts = [&](int t) {
        const T* cst = sh.u.b.cst + t * kCst;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const V2 v = *reinterpret_cast<const V2*>(&cst[co * 6 + 2 * q]);
          kcol[2 * q] = v.x;
          kcol[2 * q + 1] = v.y;
        }
        const T* fr = cst + kKc + ci * kFHr;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const V2 v = *reinterpret_cast<const V2*>(&fr[2 * q]);
          fh[2 * q] = v.x;
          fh[2 * q + 1] = v.y;
        }
        gam = fr[12 + cs];  // selected where it is used, so that no wait follows the read
        kio = cst[co * 6 + ci];
#pragma unroll
        for (int a = 0; a < 3; ++a) kb[a] = cst[(6 + a) * 6 + ci];
      };
      // Z = S_w^{-1} + T[3..5][6..8] is formed before exchange 3 by the lanes
      // that hold those entries of T (lane (3 + a, 6 + c) adds S_w^{-1}[a][c]),
      // so that it arrives ready; no other lane reads those entries
      T zadd = T(0);
#pragma unroll
      for (int e2 = 0; e2 < 9; ++e2)
        if (P.sinv && ci == 3 + e2 / 3 && co == 6 + e2 % 3) zadd = (T)P.Si[e2];
      asm volatile("" : "+v"(zadd));
      // this lane's entries of the interval solutions, (G_k | g_k) row ci and
      // (P_{k-1} | c_{k-1}) row 6 + ci, column cs, from k = khi down
      T* zrow = Zg + (int64_t)(khi - 1) * kZI + ci * 7 + cs;
      load_consts(0);
      for (int t = 0; t < nb; ++t) {
        // exchange 1: rows of [P_k | c_k].  Every exchange writes one entry
        // per lane, unconditionally, so that no LDS access sits under a
        // branch and each read waits only for its own exchange.
        sh.PL[lane0] = pv;
        lds_handoff();
        T prow[7];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const V2 v = *reinterpret_cast<const V2*>(&sh.PL[ci * 10 + 2 * q]);
          prow[2 * q] = v.x;
          prow[2 * q + 1] = v.y;
        }
        prow[6] = sh.PL[ci * 10 + 9];
        // Q = [P | c] [K ; e_9],  C = H K + [Gam | 0 | -D^{-1} r^l]
        T q = co == 9 ? prow[6] : T(0);
        T cc = cst_lane ? gam : T(0);
#pragma unroll
        for (int m = 0; m < 6; ++m) {
          q = fma(prow[m], kcol[m], q);
          cc = fma(fh[6 + m], kcol[m], cc);
        }
        // exchange 2: columns of Q
        sh.QL[lane0] = q;
        lds_handoff();
        T qcol[6];
#pragma unroll
        for (int r = 0; r < 6; ++r) qcol[r] = sh.QL[r * 10 + co];
        T e = -cc;
#pragma unroll
        for (int m = 0; m < 6; ++m) e = fma(fh[m], qcol[m], e);
        const T tv = q + e;  // T = Psi_w [K ; e_9] on the rate rows
        const T kio_t = kio, kb0 = kb[0], kb1 = kb[1], kb2 = kb[2];
        // exchange 3: column o of T's rate rows, row i of E[:, 6..8], and
        // T[3..5][6..8] (the same for every lane; it arrives as
        // S_w^{-1} + T[3..5][6..8] when S_w is invertible)
        sh.TL[lane0] = tv + zadd;
        sh.EL[lane0] = e;
        lds_handoff();
        T tc[3], er[3], t1[9];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          tc[a] = sh.TL[(3 + a) * 10 + co];
          er[a] = sh.EL[ci * 10 + 6 + a];
#pragma unroll
          for (int c = 0; c < 3; ++c) t1[a * 3 + c] = sh.TL[(3 + a) * 10 + 6 + c];
        }
        // the next interval's constants (this interval's are all in registers
        // by now), issued behind the exchange reads; the wait below covers
        // only the exchange, so they arrive during the 3 x 3 solve.  The
        // constants take 13 LDS reads in FP64 and 9 in FP32 as compiled; the
        // last interval of a batch reads its own again, so that the reads are
        // not under a branch
        __builtin_amdgcn_sched_barrier(0);
        load_consts(t + 1 < nb ? t + 1 : t);
        lds_wait_all_but<sizeof(T) == 8 ? 13 : 9>();
        // the 3 x 3 system Z M = W: Z = S_w^{-1} + T[:, 6..8] (as exchanged),
        // W = T when S_w is invertible, else Z = I + S_w T[:, 6..8],
        // W = S_w T; M by the adjugate of Z
        T z[9], w[3];
        if (P.sinv) {
#pragma unroll
          for (int e2 = 0; e2 < 9; ++e2) z[e2] = t1[e2];
#pragma unroll
          for (int a = 0; a < 3; ++a) w[a] = tc[a];
        } else {
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              T s = (a == c) ? T(1) : T(0);
#pragma unroll
              for (int m = 0; m < 3; ++m) s = fma((T)P.Sw[a * 3 + m], t1[m * 3 + c], s);
              z[a * 3 + c] = s;
            }
#pragma unroll
          for (int a = 0; a < 3; ++a)
            w[a] = fma((T)P.Sw[a * 3 + 0], tc[0], fma((T)P.Sw[a * 3 + 1], tc[1], (T)P.Sw[a * 3 + 2] * tc[2]));
        }
        const T j00 = z[4] * z[8] - z[5] * z[7], j01 = z[2] * z[7] - z[1] * z[8], j02 = z[1] * z[5] - z[2] * z[4];
        const T j10 = z[5] * z[6] - z[3] * z[8], j11 = z[0] * z[8] - z[2] * z[6], j12 = z[2] * z[3] - z[0] * z[5];
        const T j20 = z[3] * z[7] - z[4] * z[6], j21 = z[1] * z[6] - z[0] * z[7], j22 = z[0] * z[4] - z[1] * z[3];
        const T det = z[0] * j00 + z[1] * j10 + z[2] * j20;
        if (det == 0.0) singular = true;
        // 1/det: the hardware reciprocal (relative error below 5e-8 for FP64
        // on gfx950) refined by one Newton step (about 2e-15); det is O(1)
        // here, so no scaling is needed
        T rd = hw_rcp(det);
        rd = fma(rd, fma(-det, rd, T(1)), rd);
        // y = adj(Z) W[:, o]; [M | m][:, o] = y / det
        const T y0 = fma(j00, w[0], fma(j01, w[1], j02 * w[2]));
        const T y1 = fma(j10, w[0], fma(j11, w[1], j12 * w[2]));
        const T y2 = fma(j20, w[0], fma(j21, w[1], j22 * w[2]));
        // P_{k-1} = E - E[:, 6..8] M, c_{k-1} = E[:, 9] - E[:, 6..8] m,
        // G_k = K - B_k M, g_k = rho - B_k m
        const T pn = fma(-rd, fma(er[0], y0, fma(er[1], y1, er[2] * y2)), e);
        const T gn = fma(-rd, fma(kb0, y0, fma(kb1, y1, kb2 * y2)), kio_t);
        if (cst_lane) {
          zrow[0] = gn;
          zrow[6 * 7] = pn;
        }
        zrow -= kZI;
        pv = pn;
      }
      // a zero determinant makes the rest of the batch non-finite; the
      // sweep stops after the batch
      singular = __any(singular);
      if (singular || nhi < 1) break;
      khi = nhi;
      klo = nlo;
    }
    if (singular) {
      st = SGCM_BVP_SINGULAR;
      if (it < 0) it = 0;
      break;
    }

    // ---- forward pass dx_0 = -F_0, dx_k = G_k dx_{k-1} + g_k,
    //      dlambda_{k-1} = P_{k-1} dx_{k-1} + c_{k-1}, dlambda_N = p_w dx_N - F_N;
    //      the full-step point Y + d goes to Yt ----
    wave_mem_sync();  // interval solutions visible to every lane
    T dx[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) dx[j] = (T)(-sh.F0[j]);
    if (lane < 6) Yt[lane] = Y[lane] + (double)dx[lane < 6 ? lane : 0];
    // chunk [c0, c0 + kFwd) of interval solutions and Y rows c0 - 1 .. c0 + kFwd - 1
    // into buffer bf, direct to LDS
    auto fwd_load = [&](int c0, int bf) {
      const int l = opaque_lane(lane0);
      const int nk = (N - c0 + 1) < kFwd ? (N - c0 + 1) : kFwd;
      double* zb = sh.u.fwd + bf * kFwdBuf;
      // the interval solutions (T) move as 16-byte units
      const double* zs = reinterpret_cast<const double*>(Zg + (int64_t)(c0 - 1) * kZI);
      const int units = nk * kZI * (int)sizeof(T) / 16;
#pragma unroll
      for (int j = 0; j < (kFwd * kZI + 127) / 128; ++j)
        if (64 * j + l < units) g2lds16(zs + 128 * j + 2 * l, zb + 128 * j);
      const double* ys = Y + 12 * (int64_t)(c0 - 1);
#pragma unroll
      for (int j = 0; j < (kFwdY + 127) / 128; ++j)
        if (64 * j + l < 6 * (nk + 1)) g2lds16(ys + 128 * j + 2 * l, zb + kFwd * kZI + 128 * j);
    };
    fwd_load(1, 0);
    int bf = 0;
    for (int c0 = 1; c0 <= N; c0 += kFwd) {
      wave_mem_sync();  // this chunk has landed
      if (c0 + kFwd <= N) fwd_load(c0 + kFwd, bf ^ 1);
      const int l = opaque_lane(lane0);
      // lane r = min(l mod 16, 11) of every 16-lane row owns row r: dx_k
      // (r < 6) or dlambda_{k-1} (r >= 6).  The four rows compute the same
      // values, so the broadcast of dx stays inside a row and every lane may
      // store (lanes with equal r store equal values to the same address).
      const int r = (l & 15) < 12 ? (l & 15) : 11;
      const double* zb = sh.u.fwd + bf * kFwdBuf;
      const T* zt = reinterpret_cast<const T*>(zb);
      const int yo = kFwd * kZI + (r < 6 ? 12 : 0) + r;
      const int nk = (N - c0 + 1) < kFwd ? (N - c0 + 1) : kFwd;
      const int64_t row = 12 * (int64_t)(r < 6 ? c0 : c0 - 1) + r;
      double* ytrow = Yt + row;
      // step s: row r of [G_k g_k ; P_{k-1} c_{k-1}] (z) and the Y entry
      // (yv) come from the chunk buffer
      auto fload = [&](int s, T (&z)[7], double& yv) {
#pragma unroll
        for (int j = 0; j < 7; ++j) z[j] = zt[s * kZI + r * 7 + j];
        yv = zb[yo + 12 * s];
      };
      auto fstep = [&](int s, const T (&z)[7], const double yv) {
        // two partial sums: a dependent depth of four instead of six
        const T va = fma(z[2], dx[2], fma(z[1], dx[1], fma(z[0], dx[0], z[6])));
        const T vb = fma(z[5], dx[5], fma(z[4], dx[4], z[3] * dx[3]));
        const T v = va + vb;
        ytrow[12 * s] = yv + (double)v;
        dx[0] = row_bcast<0>(v);
        dx[1] = row_bcast<1>(v);
        dx[2] = row_bcast<2>(v);
        dx[3] = row_bcast<3>(v);
        dx[4] = row_bcast<4>(v);
        dx[5] = row_bcast<5>(v);
      };
      if (nk == kFwd) {
        // a full chunk, unrolled, with the reads of step s + 1 in flight
        // while step s computes.  The compiler's LDS waits here cover every
        // read in flight, so each buffer is pinned (an empty asm that uses
        // it, with a memory clobber) before the next reads are issued: the
        // wait then falls on that buffer alone.  Scheduling barriers keep
        // each step's arithmetic between the next reads and the next pin.
        auto pin = [&](T (&z)[7], double& yv) {
#pragma unroll
          for (int j = 0; j < 7; ++j) asm volatile("" : "+v"(z[j]) : : "memory");
          asm volatile("" : "+v"(yv) : : "memory");
        };
        T za[7], zc[7];
        double ya, yc;
        fload(0, za, ya);
#pragma unroll
        for (int s = 0; s < kFwd; s += 2) {
          pin(za, ya);
          fload(s + 1, zc, yc);
          __builtin_amdgcn_sched_barrier(0);
          fstep(s, za, ya);
          __builtin_amdgcn_sched_barrier(0);
          pin(zc, yc);
          if (s + 2 < kFwd) fload(s + 2, za, ya);
          __builtin_amdgcn_sched_barrier(0);
          fstep(s + 1, zc, yc);
          __builtin_amdgcn_sched_barrier(0);
        }
      } else {
        for (int s = 0; s < nk; ++s) {
          T z[7];
          double yv;
          fload(s, z, yv);
          fstep(s, z, yv);
        }
      }
      bf ^= 1;
    }
    if (lane >= 6 && lane < 12) {
      const int i = lane - 6;
      double d = -sh.FN[i];
#pragma unroll
      for (int j = 0; j < 6; ++j) d = fma(j == i ? P.pw : 0.0, (double)dx[j], d);
      Yt[12 * (int64_t)N + 6 + i] = Y[12 * (int64_t)N + 6 + i] + d;
    }
    wave_mem_sync();
    // the trial of the full step; the first step is taken without a test
    trial = true;
    full = lin;
    t = 1.0;
    halvings = 0;
    lin = false;
  }
  if (P.keep && Y != ws_b) {  // the next continuation stage resumes from the first buffer
    for (int i = lane; i < 12 * NP; i += 64) ws_b[i] = Y[i];
    wave_mem_sync();
  }
  if (P.outputs) bvp_outputs(P, N, h, b, Y, lam0, u0, Vout, traj);
  if (lane == 0) {
    status[b] = st;
    const int n_it = it < 0 ? 0 : it;
    iters[b] = P.resume ? iters[b] + n_it : n_it;
  }
}

template <typename T, int NB, int FC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_newton(
    BvpArgs P, const double* __restrict__ x0, double* __restrict__ lam0, double* __restrict__ u0,
    double* __restrict__ Vout, double* __restrict__ traj, int32_t* __restrict__ status,
    int32_t* __restrict__ iters, double* __restrict__ ws, const int32_t* __restrict__ order) {
  __shared__ SweepShared<T, NB, FC> sh;
  // the workspace is scratch: workgroup g uses slot g whatever BVP it takes,
  // so that consecutive workgroups keep consecutive memory
  const int64_t b = order ? order[blockIdx.x] : blockIdx.x;
  newton_bvp<T, NB, FC>(P, P.N, P.h, b, P.y1, ws + (int64_t)blockIdx.x * P.per_bvp, x0, lam0, u0, Vout, traj,
                        status, iters, sh);
}

// The order in which the workgroups of one launch take the BVPs: decreasing
// |x0|_1.  The Newton iterations a BVP needs grow with the size of its
// initial state (the nonlinear terms grow with it), and the launch ends with
// its longest BVPs, so those start first and the short ones fill the compute
// units behind them (the longest-first rule of the batch plans).  Any order
// gives the same results, so an approximate one does: a one-pass bucket sort
// of the keys into 256 buckets of equal width below the largest key (LDS
// atomics; the order inside a bucket is arbitrary).  A non-finite key counts
// as 0 (such a BVP stops at its first residual test).  n <= kOrderMax.
constexpr int kOrderMax = 4096;
__global__ __launch_bounds__(1024) void k_order(const double* __restrict__ x0, int n, int32_t* __restrict__ order) {
  __shared__ float key[kOrderMax];
  __shared__ float wmax[16];
  __shared__ int32_t cnt[256];
  const int t = threadIdx.x;
  float m = 0.0f;
  for (int i = t; i < n; i += 1024) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) s += fabs(x0[(int64_t)i * 6 + j]);
    const float f = (float)s;
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
  auto bucket = [&](int i) { return 255 - min(255, (int)(key[i] * scale)); };  // largest keys in bucket 0
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

// Bytes of the launch order behind the BVP workspaces.
size_t order_bytes(int64_t n_bvps) { return n_bvps <= kOrderMax ? ((size_t)n_bvps * 4 + 255) / 256 * 256 : 0; }

// A batch of BVPs with per-BVP mesh size and horizon.  Plain mode: workgroup
// g solves BVP order[g].  Persistent mode: each workgroup takes the next
// position of the schedule from a device counter until the batch is done.
struct BatchArgs {
  const int32_t* N;      // per BVP: mesh intervals
  const double* h;       // per BVP: mesh width T / N
  const int64_t* off;    // per BVP: workspace offset in doubles
  const double* y1;      // first Newton steps of the unit initial states of each (N, T) group
  const int64_t* y1off;  // per BVP: offset of its group's steps in y1, or -1 (no plan)
  const int32_t* order;  // schedule: BVP index at each position
  int32_t* counter;      // persistent mode: next schedule position
  int64_t n;
  int persistent;
};

// The next position of the batch order for this workgroup, taken by lane 0
// with a device-scope atomic and made uniform in a scalar register, so that
// it costs no vector register across the Newton solve.
__device__ __forceinline__ int64_t next_position(int32_t* counter) {
  int v = 0;
  if (threadIdx.x == 0) v = atomicAdd(counter, 1);
  return __builtin_amdgcn_readfirstlane(v);
}

template <typename T, int NB, int FC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_newton_batch(
    BvpArgs P, BatchArgs B, const double* __restrict__ x0, double* __restrict__ lam0, double* __restrict__ u0,
    double* __restrict__ Vout, int32_t* __restrict__ status, int32_t* __restrict__ iters,
    double* __restrict__ ws) {
  __shared__ SweepShared<T, NB, FC> sh;
  int64_t pos = B.persistent ? next_position(B.counter) : (int64_t)blockIdx.x;
  while (pos < B.n) {
    const int64_t j = B.order[pos];
    const int64_t yo = B.y1off[j];
    newton_bvp<T, NB, FC>(P, B.N[j], B.h[j], j, yo >= 0 ? B.y1 + yo : nullptr, ws + B.off[j], x0, lam0, u0,
                          Vout, nullptr, status, iters, sh);
    if (!B.persistent) break;
    pos = next_position(B.counter);
  }
}

// One workgroup per BVP in plan order (the form without a slot loop, which
// keeps the registers of the loop out of the Newton solve).
template <typename T, int NB, int FC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_newton_batch_grid(
    BvpArgs P, BatchArgs B, const double* __restrict__ x0, double* __restrict__ lam0, double* __restrict__ u0,
    double* __restrict__ Vout, int32_t* __restrict__ status, int32_t* __restrict__ iters,
    double* __restrict__ ws) {
  __shared__ SweepShared<T, NB, FC> sh;
  const int64_t j = B.order[blockIdx.x];
  const int64_t yo = B.y1off[j];
  newton_bvp<T, NB, FC>(P, B.N[j], B.h[j], j, yo >= 0 ? B.y1 + yo : nullptr, ws + B.off[j], x0, lam0, u0, Vout,
                        nullptr, status, iters, sh);
}

__global__ void k_reset_counter(int32_t* counter) {
  if (threadIdx.x == 0) *counter = 0;
}

// Calls f(NB, FC) with the instantiated tile (as integral constants) that
// matches the arguments' sweep batch and forward chunk.
template <int V>
using Int = std::integral_constant<int, V>;
template <int NB, class F>
void with_chunk(const BvpArgs& a, F&& f) {
  if (a.fc == 8)
    f(Int<NB>{}, Int<8>{});
  else
    f(Int<NB>{}, Int<12>{});
}
template <class F>
void with_tile(const BvpArgs& a, F&& f) {
  switch (a.nb) {
    case 10: with_chunk<10>(a, f); break;
    case 12: with_chunk<12>(a, f); break;
    case 16: with_chunk<16>(a, f); break;
    default: with_chunk<8>(a, f); break;
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

// Workspace of one BVP in doubles, a multiple of 256 bytes: the iterate and
// the trial point ((N + 1) x 12 each), F_0 and F_N (16), the
// interval solutions N x 84 (in the solve's type) and the point blocks
// kPB x pb_stride(N) (71 entries per point, in the solve's type).
int64_t bvp_doubles(int64_t N, int fp32) {
  const int64_t esize = fp32 ? 4 : 8;
  const int64_t d = 24 * (N + 1) + 16 + kZI * N + (kPB * pb_stride(N) * esize + 7) / 8;
  return (d + 31) / 32 * 32;
}

// Validate a problem and derive the kernel arguments.
int make_bvp_args(const sgcm_problem* p, BvpArgs* a) {
  if (!p) return SGCM_EINVAL;
  if (p->model == SGCM_MODEL_EXAMPLE3) return SGCM_EUNSUPPORTED;  // its own solver (example3.hip)
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
  if (p->max_halvings < 0 || p->max_halvings > 60) return SGCM_EINVAL;
  if (p->continuation < 0 || p->continuation > 64) return SGCM_EINVAL;
  if (p->scheme != SGCM_TRAPEZOID && p->scheme != SGCM_LOBATTO4) return SGCM_EINVAL;
  if (p->scheme == SGCM_LOBATTO4 && p->precision != SGCM_FP64) return SGCM_EUNSUPPORTED;
  if (p->sweep_batch < 0 || p->forward_chunk < 0) return SGCM_EINVAL;
  if ((p->sweep_batch != 0 && p->sweep_batch != 8 && p->sweep_batch != 10 && p->sweep_batch != 12 &&
       p->sweep_batch != 16) ||
      (p->forward_chunk != 0 && p->forward_chunk != 8 && p->forward_chunk != 12))
    return SGCM_EUNSUPPORTED;
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
  a->fp32 = p->precision == SGCM_FP32;
  // With three independent controls S_w is invertible and the 3 x 3 system of
  // a sweep step, (I + S_w T1) M = S_w T, is solved as (S_w^{-1} + T1) M = T.
  a->sinv = 0;
  if (p->m == 3) {
    const double* S = a->Sw;
    const double c00 = S[4] * S[8] - S[5] * S[7], c01 = S[5] * S[6] - S[3] * S[8], c02 = S[3] * S[7] - S[4] * S[6];
    const double det = S[0] * c00 + S[1] * c01 + S[2] * c02;
    double nrm = 0.0;
    for (int e = 0; e < 9; ++e) nrm = std::fmax(nrm, std::fabs(S[e]));
    if (std::isfinite(det) && std::fabs(det) > 1e-6 * nrm * nrm * nrm) {
      const double r = 1.0 / det;
      a->Si[0] = c00 * r;
      a->Si[1] = (S[2] * S[7] - S[1] * S[8]) * r;
      a->Si[2] = (S[1] * S[5] - S[2] * S[4]) * r;
      a->Si[3] = c01 * r;
      a->Si[4] = (S[0] * S[8] - S[2] * S[6]) * r;
      a->Si[5] = (S[2] * S[3] - S[0] * S[5]) * r;
      a->Si[6] = c02 * r;
      a->Si[7] = (S[1] * S[6] - S[0] * S[7]) * r;
      a->Si[8] = (S[0] * S[4] - S[1] * S[3]) * r;
      a->sinv = 1;
    }
  }
  if (!a->sinv)
    for (int e = 0; e < 9; ++e) a->Si[e] = 0.0;
  a->scheme = p->scheme;
  a->per_bvp = p->scheme == SGCM_LOBATTO4 ? lobatto_doubles(p->N) : bvp_doubles(p->N, a->fp32);
  // the four-point Lobatto IIIA coefficients (closed forms; row 0 is zero
  // and row 3 the Lobatto quadrature weights)
  {
    const double r5 = std::sqrt(5.0);
    const double lob[4][4] = {{0.0, 0.0, 0.0, 0.0},
                              {(11.0 + r5) / 120.0, (25.0 - r5) / 120.0, (25.0 - 13.0 * r5) / 120.0, (-1.0 + r5) / 120.0},
                              {(11.0 - r5) / 120.0, (25.0 + 13.0 * r5) / 120.0, (25.0 + r5) / 120.0, (-1.0 - r5) / 120.0},
                              {1.0 / 12.0, 5.0 / 12.0, 5.0 / 12.0, 1.0 / 12.0}};
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) a->lob[i][j] = lob[i][j];
  }
  a->y1 = nullptr;
  a->y1_check = nullptr;
  a->max_halvings = p->max_halvings;
  a->nb = p->sweep_batch ? p->sweep_batch : 8;
  a->fc = p->forward_chunk ? p->forward_chunk : 12;
  a->resume = 0;
  a->keep = 0;
  a->outputs = 1;
  return SGCM_OK;
}

// Number of continuation stages before the problem's own: p->continuation
// for two controls, else none.
int continuation_stages(const sgcm_problem* p) { return p->m == 2 ? p->continuation : 0; }

// Stage k of the continuation of a two-control problem (k < stages: the
// three-control problem with B_k = [B_1 B_2 s_k b3], s_k = 1 - k / stages,
// b3 the unit normal B_1 x B_2 / |B_1 x B_2| of the torque plane; k = stages:
// the problem itself), without continuation of its own.
sgcm_problem stage_problem(const sgcm_problem* p, int k) {
  sgcm_problem q = *p;
  q.continuation = 0;
  const int K = continuation_stages(p);
  if (k < K) {
    const double* B1 = p->B;
    const double* B2 = p->B + 3;
    double b3[3] = {B1[1] * B2[2] - B1[2] * B2[1], B1[2] * B2[0] - B1[0] * B2[2], B1[0] * B2[1] - B1[1] * B2[0]};
    const double nb = std::sqrt(b3[0] * b3[0] + b3[1] * b3[1] + b3[2] * b3[2]);
    const double sk = 1.0 - (double)k / K;
    q.m = 3;
    for (int i = 0; i < 3; ++i) q.B[6 + i] = sk * (b3[i] / nb);
  }
  return q;
}

}  // namespace
}  // namespace sgcm

using namespace sgcm;

// The first Newton steps made inside a call.  The step from Y = 0 is linear
// in the initial state (the residual there is [-xbar; 0; 0] and the Jacobian
// does not depend on xbar), so a call with many BVPs first computes the steps
// of the six unit initial states by doubling (about log2 N dependent steps of
// 6 x 6 algebra, first_steps.hip), and every BVP forms its step as their
// combination: no workgroup of the main launch takes the long serial sweep of
// that step.  The results are those of a solve with a plan of the same
// problem.
constexpr int64_t kInCallPlanMin = 64;  // BVPs per call from which this pays

struct InCallPlan {
  size_t y1, chk, total;  // byte offsets in the region, its size
};

// The region behind the BVP workspaces and the launch order, or total = 0
// when the call takes its first steps per BVP.
static InCallPlan in_call_plan(const sgcm_problem* p, int64_t n_bvps) {
  InCallPlan r{};
  if (p->scheme != SGCM_TRAPEZOID || n_bvps < kInCallPlanMin) return r;
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  size_t o = 0;
  r.y1 = o;
  o += up((size_t)6 * 12 * ((size_t)p->N + 1) * sizeof(double));
  r.chk = o;
  o += up(12 * sizeof(int32_t));
  r.total = o;
  return r;
}

// The arguments of the problem whose first steps a call or a plan takes:
// the first continuation stage, in FP64.
static int first_step_args(const sgcm_problem* p, BvpArgs* qa) {
  sgcm_problem q = stage_problem(p, 0);
  q.precision = SGCM_FP64;
  return make_bvp_args(&q, qa);
}

extern "C" int sgcm_solve_bvps_workspace(const sgcm_problem* p, int64_t n_bvps, size_t* bytes) {
  BvpArgs a;
  if (!bytes || n_bvps < 0) return SGCM_EINVAL;
  if (p && p->model == SGCM_MODEL_EXAMPLE3) return ex3_workspace(p, n_bvps, bytes);
  int rc = make_bvp_args(p, &a);
  if (rc != SGCM_OK) return rc;
  *bytes = (size_t)a.per_bvp * sizeof(double) * (size_t)n_bvps + order_bytes(n_bvps) +
           in_call_plan(p, n_bvps).total;
  return SGCM_OK;
}

// sgcm_solve_bvps, with the first Newton steps of a plan (y1) or without (null).
static int solve_bvps(const sgcm_problem* p, const double* y1, int64_t n_bvps, const double* x0, double* lambda0,
               double* u0, double* V, double* traj, int32_t* status, int32_t* iters, void* workspace,
               size_t ws_bytes, void* stream) {
  BvpArgs a;
  if (n_bvps < 0) return SGCM_EINVAL;
  if (p && p->model == SGCM_MODEL_EXAMPLE3 && !y1)
    return ex3_solve(p, n_bvps, x0, 0, lambda0, u0, V, traj, status, iters, workspace, ws_bytes, stream);
  int rc = make_bvp_args(p, &a);
  if (rc != SGCM_OK) return rc;
  a.y1 = y1;
  if (n_bvps == 0) return SGCM_OK;
  if (n_bvps > 0x7fffffffLL) return SGCM_EUNSUPPORTED;
  if (!x0 || !lambda0 || !u0 || !status || !iters || !workspace) return SGCM_EINVAL;
  if (((uintptr_t)workspace & 255u) != 0) return SGCM_EINVAL;
  const size_t bvp_bytes = (size_t)a.per_bvp * sizeof(double) * (size_t)n_bvps;
  const InCallPlan icp = y1 ? InCallPlan{} : in_call_plan(p, n_bvps);
  if (ws_bytes < bvp_bytes + order_bytes(n_bvps) + icp.total) return SGCM_EINVAL;
  const int K = continuation_stages(p);
  if (K > 0) {  // the torque plane needs a normal: B_1 and B_2 not parallel
    const double* B1 = p->B;
    const double* B2 = p->B + 3;
    const double c0 = B1[1] * B2[2] - B1[2] * B2[1], c1 = B1[2] * B2[0] - B1[0] * B2[2],
                 c2 = B1[0] * B2[1] - B1[1] * B2[0];
    if (!(c0 * c0 + c1 * c1 + c2 * c2 > 0.0)) return SGCM_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const int32_t* y1_check = nullptr;
  if (icp.total > 0) {  // the first steps of the unit initial states, in this call
    char* base = reinterpret_cast<char*>(workspace) + bvp_bytes + order_bytes(n_bvps);
    BvpArgs qa;
    rc = first_step_args(p, &qa);
    if (rc != SGCM_OK) return rc;
    double* uy1 = reinterpret_cast<double*>(base + icp.y1);
    int32_t* chk = reinterpret_cast<int32_t*>(base + icp.chk);
    rc = launch_first_steps(qa, p->N, uy1, chk, s);
    if (rc != SGCM_OK) return rc;
    y1 = uy1;
    y1_check = chk;
    a.y1 = y1;
    a.y1_check = y1_check;
  }
  int32_t* order = nullptr;
  if (n_bvps > 1 && n_bvps <= kOrderMax) {
    order = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(workspace) + bvp_bytes);
    hipLaunchKernelGGL(k_order, dim3(1), dim3(1024), 0, s, x0, (int)n_bvps, order);
  }
  // one launch per continuation stage (one in all without continuation), all
  // with the same launch order, so that workgroup g keeps workspace slot g
  for (int k = 0; k <= K; ++k) {
    if (K > 0) {
      const sgcm_problem q = stage_problem(p, k);
      rc = make_bvp_args(&q, &a);
      if (rc != SGCM_OK) return rc;
      a.y1 = k == 0 ? y1 : nullptr;
      a.y1_check = k == 0 ? y1_check : nullptr;
      a.resume = k > 0;
      a.keep = k < K;
      a.outputs = k == K;
    }
    if (a.scheme == SGCM_LOBATTO4) {
      if (launch_lobatto(a, n_bvps, x0, lambda0, u0, V, traj, status, iters, (double*)workspace, order, s) != SGCM_OK)
        return SGCM_EDEVICE;
      continue;
    }
    with_tile(a, [&](auto nb, auto fc) {
      constexpr int NB = decltype(nb)::value, FC = decltype(fc)::value;
      if (a.fp32)
        hipLaunchKernelGGL((k_newton<float, NB, FC>), dim3((unsigned)n_bvps), dim3(64), 0, s, a, x0, lambda0, u0, V,
                           traj, status, iters, (double*)workspace, order);
      else
        hipLaunchKernelGGL((k_newton<double, NB, FC>), dim3((unsigned)n_bvps), dim3(64), 0, s, a, x0, lambda0, u0,
                           V, traj, status, iters, (double*)workspace, order);
    });
    if (hipGetLastError() != hipSuccess) return SGCM_EDEVICE;
  }
  return SGCM_OK;
}

extern "C" int sgcm_solve_bvps(const sgcm_problem* p, int64_t n_bvps, const double* x0, double* lambda0,
                               double* u0, double* V, double* traj, int32_t* status, int32_t* iters,
                               void* workspace, size_t ws_bytes, void* stream) {
  sgcm::CallRange range("sgcm_solve_bvps");
  return solve_bvps(p, nullptr, n_bvps, x0, lambda0, u0, V, traj, status, iters, workspace, ws_bytes, stream);
}

// ---- the solve without allocation ---------------------------------------------

// The workspace of sgcm_solve_bvps_static: one copy of this array per device
// the library runs on, held until the process ends.  In host code its name is
// a host-side stand-in; kernels get its device address, looked up once per
// device with hipGetSymbolAddress.
static __device__ __align__(256) double scratch[SGCM_STATIC_SCRATCH_BYTES / sizeof(double)];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device (null: not looked up)

// The device address of `scratch` on the current device.
static int static_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SGCM_EDEVICE;
  if (dev < 0 || dev >= kMaxDevices) return SGCM_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return SGCM_EDEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SGCM_OK;
}

extern "C" int sgcm_solve_bvps_static(const sgcm_problem* p, int64_t n_bvps, const double* x0, double* lambda0,
                                      double* u0, double* V, double* traj, int32_t* status, int32_t* iters,
                                      void* stream) {
  size_t need = 0;
  int rc = sgcm_solve_bvps_workspace(p, n_bvps, &need);  // validates p and n_bvps
  if (rc != SGCM_OK) return rc;
  if (need > (size_t)SGCM_STATIC_SCRATCH_BYTES) return SGCM_EUNSUPPORTED;
  if (n_bvps == 0) return SGCM_OK;
  void* ws = nullptr;
  rc = static_scratch(&ws);
  if (rc != SGCM_OK) return rc;
  return solve_bvps(p, nullptr, n_bvps, x0, lambda0, u0, V, traj, status, iters, ws,
                    (size_t)SGCM_STATIC_SCRATCH_BYTES, stream);
}

struct sgcm_plan {
  sgcm_problem p;
  int dev;     // the device current at creation, which holds y1
  double* y1;  // device, 6 x (N + 1) x 12
};

// The first Newton step of the six unit initial states of problem p into y1
// (device, 6 x (N + 1) x 12), on stream s, which is then synchronized.
// SGCM_EUNSUPPORTED when the step is not finite (a singular linearised
// system).
static int first_steps(const sgcm_problem* p, double* y1, hipStream_t s) {
  BvpArgs qa;
  int rc = first_step_args(p, &qa);
  if (rc != SGCM_OK) return rc;
  int32_t* chk = nullptr;  // the 12 statuses and iteration counts
  if (hipMalloc((void**)&chk, 12 * sizeof(int32_t)) != hipSuccess) {
    (void)hipGetLastError();
    return SGCM_ENOMEM;
  }
  int32_t hst[12];
  rc = launch_first_steps(qa, p->N, y1, chk, s);
  if (rc == SGCM_OK && hipMemcpyAsync(hst, chk, sizeof(hst), hipMemcpyDeviceToHost, s) != hipSuccess)
    rc = SGCM_EDEVICE;
  if (rc == SGCM_OK && hipStreamSynchronize(s) != hipSuccess) rc = SGCM_EDEVICE;
  (void)hipFree(chk);  // waits for the device
  for (int j = 0; rc == SGCM_OK && j < 6; ++j)
    if ((hst[j] != SGCM_BVP_CONVERGED && hst[j] != SGCM_BVP_MAXITER) || hst[6 + j] != 0) rc = SGCM_EUNSUPPORTED;
  if (rc != SGCM_OK) (void)hipGetLastError();
  return rc;
}

extern "C" int sgcm_plan_create(const sgcm_problem* p, void* stream, sgcm_plan** out) {
  sgcm::CallRange range("sgcm_plan_create");
  if (!out) return SGCM_EINVAL;
  *out = nullptr;
  BvpArgs a;
  int rc = make_bvp_args(p, &a);
  if (rc != SGCM_OK) return rc;
  if (p->scheme != SGCM_TRAPEZOID) return SGCM_EUNSUPPORTED;  // plans hold trapezoidal first steps
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SGCM_EDEVICE;
  sgcm_plan* plan = new (std::nothrow) sgcm_plan();
  if (!plan) return SGCM_ENOMEM;
  plan->p = *p;
  plan->dev = dev;
  plan->y1 = nullptr;
  const size_t y1_bytes = (size_t)6 * 12 * ((size_t)p->N + 1) * sizeof(double);
  if (hipMalloc((void**)&plan->y1, y1_bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete plan;
    return SGCM_ENOMEM;
  }
  // a singular or non-finite linearised step has no plan (the solve without
  // one reports it per BVP)
  rc = first_steps(p, plan->y1, (hipStream_t)stream);
  if (rc != SGCM_OK) {
    (void)hipFree(plan->y1);
    delete plan;
    return rc;
  }
  *out = plan;
  return SGCM_OK;
}

extern "C" int sgcm_solve_bvps_plan(const sgcm_plan* plan, int64_t n_bvps, const double* x0, double* lambda0,
                                    double* u0, double* V, double* traj, int32_t* status, int32_t* iters,
                                    void* workspace, size_t ws_bytes, void* stream) {
  sgcm::CallRange range("sgcm_solve_bvps_plan");
  if (!plan) return SGCM_EINVAL;
  if (n_bvps > 0) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return SGCM_EDEVICE;
    if (dev != plan->dev) return SGCM_EINVAL;  // the plan's steps live on its own device
  }
  return solve_bvps(&plan->p, plan->y1, n_bvps, x0, lambda0, u0, V, traj, status, iters, workspace, ws_bytes,
                    stream);
}

extern "C" void sgcm_plan_destroy(sgcm_plan* plan) {
  if (!plan) return;
  (void)hipFree(plan->y1);
  delete plan;
}

extern "C" int sgcm_characteristic_rhs(const sgcm_problem* p, int64_t n_points, const double* y, double* phi,
                                       double* dphi, void* stream) {
  sgcm::CallRange range("sgcm_characteristic_rhs");
  BvpArgs a;
  if (n_points < 0) return SGCM_EINVAL;
  if (p && p->model == SGCM_MODEL_EXAMPLE3) return ex3_characteristic_rhs(p, n_points, y, phi, dphi, stream);
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

// ---- batches with per-BVP mesh size and horizon ----------------------------

// The least number of BVPs of one (N, T) for which a batch solves the first
// Newton steps of the unit initial states once (see sgcm_batch_create).
constexpr int kMinGroupSteps = 8;

struct sgcm_batch {
  BvpArgs args;  // the problem; args.N, args.h, args.per_bvp are unused
  int64_t n = 0;
  int dev = -1;
  int32_t* N = nullptr;
  double* h = nullptr;
  int64_t* off = nullptr;
  int32_t* order = nullptr;
  int32_t* counter = nullptr;
  double* y1 = nullptr;       // first Newton steps of the unit initial states, per (N, T) group
  int64_t* y1off = nullptr;   // per BVP: its group's steps in y1, or -1
  size_t ws_doubles = 0;
  sgcm_schedule sched{1, 0};
  int64_t slots = 0;  // persistent workgroups (0: one workgroup per BVP)
};

extern "C" int sgcm_batch_create(const sgcm_problem* p, int64_t n_bvps, const int32_t* N, const double* T,
                                 const sgcm_schedule* sched, sgcm_batch** out) {
  sgcm::CallRange range("sgcm_batch_create");
  if (!out) return SGCM_EINVAL;
  *out = nullptr;
  if (!p || n_bvps < 1 || n_bvps > 0x7fffffffLL || !N || !T) return SGCM_EINVAL;
  sgcm_schedule sc = sched ? *sched : sgcm_schedule{1, 0};
  if (sc.order < 0 || sc.order > 1 || sc.slots_per_cu < 0 || sc.slots_per_cu > 8) return SGCM_EINVAL;
  sgcm_problem q = *p;  // the problem's own mesh and horizon are not used
  q.N = 1;
  q.T = 1.0;
  BvpArgs a;
  int rc = make_bvp_args(&q, &a);
  if (rc != SGCM_OK) return rc;
  if (continuation_stages(p) > 0) return SGCM_EUNSUPPORTED;  // batches take one stage
  if (p->scheme != SGCM_TRAPEZOID) return SGCM_EUNSUPPORTED;   // batches run the trapezoidal kernel
  std::vector<int32_t> hN(N, N + n_bvps), horder(n_bvps);
  std::vector<double> hh(n_bvps);
  std::vector<int64_t> hoff(n_bvps);
  int64_t total = 0;
  for (int64_t i = 0; i < n_bvps; ++i) {
    if (N[i] < 1 || N[i] > 65536 || !(std::isfinite(T[i]) && T[i] > 0.0)) return SGCM_EINVAL;
    hh[i] = T[i] / N[i];
    hoff[i] = total;
    total += bvp_doubles(N[i], a.fp32);
    horder[i] = (int32_t)i;
  }
  if (sc.order == 1)  // larger N T first (the longest chains start first)
    std::stable_sort(horder.begin(), horder.end(), [&](int32_t x, int32_t y) {
      return (double)N[x] * T[x] > (double)N[y] * T[y];
    });
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SGCM_EDEVICE;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return SGCM_EDEVICE;
  sgcm_batch* b = new (std::nothrow) sgcm_batch();
  if (!b) return SGCM_ENOMEM;
  b->args = a;
  b->n = n_bvps;
  b->dev = dev;
  b->ws_doubles = (size_t)total;
  b->sched = sc;
  b->slots = (int64_t)sc.slots_per_cu * cus;
  auto up = [](void** dst, const void* src, size_t bytes) -> bool {
    if (hipMalloc(dst, bytes) != hipSuccess) return false;
    return src == nullptr || hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  const int32_t zero = 0;
  // one set of first Newton steps per distinct (N, T) of at least
  // kMinGroupSteps BVPs, as for a solve plan (a smaller group would pay a
  // launch and its steps' memory for a few BVPs; its BVPs solve their own)
  std::vector<std::pair<int32_t, double>> keys(n_bvps);
  for (int64_t i = 0; i < n_bvps; ++i) keys[i] = {N[i], T[i]};
  std::vector<std::pair<int32_t, double>> sorted_keys(keys);
  std::sort(sorted_keys.begin(), sorted_keys.end());
  std::vector<std::pair<int32_t, double>> groups;
  for (size_t i = 0; i < sorted_keys.size();) {
    size_t j = i;
    while (j < sorted_keys.size() && sorted_keys[j] == sorted_keys[i]) ++j;
    if (j - i >= (size_t)kMinGroupSteps) groups.push_back(sorted_keys[i]);
    i = j;
  }
  std::vector<int64_t> goff(groups.size());
  int64_t y1_total = 0;
  for (size_t g = 0; g < groups.size(); ++g) {
    goff[g] = y1_total;
    y1_total += (int64_t)6 * 12 * (groups[g].first + 1);
  }
  std::vector<int64_t> hy1off(n_bvps, -1);
  for (int64_t i = 0; i < n_bvps; ++i) {
    const auto it = std::lower_bound(groups.begin(), groups.end(), keys[i]);
    if (it != groups.end() && *it == keys[i]) hy1off[i] = goff[it - groups.begin()];
  }
  bool ok = up((void**)&b->N, hN.data(), n_bvps * sizeof(int32_t)) &&
            up((void**)&b->h, hh.data(), n_bvps * sizeof(double)) &&
            up((void**)&b->off, hoff.data(), n_bvps * sizeof(int64_t)) &&
            up((void**)&b->order, horder.data(), n_bvps * sizeof(int32_t)) &&
            up((void**)&b->counter, &zero, sizeof(int32_t)) &&
            (y1_total == 0 || up((void**)&b->y1, nullptr, (size_t)y1_total * sizeof(double)));
  if (!ok) {
    (void)hipGetLastError();
    sgcm_batch_destroy(b);
    return SGCM_ENOMEM;
  }
  for (size_t g = 0; g < groups.size(); ++g) {
    sgcm_problem qg = *p;
    qg.N = groups[g].first;
    qg.T = groups[g].second;
    rc = first_steps(&qg, b->y1 + goff[g], nullptr);
    if (rc == SGCM_EUNSUPPORTED) {  // that group's BVPs take their own first step
      for (int64_t i = 0; i < n_bvps; ++i)
        if (keys[i] == groups[g]) hy1off[i] = -1;
    } else if (rc != SGCM_OK) {
      sgcm_batch_destroy(b);
      return rc;
    }
  }
  if (!up((void**)&b->y1off, hy1off.data(), n_bvps * sizeof(int64_t))) {
    (void)hipGetLastError();
    sgcm_batch_destroy(b);
    return SGCM_ENOMEM;
  }
  *out = b;
  return SGCM_OK;
}

extern "C" int sgcm_batch_workspace(const sgcm_batch* b, size_t* bytes) {
  if (!b || !bytes) return SGCM_EINVAL;
  *bytes = b->ws_doubles * sizeof(double);
  return SGCM_OK;
}

extern "C" int sgcm_solve_bvps_batch(const sgcm_batch* b, const double* x0, double* lambda0, double* u0,
                                     double* V, int32_t* status, int32_t* iters, void* workspace,
                                     size_t ws_bytes, void* stream) {
  sgcm::CallRange range("sgcm_solve_bvps_batch");
  if (!b || !x0 || !lambda0 || !u0 || !status || !iters || !workspace) return SGCM_EINVAL;
  if (((uintptr_t)workspace & 255u) != 0 || ws_bytes < b->ws_doubles * sizeof(double)) return SGCM_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SGCM_EDEVICE;
  if (dev != b->dev) return SGCM_EINVAL;
  BatchArgs B;
  B.N = b->N;
  B.h = b->h;
  B.off = b->off;
  B.order = b->order;
  B.counter = b->counter;
  B.y1 = b->y1;
  B.y1off = b->y1off;
  B.n = b->n;
  B.persistent = b->slots > 0;
  hipStream_t s = (hipStream_t)stream;
  if (B.persistent) {
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, b->counter);
  }
  const unsigned g = (unsigned)(B.persistent ? (b->slots < b->n ? b->slots : b->n) : b->n);
  with_tile(b->args, [&](auto nb, auto fc) {
    constexpr int NB = decltype(nb)::value, FC = decltype(fc)::value;
    if (!B.persistent) {
      if (b->args.fp32)
        hipLaunchKernelGGL((k_newton_batch_grid<float, NB, FC>), dim3(g), dim3(64), 0, s, b->args, B, x0, lambda0,
                           u0, V, status, iters, (double*)workspace);
      else
        hipLaunchKernelGGL((k_newton_batch_grid<double, NB, FC>), dim3(g), dim3(64), 0, s, b->args, B, x0, lambda0,
                           u0, V, status, iters, (double*)workspace);
    } else if (b->args.fp32)
      hipLaunchKernelGGL((k_newton_batch<float, NB, FC>), dim3(g), dim3(64), 0, s, b->args, B, x0, lambda0, u0, V,
                         status, iters, (double*)workspace);
    else
      hipLaunchKernelGGL((k_newton_batch<double, NB, FC>), dim3(g), dim3(64), 0, s, b->args, B, x0, lambda0, u0, V,
                         status, iters, (double*)workspace);
  });
  return hipGetLastError() == hipSuccess ? SGCM_OK : SGCM_EDEVICE;
}

extern "C" void sgcm_batch_destroy(sgcm_batch* b) {
  if (!b) return;
  (void)hipFree(b->N);
  (void)hipFree(b->h);
  (void)hipFree(b->off);
  (void)hipFree(b->order);
  (void)hipFree(b->counter);
  (void)hipFree(b->y1);
  (void)hipFree(b->y1off);
  delete b;
}

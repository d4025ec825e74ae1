// FP64 CPU oracle for the sparse grid characteristics method (Kang & Wilcox,
// "Mitigating the Curse of Dimensionality: Sparse Grid Characteristics Method
// for Optimal Feedback Control and HJB Equations").
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
// GPU library is checked against.  Only the test-suite, the smoke check and
// the CPU-baseline leg of the benchmark may load it.  It shares no code,
// header, table or helper with the GPU library.
//
// What it computes, in the paper's order:
//   * the CGL (Clenshaw-Curtis) nested 1-D sets X^i and new points dX^i
//     (Sec. 3.2, eq. CGL) and the Smolyak sparse grid G^q = U_{|i|<=q} dX^i
//     (Sec. 3.2);
//   * Lagrange basis functions on X^i (Sec. 3.3, the product formula for the
//     CGL grid), hierarchical surpluses by the level recursion of eq. interpo,
//     evaluation of the hierarchical interpolant (route A) and, independently,
//     of the combination formula eq. interpolation2 (route B);
//   * the characteristics two-point BVP of eq. hamchar at one initial state:
//     state and costate equations evaluated at u* = argmin_u H (Sec. 2),
//     discretised by trapezoidal collocation on a uniform mesh, or by the
//     four-point Lobatto IIIA collocation the paper uses (Sec. 3.1, Sec. 5.1),
//     solved by Newton's method from the zero trajectory, with the Jacobian from
//     hyper-dual (second-order forward-mode) automatic differentiation of the
//     hand-written f, L and h only, and a plain banded LU with row partial
//     pivoting;
//   * the outputs of eq. optuv: u*(t,x) = u*(t,x,lambda(t)) and
//     V = z(T) + h(x(T)), z integrated with the same trapezoidal rule.
//
// Readings where the paper is silent (the discretisation, the initial guess,
// the stopping rule) are listed in the design notes of the repository; the
// short version is: trapezoid (the two-point Lobatto IIIA member) on a uniform
// mesh; Newton from Y = 0 whose first step (the solve of the problem
// linearised about the origin) is not counted; stop when the max-norm of the
// collocation residual is <= tol, tested before every update; each counted
// step damped by backtracking on that max-norm (the full step whenever it
// decreases the norm enough); for two controls, optionally a continuation
// from the three-control problem (see solve_bvp).
//
// Parity status: every exported function is pinned by the CPU test-suite
// (printed grids, polynomial exactness, the discrete and continuous Riccati
// closed forms, the Example III closed form, symbolic Jacobians and brute-force
// shooting).  No function here is "parity unpinned".

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// Hyper-dual numbers: v + e1*a + e2*b + e1e2*c with e1^2 = e2^2 = 0.
// Seeding e1 along z_a and e2 along z_b gives dH/dz_a in the e1 part and
// d2H/dz_a dz_b in the e1e2 part, exactly (no truncation error).
// ---------------------------------------------------------------------------
struct HD {
  double v, e1, e2, e12;
  HD() : v(0), e1(0), e2(0), e12(0) {}
  HD(double x) : v(x), e1(0), e2(0), e12(0) {}
  HD(double a, double b, double c, double d) : v(a), e1(b), e2(c), e12(d) {}
};
inline HD operator+(HD a, HD b) { return HD(a.v + b.v, a.e1 + b.e1, a.e2 + b.e2, a.e12 + b.e12); }
inline HD operator-(HD a, HD b) { return HD(a.v - b.v, a.e1 - b.e1, a.e2 - b.e2, a.e12 - b.e12); }
inline HD operator-(HD a) { return HD(-a.v, -a.e1, -a.e2, -a.e12); }
inline HD operator*(HD a, HD b) {
  return HD(a.v * b.v, a.v * b.e1 + a.e1 * b.v, a.v * b.e2 + a.e2 * b.v,
            a.v * b.e12 + a.e1 * b.e2 + a.e2 * b.e1 + a.e12 * b.v);
}
// chain rule for a scalar function g with value g0, first derivative g1 and
// second derivative g2 at a.v
inline HD chain(HD a, double g0, double g1, double g2) {
  return HD(g0, g1 * a.e1, g1 * a.e2, g1 * a.e12 + g2 * a.e1 * a.e2);
}
inline HD recip(HD a) {
  double r = 1.0 / a.v;
  return chain(a, r, -r * r, 2.0 * r * r * r);
}
inline HD operator/(HD a, HD b) { return a * recip(b); }
inline HD sin(HD a) { return chain(a, std::sin(a.v), std::cos(a.v), -std::sin(a.v)); }
inline HD cos(HD a) { return chain(a, std::cos(a.v), -std::sin(a.v), -std::cos(a.v)); }
inline HD tan(HD a) {
  double t = std::tan(a.v);
  double s = 1.0 + t * t;
  return chain(a, t, s, 2.0 * t * s);
}
inline double sin(double a) { return std::sin(a); }
inline double cos(double a) { return std::cos(a); }
inline double tan(double a) { return std::tan(a); }

}  // namespace

// ---------------------------------------------------------------------------
// Problem description (the oracle's own struct; filled from Python).
// ---------------------------------------------------------------------------
extern "C" {

enum { ORC_RIGID_BODY = 0, ORC_LINEARISED = 1, ORC_EXAMPLE3 = 2 };
enum { ORC_CONVERGED = 0, ORC_MAXITER = 1, ORC_SINGULAR = 2, ORC_NONFINITE = 3 };

typedef struct {
  int32_t model;     // ORC_RIGID_BODY, ORC_LINEARISED or ORC_EXAMPLE3
  int32_t n, m;      // state and control dimension (6,3), (6,2) or (3,1)
  double J[3];       // diagonal inertia
  double B[9];       // 3 x m input matrix, column-major: B[i + 3*j]
  double q_w, r_w, p_w;  // running state weight, control weight, terminal weight
  double T;          // horizon
  int32_t N;         // uniform mesh intervals
  double tol;        // Newton stopping tolerance on max|F|
  int32_t max_iter;  // Newton iterations after the first (linearised) step
  int32_t max_halvings;  // backtracking cap H of each Newton step (0: full steps)
  int32_t continuation;  // K > 0: continuation stages (two controls, or Example III), see solve_bvp
  int32_t scheme;        // ORC_TRAPEZOID or ORC_LOBATTO4 (collocation formula)
} oracle_problem;

enum { ORC_TRAPEZOID = 0, ORC_LOBATTO4 = 1 };

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Hand-written model functions.  Only f, L and h are written by hand; every
// derivative is taken by automatic differentiation below.
// ---------------------------------------------------------------------------

// Rigid body with Euler angles v = (phi, theta, psi) in (3,2,1) order
// (Sec. 5, eq. sat_model with the stored-momentum term replaced by the
// gyroscopic term):  v' = E(v) w,   J w' = -w x (J w) + B u.
template <class T>
void f_rigid(const oracle_problem& p, const T* x, const T* u, T* fx) {
  T phi = x[0], th = x[1];
  T w1 = x[3], w2 = x[4], w3 = x[5];
  T sp = sin(phi), cp = cos(phi), tt = tan(th), ct = cos(th);
  fx[0] = w1 + sp * tt * w2 + cp * tt * w3;
  fx[1] = cp * w2 - sp * w3;
  fx[2] = (sp * w2 + cp * w3) / ct;
  T Jw1 = p.J[0] * w1, Jw2 = p.J[1] * w2, Jw3 = p.J[2] * w3;
  // w x (J w)
  T c1 = w2 * Jw3 - w3 * Jw2;
  T c2 = w3 * Jw1 - w1 * Jw3;
  T c3 = w1 * Jw2 - w2 * Jw1;
  T Bu[3] = {T(0.0), T(0.0), T(0.0)};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < p.m; ++j) Bu[i] = Bu[i] + p.B[i + 3 * j] * u[j];
  fx[3] = (Bu[0] - c1) / T(p.J[0]);
  fx[4] = (Bu[1] - c2) / T(p.J[1]);
  fx[5] = (Bu[2] - c3) / T(p.J[2]);
}

// The rigid body linearised about the origin: v' = w, J w' = B u.
template <class T>
void f_linear(const oracle_problem& p, const T* x, const T* u, T* fx) {
  fx[0] = x[3];
  fx[1] = x[4];
  fx[2] = x[5];
  for (int i = 0; i < 3; ++i) {
    T acc(0.0);
    for (int j = 0; j < p.m; ++j) acc = acc + p.B[i + 3 * j] * u[j];
    fx[3 + i] = acc / T(p.J[i]);
  }
}

// Example III (Sec. 5.3): three states, one control.
template <class T>
void f_example3(const oracle_problem&, const T* x, const T* u, T* fx) {
  T s = T(1.0) + x[0] * x[0] + x[1] * x[1];
  T y = x[2] / s;
  fx[0] = -x[0] + x[1];
  fx[1] = -x[1] + y;
  fx[2] = (T(-2.0) * x[0] * x[0] + T(2.0) * x[0] * x[1] - T(2.0) * x[1] * x[1] +
           T(2.0) * x[1] * y) * y + s * u[0];
}

template <class T>
void f_model(const oracle_problem& p, const T* x, const T* u, T* fx) {
  switch (p.model) {
    case ORC_RIGID_BODY: f_rigid(p, x, u, fx); break;
    case ORC_LINEARISED: f_linear(p, x, u, fx); break;
    default: f_example3(p, x, u, fx); break;
  }
}

// running cost L(x, u)
template <class T>
T L_model(const oracle_problem& p, const T* x, const T* u) {
  if (p.model == ORC_EXAMPLE3) {
    T s = T(1.0) + x[0] * x[0] + x[1] * x[1];
    T y = x[2] / s;
    return T(0.5) * (y * y + u[0] * u[0]);
  }
  T xx(0.0), uu(0.0);
  for (int i = 0; i < p.n; ++i) xx = xx + x[i] * x[i];
  for (int j = 0; j < p.m; ++j) uu = uu + u[j] * u[j];
  return T(0.5) * (T(p.q_w) * xx + T(p.r_w) * uu);
}

// final cost h(x)
template <class T>
T h_model(const oracle_problem& p, const T* x) {
  if (p.model == ORC_EXAMPLE3) return T(0.0);
  T xx(0.0);
  for (int i = 0; i < p.n; ++i) xx = xx + x[i] * x[i];
  return T(0.5 * p.p_w) * xx;
}

// Hamiltonian H(x, lambda, u) = L + lambda^T f  (Sec. 2).  z = (x, lambda, u).
template <class T>
T hamiltonian(const oracle_problem& p, const T* z) {
  const int n = p.n;
  T fx[8];
  f_model(p, z, z + 2 * n, fx);
  T H = L_model(p, z, z + 2 * n);
  for (int i = 0; i < n; ++i) H = H + z[n + i] * fx[i];
  return H;
}

constexpr int MAXZ = 2 * 6 + 3;  // largest (x, lambda, u) vector

// Gradient and Hessian of H over z = (x, lambda, u) at a point, by hyper-dual
// numbers (one evaluation per unordered pair of coordinates).
void hamiltonian_hessian(const oracle_problem& p, const double* z, double* grad,
                         double* hess /* nz x nz row-major */) {
  const int nz = 2 * p.n + p.m;
  HD zz[MAXZ];
  for (int a = 0; a < nz; ++a) {
    for (int b = a; b < nz; ++b) {
      for (int c = 0; c < nz; ++c) zz[c] = HD(z[c]);
      zz[a].e1 = 1.0;
      zz[b].e2 = 1.0;
      HD H = hamiltonian(p, zz);
      hess[a * nz + b] = H.e12;
      hess[b * nz + a] = H.e12;
      if (b == a) grad[a] = H.e1;
    }
  }
}

// Small dense solve A x = b (n <= 15) by Gaussian elimination with partial
// pivoting; returns false on an exactly zero pivot.  A and b are overwritten.
bool dense_solve(int n, double* A, double* b, int nrhs) {
  for (int j = 0; j < n; ++j) {
    int piv = j;
    for (int i = j + 1; i < n; ++i)
      if (std::fabs(A[i * n + j]) > std::fabs(A[piv * n + j])) piv = i;
    if (A[piv * n + j] == 0.0) return false;
    if (piv != j) {
      for (int c = 0; c < n; ++c) std::swap(A[j * n + c], A[piv * n + c]);
      for (int r = 0; r < nrhs; ++r) std::swap(b[j * nrhs + r], b[piv * nrhs + r]);
    }
    for (int i = j + 1; i < n; ++i) {
      double l = A[i * n + j] / A[j * n + j];
      for (int c = j; c < n; ++c) A[i * n + c] -= l * A[j * n + c];
      for (int r = 0; r < nrhs; ++r) b[i * nrhs + r] -= l * b[j * nrhs + r];
    }
  }
  for (int j = n - 1; j >= 0; --j) {
    for (int r = 0; r < nrhs; ++r) {
      double s = b[j * nrhs + r];
      for (int c = j + 1; c < n; ++c) s -= A[j * n + c] * b[c * nrhs + r];
      b[j * nrhs + r] = s / A[j * n + j];
    }
  }
  return true;
}

// u*(x, lambda) = argmin_u H (Sec. 2).  For the models here H is a convex
// quadratic in u (control-affine f, cost quadratic in u), so one Newton step
// on dH/du = 0 from u = 0 lands exactly on the minimiser:
// u* = -H_uu^{-1} H_u(x, lambda, 0).
void ustar(const oracle_problem& p, const double* y, double* u) {
  const int n = p.n, m = p.m, nz = 2 * n + m;
  double z[MAXZ];
  for (int i = 0; i < 2 * n; ++i) z[i] = y[i];
  for (int j = 0; j < m; ++j) z[2 * n + j] = 0.0;
  double g[3], Huu[9];
  HD zz[MAXZ];
  for (int a = 0; a < m; ++a) {
    for (int b = a; b < m; ++b) {
      for (int c = 0; c < nz; ++c) zz[c] = HD(z[c]);
      zz[2 * n + a].e1 = 1.0;
      zz[2 * n + b].e2 = 1.0;
      HD H = hamiltonian(p, zz);
      Huu[a * m + b] = Huu[b * m + a] = H.e12;
      if (a == b) g[a] = -H.e1;
    }
  }
  dense_solve(m, Huu, g, 1);
  for (int j = 0; j < m; ++j) u[j] = g[j];
}

// The right-hand side of the characteristic equations eq. hamchar at
// y = (x, lambda):  Phi = [ (dH/dlambda)^T ; -(dH/dx)^T ] at u = u*(x, lambda),
// and its Jacobian dPhi/dy.  Because dH/du = 0 at u* for every y, the
// derivative of y -> (dH/dy)(y, u*(y)) is the Schur complement
// H_yy - H_yu H_uu^{-1} H_uy (implicit function theorem).
void phi_and_jacobian(const oracle_problem& p, const double* y, double* Phi,
                      double* dPhi /* 2n x 2n row-major, may be null */) {
  const int n = p.n, m = p.m, ny = 2 * n, nz = ny + m;
  double z[MAXZ];
  for (int i = 0; i < ny; ++i) z[i] = y[i];
  ustar(p, y, z + ny);
  double grad[MAXZ], hess[MAXZ * MAXZ];
  if (dPhi == nullptr) {
    // gradient only: one dual evaluation per coordinate of y
    HD zz[MAXZ];
    for (int a = 0; a < ny; ++a) {
      for (int c = 0; c < nz; ++c) zz[c] = HD(z[c]);
      zz[a].e1 = 1.0;
      grad[a] = hamiltonian(p, zz).e1;
    }
  } else {
    hamiltonian_hessian(p, z, grad, hess);
  }
  for (int i = 0; i < n; ++i) {
    Phi[i] = grad[n + i];   // x' =  dH/dlambda
    Phi[n + i] = -grad[i];  // lambda' = -dH/dx
  }
  if (dPhi == nullptr) return;
  // Hstar_yy = H_yy - H_yu H_uu^{-1} H_uy
  double Huu[9], X[3 * 12];
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b) Huu[a * m + b] = hess[(ny + a) * nz + ny + b];
  for (int a = 0; a < m; ++a)
    for (int c = 0; c < ny; ++c) X[a * ny + c] = hess[(ny + a) * nz + c];
  dense_solve(m, Huu, X, ny);  // X = H_uu^{-1} H_uy  (m x ny)
  double Hs[12 * 12];
  for (int a = 0; a < ny; ++a)
    for (int b = 0; b < ny; ++b) {
      double s = hess[a * nz + b];
      for (int k = 0; k < m; ++k) s -= hess[a * nz + ny + k] * X[k * ny + b];
      Hs[a * ny + b] = s;
    }
  // Phi' = [[ Hs_{lambda,y} ], [ -Hs_{x,y} ]]
  for (int i = 0; i < n; ++i)
    for (int b = 0; b < ny; ++b) {
      dPhi[i * ny + b] = Hs[(n + i) * ny + b];
      dPhi[(n + i) * ny + b] = -Hs[i * ny + b];
    }
}

// gradient and Hessian of the final cost h at x
void terminal_derivs(const oracle_problem& p, const double* x, double* g, double* Hh) {
  const int n = p.n;
  HD xx[8];
  for (int a = 0; a < n; ++a)
    for (int b = a; b < n; ++b) {
      for (int c = 0; c < n; ++c) xx[c] = HD(x[c]);
      xx[a].e1 = 1.0;
      xx[b].e2 = 1.0;
      HD h = h_model(p, xx);
      Hh[a * n + b] = Hh[b * n + a] = h.e12;
      if (a == b) g[a] = h.e1;
    }
}

// ---------------------------------------------------------------------------
// Trapezoidal collocation of eq. hamchar on t_k = k T / N, k = 0..N.
// Unknown Y = (y_0, ..., y_N), y_k = (x_k, lambda_k).
// F = [ x_0 - xbar ;
//       y_k - y_{k-1} - (h/2)(Phi(y_{k-1}) + Phi(y_k)),  k = 1..N ;
//       lambda_N - (dh/dx)(x_N)^T ].
// ---------------------------------------------------------------------------
struct Collocation {
  const oracle_problem& p;
  int n, ny, N, dim;
  double hstep;
  std::vector<double> Phi, dPhi;  // per mesh point
  explicit Collocation(const oracle_problem& pp)
      : p(pp), n(pp.n), ny(2 * pp.n), N(pp.N), dim(2 * pp.n * (pp.N + 1)),
        hstep(pp.T / pp.N), Phi((size_t)ny * (N + 1)), dPhi((size_t)ny * ny * (N + 1)) {}
  int kl() const { return 3 * n - 1; }
  int ku() const { return 3 * n - 1; }
  const double* mesh_point(const double* Y, int k) const { return Y + (size_t)k * ny; }

  void eval_points(const double* Y, bool with_jac) {
    for (int k = 0; k <= N; ++k)
      phi_and_jacobian(p, Y + (size_t)k * ny, &Phi[(size_t)k * ny],
                       with_jac ? &dPhi[(size_t)k * ny * ny] : nullptr);
  }

  void residual(const double* xbar, const double* Y, double* F) {
    for (int i = 0; i < n; ++i) F[i] = Y[i] - xbar[i];
    for (int k = 1; k <= N; ++k) {
      const double* y0 = Y + (size_t)(k - 1) * ny;
      const double* y1 = Y + (size_t)k * ny;
      const double* P0 = &Phi[(size_t)(k - 1) * ny];
      const double* P1 = &Phi[(size_t)k * ny];
      double* Fk = F + n + (size_t)(k - 1) * ny;
      for (int i = 0; i < ny; ++i) Fk[i] = y1[i] - y0[i] - 0.5 * hstep * (P0[i] + P1[i]);
    }
    const double* yN = Y + (size_t)N * ny;
    double g[8], Hh[64];
    terminal_derivs(p, yN, g, Hh);
    double* FN = F + n + (size_t)N * ny;
    for (int i = 0; i < n; ++i) FN[i] = yN[n + i] - g[i];
  }

  // Entry (row, col) of F'(Y) for a row-block / column layout; calls back
  // set(row, col, value) for every structurally non-zero entry.
  template <class SetFn>
  void jacobian(const double* Y, SetFn set) {
    for (int i = 0; i < n; ++i) set(i, i, 1.0);  // d(x_0 - xbar)/dx_0
    for (int k = 1; k <= N; ++k) {
      const double* D0 = &dPhi[(size_t)(k - 1) * ny * ny];
      const double* D1 = &dPhi[(size_t)k * ny * ny];
      int row0 = n + (k - 1) * ny;
      int colA = (k - 1) * ny, colB = k * ny;
      for (int i = 0; i < ny; ++i)
        for (int j = 0; j < ny; ++j) {
          double dij = (i == j) ? 1.0 : 0.0;
          set(row0 + i, colA + j, -dij - 0.5 * hstep * D0[i * ny + j]);
          set(row0 + i, colB + j, dij - 0.5 * hstep * D1[i * ny + j]);
        }
    }
    const double* yN = Y + (size_t)N * ny;
    double g[8], Hh[64];
    terminal_derivs(p, yN, g, Hh);
    int rowN = n + N * ny, colN = N * ny;
    for (int i = 0; i < n; ++i) {
      for (int j = 0; j < n; ++j) set(rowN + i, colN + j, -Hh[i * n + j]);
      set(rowN + i, colN + n + i, 1.0);
    }
  }
};

// ---------------------------------------------------------------------------
// Four-point Lobatto IIIA collocation of eq. hamchar (the paper's BVP
// formula, Sec. 3.1 and Sec. 5.1) on t_k = k T / N.  On each interval the
// collocation points are t_k + c_j h, c = (0, (5 - sqrt 5)/10, (5 + sqrt 5)/10, 1);
// the stage values Z_{k,1} = y_k, Z_{k,2}, Z_{k,3}, Z_{k,4} = y_{k+1} satisfy
//   Z_{k,i} = y_k + h sum_j a_ij Phi(Z_{k,j}),  i = 2, 3, 4,
// with a_ij = integral from 0 to c_i of the Lagrange polynomial l_j on c (the
// collocation polynomial through the four points satisfies the ODE at each
// of them).  Unknowns: Y = (y_0, [Z_{k,2}, Z_{k,3}, y_{k+1}] for k = 0..N-1);
// F = [ x_0 - xbar ; the 3 x 2n stage equations of every interval ;
//       lambda_N - (dh/dx)(x_N)^T ].
// ---------------------------------------------------------------------------

// The Lobatto IIIA coefficients of the four-point formula from their
// definition: the Lagrange polynomials on c expanded in monomials and
// integrated term by term.
struct LobattoTableau {
  double c[4], a[4][4];
  LobattoTableau() {
    const double r5 = std::sqrt(5.0);
    c[0] = 0.0;
    c[1] = (5.0 - r5) / 10.0;
    c[2] = (5.0 + r5) / 10.0;
    c[3] = 1.0;
    for (int j = 0; j < 4; ++j) {
      double poly[4] = {1.0, 0.0, 0.0, 0.0};  // coefficients of s^0..s^3
      for (int m = 0; m < 4; ++m) {
        if (m == j) continue;
        const double den = c[j] - c[m];
        double next[4] = {0.0, 0.0, 0.0, 0.0};
        for (int e = 0; e < 3; ++e) {  // poly * (s - c_m) / (c_j - c_m)
          next[e + 1] += poly[e] / den;
          next[e] -= poly[e] * c[m] / den;
        }
        for (int e = 0; e < 4; ++e) poly[e] = next[e];
      }
      for (int i = 0; i < 4; ++i) {
        double v = 0.0, pw = c[i];
        for (int e = 0; e < 4; ++e) {
          v += poly[e] * pw / (e + 1);
          pw *= c[i];
        }
        a[i][j] = v;
      }
    }
  }
};

struct LobattoCollocation {
  const oracle_problem& p;
  int n, ny, N, dim;
  double hstep;
  LobattoTableau tab;
  std::vector<double> Phi, dPhi;  // per collocation point: y_k at 3k, Z_{k,2} at 3k+1, Z_{k,3} at 3k+2
  explicit LobattoCollocation(const oracle_problem& pp)
      : p(pp), n(pp.n), ny(2 * pp.n), N(pp.N), dim(2 * pp.n * (3 * pp.N + 1)), hstep(pp.T / pp.N),
        Phi((size_t)ny * (3 * N + 1)), dPhi((size_t)ny * ny * (3 * N + 1)) {}
  int kl() const { return 4 * ny - 1; }
  int ku() const { return 4 * ny - 1; }
  // offset in Y of collocation point q (= 3k + j - 1 for stage j of interval k)
  static size_t point(int q, int ny) { return (size_t)q * ny; }

  void eval_points(const double* Y, bool with_jac) {
    for (int q = 0; q <= 3 * N; ++q)
      phi_and_jacobian(p, Y + point(q, ny), &Phi[(size_t)q * ny], with_jac ? &dPhi[(size_t)q * ny * ny] : nullptr);
  }

  void residual(const double* xbar, const double* Y, double* F) {
    for (int i = 0; i < n; ++i) F[i] = Y[i] - xbar[i];
    for (int k = 0; k < N; ++k) {
      const double* yk = Y + point(3 * k, ny);
      for (int i = 1; i < 4; ++i) {
        const double* zi = Y + point(3 * k + i, ny);
        double* Fi = F + n + (size_t)(3 * k + i - 1) * ny;
        for (int r = 0; r < ny; ++r) {
          double s = 0.0;
          for (int j = 0; j < 4; ++j) s += tab.a[i][j] * Phi[(size_t)(3 * k + j) * ny + r];
          Fi[r] = zi[r] - yk[r] - hstep * s;
        }
      }
    }
    const double* yN = Y + point(3 * N, ny);
    double g[8], Hh[64];
    terminal_derivs(p, yN, g, Hh);
    double* FN = F + n + (size_t)3 * N * ny;
    for (int i = 0; i < n; ++i) FN[i] = yN[n + i] - g[i];
  }

  template <class SetFn>
  void jacobian(const double* Y, SetFn set) {
    for (int i = 0; i < n; ++i) set(i, i, 1.0);
    for (int k = 0; k < N; ++k)
      for (int i = 1; i < 4; ++i) {
        const int row0 = n + (3 * k + i - 1) * ny;
        for (int j = 0; j < 4; ++j) {
          const double* D = &dPhi[(size_t)(3 * k + j) * ny * ny];
          const int col0 = (3 * k + j) * ny;
          for (int r = 0; r < ny; ++r)
            for (int c = 0; c < ny; ++c) {
              double v = -hstep * tab.a[i][j] * D[r * ny + c];
              if (r == c && j == i) v += 1.0;
              if (r == c && j == 0) v -= 1.0;
              set(row0 + r, col0 + c, v);
            }
        }
      }
    const double* yN = Y + point(3 * N, ny);
    double g[8], Hh[64];
    terminal_derivs(p, yN, g, Hh);
    const int rowN = n + 3 * N * ny, colN = 3 * N * ny;
    for (int i = 0; i < n; ++i) {
      for (int j = 0; j < n; ++j) set(rowN + i, colN + j, -Hh[i * n + j]);
      set(rowN + i, colN + n + i, 1.0);
    }
  }

  // the mesh values y_k (rows of the trajectory) inside Y
  const double* mesh_point(const double* Y, int k) const { return Y + point(3 * k, ny); }
};

// Banded matrix with kl sub-diagonals and ku super-diagonals, stored by
// columns with kl extra super-diagonals for the fill-in of row pivoting:
// A(i,j) lives at ab[(kv + i - j) + j*ldab], kv = ku + kl.
struct Band {
  int n, kl, ku, kv, ldab;
  std::vector<double> ab;
  std::vector<int> piv;
  Band(int n_, int kl_, int ku_)
      : n(n_), kl(kl_), ku(ku_), kv(kl_ + ku_), ldab(2 * kl_ + ku_ + 1),
        ab((size_t)(2 * kl_ + ku_ + 1) * n_, 0.0), piv(n_) {}
  double& at(int i, int j) { return ab[(size_t)(kv + i - j) + (size_t)j * ldab]; }
  void clear() { std::fill(ab.begin(), ab.end(), 0.0); }

  // Gaussian elimination with row partial pivoting (first index of maximal
  // |a| in the column).  Returns false on an exactly zero pivot.
  bool factor() {
    for (int j = 0; j < n; ++j) {
      int last = std::min(n - 1, j + kl);
      int p = j;
      double best = std::fabs(at(j, j));
      for (int i = j + 1; i <= last; ++i) {
        double a = std::fabs(at(i, j));
        if (a > best) { best = a; p = i; }
      }
      piv[j] = p;
      if (at(p, j) == 0.0) return false;
      int cmax = std::min(n - 1, j + kv);
      if (p != j)
        for (int c = j; c <= cmax; ++c) std::swap(at(j, c), at(p, c));
      double d = at(j, j);
      for (int i = j + 1; i <= last; ++i) {
        double l = at(i, j) / d;
        at(i, j) = l;
        if (l != 0.0)
          for (int c = j + 1; c <= cmax; ++c) at(i, c) -= l * at(j, c);
      }
    }
    return true;
  }
  void solve(double* b) {
    for (int j = 0; j < n; ++j) {
      if (piv[j] != j) std::swap(b[j], b[piv[j]]);
      int last = std::min(n - 1, j + kl);
      for (int i = j + 1; i <= last; ++i) b[i] -= at(i, j) * b[j];
    }
    for (int j = n - 1; j >= 0; --j) {
      int cmax = std::min(n - 1, j + kv);
      double s = b[j];
      for (int c = j + 1; c <= cmax; ++c) s -= at(j, c) * b[c];
      b[j] = s / at(j, j);
    }
  }
};

bool all_finite(const double* a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

double max_abs(const double* a, size_t n) {
  double m = 0.0;
  for (size_t i = 0; i < n; ++i) m = std::max(m, std::fabs(a[i]));
  return m;
}

// Newton's method on F(Y) = 0 (see the file header for the rule).  Y must
// hold dim doubles; returns the status and writes the iteration count.
//
// Globalisation (the paper fixes none; Sec. 2 Assumption 1 only asks for a
// solution of the characteristic BVP): each counted Newton step d is damped by
// backtracking on the max-norm of the residual.  The trial points are
// Y + t d for t = 1, 1/2, ..., 2^-H (H = max_halvings); the first whose
// residual is finite and satisfies the sufficient-decrease test
//   max|F(Y + t d)| <= (1 - sigma t) max|F(Y)|,  sigma = 1e-4,
// is taken; if none does, the last trial (t = 2^-H) is taken.  So the full
// step is taken whenever it passes the test, and H = 0 is plain Newton.  The
// first step from Y = 0 (the solve of the linearised problem, the initial
// guess) is always taken in full.
constexpr double kArmijoSigma = 1e-4;

// Newton's iteration on F(Y) = 0.  from_zero: start at Y = 0 and take the
// first (uncounted) step in full; else start at the given Y with its test.
template <class Coll>
int newton_iterate(const oracle_problem& p, const double* xbar, double* Y, bool from_zero, int* iters_out,
                   double* fnorm_out) {
  Coll C(p);
  const int dim = C.dim;
  Band A(dim, C.kl(), C.ku());
  std::vector<double> F(dim), d(dim), Yt(dim), Ft(dim);
  // the Newton step d = -F'(Y)^{-1} F(Y); false on an exactly zero pivot
  auto newton_direction = [&]() -> bool {
    C.eval_points(Y, true);
    C.residual(xbar, Y, F.data());
    A.clear();
    C.jacobian(Y, [&](int i, int j, double v) { A.at(i, j) = v; });
    if (!A.factor()) return false;
    for (int i = 0; i < dim; ++i) d[i] = -F[i];
    A.solve(d.data());
    return true;
  };
  *fnorm_out = NAN;
  if (from_zero) {
    // the first step: the solve of the problem linearised about Y = 0
    std::fill(Y, Y + dim, 0.0);
    if (!newton_direction()) { *iters_out = 0; return ORC_SINGULAR; }
    for (int i = 0; i < dim; ++i) Y[i] += d[i];
  }
  for (int it = 0;; ++it) {
    C.eval_points(Y, false);
    C.residual(xbar, Y, F.data());
    *iters_out = it;
    if (!all_finite(F.data(), dim)) return ORC_NONFINITE;
    double fn = max_abs(F.data(), dim);
    *fnorm_out = fn;
    if (fn <= p.tol) return ORC_CONVERGED;
    if (it == p.max_iter) return ORC_MAXITER;
    if (!newton_direction()) return ORC_SINGULAR;
    double t = 1.0;
    for (int j = 0;; ++j) {
      for (int i = 0; i < dim; ++i) Yt[i] = Y[i] + t * d[i];
      if (j == p.max_halvings) break;  // the last trial is taken
      C.eval_points(Yt.data(), false);
      C.residual(xbar, Yt.data(), Ft.data());
      if (all_finite(Ft.data(), dim) && max_abs(Ft.data(), dim) <= (1.0 - kArmijoSigma * t) * fn) break;
      t *= 0.5;
    }
    std::copy(Yt.begin(), Yt.end(), Y);
  }
}

// Newton's iteration with the problem's collocation formula.
int newton_solve(const oracle_problem& p, const double* xbar, double* Y, bool from_zero, int* iters_out,
                 double* fnorm_out) {
  if (p.scheme == ORC_LOBATTO4) return newton_iterate<LobattoCollocation>(p, xbar, Y, from_zero, iters_out, fnorm_out);
  return newton_iterate<Collocation>(p, xbar, Y, from_zero, iters_out, fnorm_out);
}

// Number of unknowns of the collocation system of p.
int64_t collocation_dim(const oracle_problem& p) {
  return p.scheme == ORC_LOBATTO4 ? 2 * (int64_t)p.n * (3 * (int64_t)p.N + 1) : 2 * (int64_t)p.n * (p.N + 1);
}

// The characteristic BVP from xbar.  With two controls and continuation K > 0
// the linearisation about the origin loses a controllable direction (the
// torques span a plane), the linearised first step drifts along it, and
// Newton's iteration from there fails over most of the box.  The solution is
// then reached by continuation in the authority of a third, virtual torque
// along b3 = B_1 x B_2 / |B_1 x B_2|, the normal of that plane: stage k = 0..K-1
// solves the three-control problem with B_k = [B_1 B_2 s_k b3],
// s_k = 1 - k / K, the first from Y = 0 as above and each later one (and the
// final stage K, the two-control problem itself) from the solution of the one
// before.  The status is that of the last stage solved (a failed stage ends
// the continuation) and the iteration count is the total over the stages.
//
// Example III with K > 0 continues in the initial state instead: stage
// k = 1..K solves the BVP from (k / K) xbar, the first from Y = 0 and each
// later one from the solution of the one before (the corners of the box,
// where the linearised first step is far from the solution, converge this
// way); the same status and iteration rules.
int solve_bvp(const oracle_problem& p, const double* xbar, double* Y, int* iters_out, double* fnorm_out) {
  if (p.model == ORC_EXAMPLE3 && p.continuation > 0) {
    int total = 0, st = ORC_CONVERGED;
    for (int k = 1; k <= p.continuation; ++k) {
      const double s = (double)k / p.continuation;
      double xk[3];
      for (int i = 0; i < 3; ++i) xk[i] = s * xbar[i];
      int it = 0;
      st = newton_solve(p, xk, Y, k == 1, &it, fnorm_out);
      total += it;
      if (st != ORC_CONVERGED) break;
    }
    *iters_out = total;
    return st;
  }
  if (p.continuation <= 0 || p.m != 2) return newton_solve(p, xbar, Y, true, iters_out, fnorm_out);
  const double* B1 = p.B;
  const double* B2 = p.B + 3;
  double b3[3] = {B1[1] * B2[2] - B1[2] * B2[1], B1[2] * B2[0] - B1[0] * B2[2], B1[0] * B2[1] - B1[1] * B2[0]};
  const double nb = std::sqrt(b3[0] * b3[0] + b3[1] * b3[1] + b3[2] * b3[2]);
  for (double& v : b3) v /= nb;
  int total = 0, st = ORC_CONVERGED;
  for (int k = 0; k <= p.continuation; ++k) {
    oracle_problem q = p;
    if (k < p.continuation) {
      const double s = 1.0 - (double)k / p.continuation;
      q.m = 3;
      for (int i = 0; i < 3; ++i) q.B[6 + i] = s * b3[i];
    }
    int it = 0;
    st = newton_solve(q, xbar, Y, k == 0, &it, fnorm_out);
    total += it;
    if (st != ORC_CONVERGED) break;
  }
  *iters_out = total;
  return st;
}

// ---------------------------------------------------------------------------
// Sparse grid (Sec. 3.2) on the CGL family (eq. CGL).
// ---------------------------------------------------------------------------

int cgl_size(int i) { return i == 1 ? 1 : (1 << (i - 1)) + 1; }

// point k (1-based) of X^i, eq. CGL: (1 - cos((k-1) pi / 2^{i-1})) / 2
double cgl_point_formula(int i, int k) {
  if (i == 1) return 0.5;
  const double PI = 3.14159265358979323846;
  double n = std::ldexp(1.0, i - 1);
  return 0.5 * (1.0 - std::cos((k - 1) * PI / n));
}

// the same values, computed once per level (a lookup table of the formula)
constexpr int kMaxTableLevel = 12;
double cgl_point(int i, int k) {
  static const std::vector<std::vector<double>> table = [] {
    std::vector<std::vector<double>> t(kMaxTableLevel + 1);
    for (int lev = 1; lev <= kMaxTableLevel; ++lev)
      for (int kk = 1; kk <= cgl_size(lev); ++kk) t[lev].push_back(cgl_point_formula(lev, kk));
    return t;
  }();
  if (i > kMaxTableLevel) return cgl_point_formula(i, k);
  return table[i][k - 1];
}

// The 1-based indices k of the new points dX^i = X^i - X^{i-1} inside X^i.
// X^{i-1} sits in X^i at the even offsets k-1 (the angle (k-1) pi / 2^{i-1}
// with k-1 = 2k' equals k' pi / 2^{i-2}); for i = 2 the old point is the
// middle one (cos(pi/2) = 0 gives 1/2).
std::vector<int> new_point_indices(int i) {
  std::vector<int> ks;
  if (i == 1) { ks.push_back(1); return ks; }
  if (i == 2) { ks.push_back(1); ks.push_back(3); return ks; }
  for (int k = 2; k <= cgl_size(i); k += 2) ks.push_back(k);
  return ks;
}

// Integer identity of a 1-D grid point: points are numbered by the level at
// which they first appear and, within a level, by increasing coordinate:
// level 1 -> 0; level 2 -> 1 (x=0), 2 (x=1); level i>=3 -> 2^{i-2}+1 .. 2^{i-1}.
int point_id(int i, int k) {
  int t = k - 1;  // 0-based offset in X^i
  while (i > 2 && t % 2 == 0) { t /= 2; --i; }
  if (i == 1) return 0;
  if (i == 2) return t == 0 ? 1 : (t == 1 ? 0 : 2);
  return (1 << (i - 2)) + 1 + (t - 1) / 2;
}

// Lagrange basis on X^i for the point x^i_k (Sec. 3.3, product formula):
// prod_{m != k} (x - x^i_m) / (x^i_k - x^i_m).  X^1 has the constant 1.
double lagrange(int i, int k, double x) {
  if (i == 1) return 1.0;
  double xk = cgl_point(i, k), r = 1.0;
  for (int m = 1; m <= cgl_size(i); ++m) {
    if (m == k) continue;
    double xm = cgl_point(i, m);
    r *= (x - xm) / (xk - xm);
  }
  return r;
}

struct Node {
  std::vector<int> lev;  // i_1..i_d
  std::vector<int> k;    // 1-based index in X^{i_j}
  std::vector<int> key;  // point ids
  int levsum;
};

// The multi-indices i >= 1 with |i| <= q (lexicographic), by recursion.
void multi_indices(int d, int q, std::vector<std::vector<int>>& out) {
  std::vector<int> cur(d, 1);
  struct R {
    static void go(int dim, int d, int left, std::vector<int>& cur,
                   std::vector<std::vector<int>>& out) {
      if (dim == d) { out.push_back(cur); return; }
      int rest = d - dim - 1;  // each later dimension needs at least 1
      for (int v = 1; v <= left - rest; ++v) {
        cur[dim] = v;
        go(dim + 1, d, left - v, cur, out);
      }
    }
  };
  R::go(0, d, q, cur, out);
}

// G^q = union over |i| <= q of dX^{i_1} x ... x dX^{i_d}, q = level + d,
// in the canonical order: lexicographic order of the point-id tuples.
std::vector<Node> sparse_grid(int d, int level) {
  int q = level + d;
  std::vector<std::vector<int>> mis;
  multi_indices(d, q, mis);
  std::vector<Node> nodes;
  for (auto& mi : mis) {
    std::vector<std::vector<int>> ks(d);
    for (int j = 0; j < d; ++j) ks[j] = new_point_indices(mi[j]);
    std::vector<int> pos(d, 0);
    while (true) {
      Node nd;
      nd.lev = mi;
      nd.k.resize(d);
      nd.key.resize(d);
      nd.levsum = 0;
      for (int j = 0; j < d; ++j) {
        nd.k[j] = ks[j][pos[j]];
        nd.key[j] = point_id(mi[j], nd.k[j]);
        nd.levsum += mi[j];
      }
      nodes.push_back(nd);
      int j = d - 1;
      while (j >= 0 && ++pos[j] == (int)ks[j].size()) { pos[j] = 0; --j; }
      if (j < 0) break;
    }
  }
  std::sort(nodes.begin(), nodes.end(),
            [](const Node& a, const Node& b) { return a.key < b.key; });
  return nodes;
}

// tensor product of the hierarchical basis functions of a node at xi
double node_basis(const Node& nd, const double* xi, int d) {
  double r = 1.0;
  for (int j = 0; j < d; ++j) r *= lagrange(nd.lev[j], nd.k[j], xi[j]);
  return r;
}

double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

template <class Coll>
void residual_of(const oracle_problem* p, int64_t nb, const double* xbar, const double* Y, double* F,
                 int nthreads) {
  const int n = p->n;
  const int64_t dim = collocation_dim(*p);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int64_t b = 0; b < nb; ++b) {
    Coll C(*p);
    C.eval_points(Y + b * dim, false);
    C.residual(xbar + b * n, Y + b * dim, F + b * dim);
  }
}

template <class Coll>
void jacobian_dense_of(const oracle_problem* p, const double* Y, double* Jd) {
  Coll C(*p);
  const int dim = C.dim;
  std::fill(Jd, Jd + (size_t)dim * dim, 0.0);
  C.eval_points(Y, true);
  C.jacobian(Y, [&](int i, int j, double v) { Jd[(size_t)i * dim + j] = v; });
}

}  // namespace

// ===========================================================================
// Exported C ABI of the oracle (ctypes).
// ===========================================================================
extern "C" {

// characteristic right-hand side and its Jacobian at npts points y (2n each)
void oracle_phi(const oracle_problem* p, int64_t npts, const double* y, double* Phi,
                double* dPhi /* may be null */) {
  const int ny = 2 * p->n;
  for (int64_t i = 0; i < npts; ++i)
    phi_and_jacobian(*p, y + i * ny, Phi + i * ny, dPhi ? dPhi + i * ny * ny : nullptr);
}

void oracle_ustar(const oracle_problem* p, int64_t npts, const double* y, double* u) {
  for (int64_t i = 0; i < npts; ++i) ustar(*p, y + i * 2 * p->n, u + i * p->m);
}

// collocation residual F(Y) for given trajectories (nb of them)
// the four-point Lobatto IIIA tableau: nodes c (4) and coefficients a (4 x 4)
void oracle_lobatto_tableau(double* c, double* a) {
  LobattoTableau t;
  for (int i = 0; i < 4; ++i) {
    c[i] = t.c[i];
    for (int j = 0; j < 4; ++j) a[i * 4 + j] = t.a[i][j];
  }
}

// number of unknowns (and of residual entries) of the collocation system
int64_t oracle_collocation_dim(const oracle_problem* p) { return collocation_dim(*p); }

// collocation residual F(Y) of nb unknown vectors Y (nb x dim)
void oracle_residual(const oracle_problem* p, int64_t nb, const double* xbar, const double* Y,
                     double* F, int nthreads) {
  if (p->scheme == ORC_LOBATTO4)
    residual_of<LobattoCollocation>(p, nb, xbar, Y, F, nthreads);
  else
    residual_of<Collocation>(p, nb, xbar, Y, F, nthreads);
}

// dense Jacobian F'(Y) (dim x dim row-major) for small meshes
void oracle_jacobian_dense(const oracle_problem* p, const double* Y, double* Jd) {
  if (p->scheme == ORC_LOBATTO4)
    jacobian_dense_of<LobattoCollocation>(p, Y, Jd);
  else
    jacobian_dense_of<Collocation>(p, Y, Jd);
}

// Solve nb BVPs from initial states x0 (nb x n).  Outputs (any may be null):
// lambda0 (nb x n), u0 (nb x m), V (nb), traj (nb x (N+1) x 2n, the mesh
// values), status, iters, fnorm (final max|F|), unknowns (nb x dim: the whole
// unknown vector, with the Lobatto interior stages).
void oracle_solve_bvps_full(const oracle_problem* p, int64_t nb, const double* x0, double* lambda0,
                            double* u0, double* V, double* traj, int32_t* status, int32_t* iters,
                            double* fnorm, double* unknowns, int nthreads) {
  const int n = p->n, m = p->m, ny = 2 * n, N = p->N;
  const int64_t dim = collocation_dim(*p);
  const bool lob = p->scheme == ORC_LOBATTO4;
  const int pts = lob ? 3 : 1;  // collocation points per interval in Y
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int64_t b = 0; b < nb; ++b) {
    std::vector<double> Y(dim);
    int it = 0;
    double fn = 0.0;
    int st = solve_bvp(*p, x0 + b * n, Y.data(), &it, &fn);
    if (status) status[b] = st;
    if (iters) iters[b] = it;
    if (fnorm) fnorm[b] = fn;
    if (lambda0)
      for (int i = 0; i < n; ++i) lambda0[b * n + i] = Y[n + i];
    if (u0) ustar(*p, Y.data(), u0 + b * m);
    if (V) {
      // z(T) by the formula's quadrature on the mesh (the trapezoidal rule,
      // or the Lobatto weights b_j = a_4j over the four points of each
      // interval), plus h(x(T))  (eq. optuv)
      const double hstep = p->T / N;
      double z = 0.0;
      if (lob) {
        LobattoTableau tab;
        for (int k = 0; k < N; ++k)
          for (int j = 0; j < 4; ++j) {
            const double* yq = &Y[(size_t)(3 * k + j) * ny];
            double u[3];
            ustar(*p, yq, u);
            z += hstep * tab.a[3][j] * L_model(*p, yq, u);
          }
      } else {
        double Lprev = 0.0;
        for (int k = 0; k <= N; ++k) {
          double u[3];
          ustar(*p, &Y[(size_t)k * ny], u);
          double Lk = L_model(*p, &Y[(size_t)k * ny], u);
          if (k > 0) z += 0.5 * hstep * (Lprev + Lk);
          Lprev = Lk;
        }
      }
      V[b] = z + h_model(*p, &Y[(size_t)pts * N * ny]);
    }
    if (traj)
      for (int k = 0; k <= N; ++k)
        std::memcpy(traj + (b * (N + 1) + k) * ny, &Y[(size_t)pts * k * ny], sizeof(double) * ny);
    if (unknowns) std::memcpy(unknowns + b * dim, Y.data(), sizeof(double) * dim);
  }
}

void oracle_solve_bvps(const oracle_problem* p, int64_t nb, const double* x0, double* lambda0,
                       double* u0, double* V, double* traj, int32_t* status, int32_t* iters,
                       double* fnorm, int nthreads) {
  oracle_solve_bvps_full(p, nb, x0, lambda0, u0, V, traj, status, iters, fnorm, nullptr, nthreads);
}

// ---- sparse grid ----------------------------------------------------------

int64_t oracle_grid_size(int d, int level) { return (int64_t)sparse_grid(d, level).size(); }

// nodes (M x d) mapped affinely from [0,1]^d to the box [lo, hi]; keys (M x d)
// point ids; levels (M x d) the multi-index of each node.  Any may be null.
int64_t oracle_grid(int d, int level, const double* lo, const double* hi, double* nodes,
                    double* xi, int32_t* keys, int32_t* levels) {
  std::vector<Node> g = sparse_grid(d, level);
  for (size_t a = 0; a < g.size(); ++a)
    for (int j = 0; j < d; ++j) {
      double s = cgl_point(g[a].lev[j], g[a].k[j]);
      if (xi) xi[a * d + j] = s;
      if (nodes) nodes[a * d + j] = lo[j] + (hi[j] - lo[j]) * s;
      if (keys) keys[a * d + j] = g[a].key[j];
      if (levels) levels[a * d + j] = g[a].lev[j];
    }
  return (int64_t)g.size();
}

// 1-D Lagrange basis u^i_k(x) on X^i (k 1-based) at nx points
void oracle_lagrange(int i, int k, int64_t nx, const double* x, double* out) {
  for (int64_t a = 0; a < nx; ++a) out[a] = lagrange(i, k, x[a]);
}

void oracle_cgl_points(int i, double* out) {
  for (int k = 1; k <= cgl_size(i); ++k) out[k - 1] = cgl_point(i, k);
}

// Hierarchical surpluses by the level recursion of eq. interpo:
// I^{d-1} = 0; for |i| = d..q: w = f(node) - I^{|i|-1}(f)(node).
// values and surplus are M x m in canonical order.
void oracle_build_surplus(int d, int level, int m, const double* values, double* surplus,
                          int nthreads) {
  std::vector<Node> g = sparse_grid(d, level);
  const int64_t M = (int64_t)g.size();
  int q = level + d;
  std::vector<double> xi((size_t)M * d);
  for (int64_t a = 0; a < M; ++a)
    for (int j = 0; j < d; ++j) xi[a * d + j] = cgl_point(g[a].lev[j], g[a].k[j]);
  for (int l = d; l <= q; ++l) {
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
    for (int64_t a = 0; a < M; ++a) {
      if (g[a].levsum != l) continue;
      for (int c = 0; c < m; ++c) surplus[a * m + c] = values[a * m + c];
      for (int64_t b = 0; b < M; ++b) {
        if (g[b].levsum >= l) continue;
        double phi = node_basis(g[b], &xi[a * d], d);
        for (int c = 0; c < m; ++c) surplus[a * m + c] -= surplus[b * m + c] * phi;
      }
    }
  }
}

// Route A: I^q(f)(x) = sum over nodes of w * prod_j a^{i_j}_{k_j}(xi_j) at
// query points x (nq x d) in box coordinates.
void oracle_eval_hier(int d, int level, int m, const double* lo, const double* hi,
                      const double* surplus, int64_t nq, const double* xq, double* out,
                      int nthreads) {
  std::vector<Node> g = sparse_grid(d, level);
  const int64_t M = (int64_t)g.size();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
  for (int64_t a = 0; a < nq; ++a) {
    double xi[16], acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int j = 0; j < d; ++j) xi[j] = (xq[a * d + j] - lo[j]) / (hi[j] - lo[j]);
    for (int64_t b = 0; b < M; ++b) {
      double phi = node_basis(g[b], xi, d);
      for (int c = 0; c < m; ++c) acc[c] += surplus[b * m + c] * phi;
    }
    for (int c = 0; c < m; ++c) out[a * m + c] = acc[c];
  }
}

// Route B: the combination formula eq. interpolation2,
// I^q(f) = sum_{q-d+1 <= |i| <= q} (-1)^{q-|i|} C(d-1, q-|i|) U^{i_1} x..x U^{i_d}(f),
// with the full tensor Lagrange interpolants on X^{i_1} x .. x X^{i_d}; it
// reads the node values directly (every tensor point is a sparse-grid node).
void oracle_eval_comb(int d, int level, int m, const double* lo, const double* hi,
                      const double* values, int64_t nq, const double* xq, double* out,
                      int nthreads) {
  std::vector<Node> g = sparse_grid(d, level);
  std::map<std::vector<int>, int64_t> index;
  for (size_t a = 0; a < g.size(); ++a) index[g[a].key] = (int64_t)a;
  int q = level + d;
  std::vector<std::vector<int>> mis;
  multi_indices(d, q, mis);
  struct Term { std::vector<int> mi; double coef; };
  std::vector<Term> terms;
  for (auto& mi : mis) {
    int s = 0;
    for (int v : mi) s += v;
    if (s < q - d + 1) continue;
    double c = binom(d - 1, q - s) * (((q - s) % 2) ? -1.0 : 1.0);
    terms.push_back({mi, c});
  }
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
  for (int64_t a = 0; a < nq; ++a) {
    double xi[16], acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int j = 0; j < d; ++j) xi[j] = (xq[a * d + j] - lo[j]) / (hi[j] - lo[j]);
    for (auto& t : terms) {
      // all tensor points of X^{i_1} x ... x X^{i_d}
      std::vector<int> kk(d, 1), key(d);
      while (true) {
        double phi = t.coef;
        for (int j = 0; j < d; ++j) {
          phi *= lagrange(t.mi[j], kk[j], xi[j]);
          key[j] = point_id(t.mi[j], kk[j]);
        }
        int64_t node = index.at(key);
        for (int c = 0; c < m; ++c) acc[c] += values[node * m + c] * phi;
        int j = d - 1;
        while (j >= 0 && ++kk[j] > cgl_size(t.mi[j])) { kk[j] = 1; --j; }
        if (j < 0) break;
      }
    }
    for (int c = 0; c < m; ++c) out[a * m + c] = acc[c];
  }
}

}  // extern "C"

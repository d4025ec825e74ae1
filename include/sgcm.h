/*
 * sgcm.h -- C ABI of the MI355X (gfx950) sparse grid characteristics method.
 *
 * The method (Kang & Wilcox, "Mitigating the Curse of Dimensionality: Sparse
 * Grid Characteristics Method for Optimal Feedback Control and HJB
 * Equations") solves, independently at every node of a Smolyak sparse grid,
 * the two-point boundary value problem of the characteristics (state and
 * costate equations, Sec. 3.1, eq. hamchar), builds the hierarchical-surplus
 * polynomial interpolant of the result on the Clenshaw-Curtis ("CGL") sparse
 * grid (Sec. 3.2 eq. CGL, Sec. 3.3 eq. interpo), and evaluates the feedback
 * law at arbitrary states (Sec. 3.3, Steps I-III and the on-line step).  It
 * also estimates the interpolant's total error at sample states against more
 * accurate BVP solutions (Sec. 4.3).
 *
 * Conventions for every function:
 *   - All functions are extern "C", never throw, and return an int status
 *     (sgcm_err) unless stated otherwise.
 *   - Arguments are validated before any GPU work is queued; a bad argument
 *     returns SGCM_EINVAL and queues nothing.  A failed launch or runtime call
 *     returns SGCM_EDEVICE.
 *   - Pointers documented as "device" must point to device memory of the
 *     current HIP device (or be NULL where allowed).  The caller owns every
 *     device buffer and the stream; the library owns only sgcm_grid,
 *     sgcm_plan and sgcm_batch objects.
 *   - Calls on a stream are stream-ordered and do not synchronise the host.
 *     "stream" is a hipStream_t passed as void*; NULL means the null stream.
 *   - Arrays are row-major and densely packed unless stated otherwise.
 */
#ifndef SGCM_H
#define SGCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
typedef enum {
  SGCM_OK = 0,
  SGCM_EINVAL = -1,       /* invalid argument (nothing was queued)            */
  SGCM_ENOMEM = -2,       /* host or device allocation failed                 */
  SGCM_EDEVICE = -3,      /* HIP launch or runtime failure                    */
  SGCM_EUNSUPPORTED = -4, /* valid request outside what the library supports */
  SGCM_ENOTCONVERGED = -5 /* node values from a BVP that did not converge: the
                             interpolant is not built (reported by the Python
                             binding, which checks the statuses of a solve
                             before it builds from its outputs)              */
} sgcm_err;

/* Per-BVP outcome written to status[] by sgcm_solve_bvps.  A per-BVP failure
 * is not a call error: the call still returns SGCM_OK. */
typedef enum {
  SGCM_BVP_CONVERGED = 0, /* max|F| <= tol                                    */
  SGCM_BVP_MAXITER = 1,   /* max_iter Newton iterations without convergence   */
  SGCM_BVP_SINGULAR = 2,  /* an exactly zero pivot in the Newton linear solve */
  SGCM_BVP_NONFINITE = 3  /* a NaN or Inf in the collocation residual         */
} sgcm_bvp_status;

/* Dynamics of the optimal-control problem (Sec. 2).  Both use the state
 * x = (phi, theta, psi, w1, w2, w3): Euler angles in (3,2,1) order and body
 * rates (Sec. 5, eq. sat_model with the stored-momentum term replaced by the
 * gyroscopic term).
 *   RIGID_BODY:  v' = E(v) w,  J w' = -w x (J w) + B u, with
 *                E(v) = [[1, s_phi t_th, c_phi t_th], [0, c_phi, -s_phi],
 *                        [0, s_phi/c_th, c_phi/c_th]].
 *   LINEARISED:  the same system linearised about x = 0: v' = w, J w' = B u
 *                (used to pin the solver by the Riccati closed form). */
typedef enum {
  SGCM_MODEL_RIGID_BODY = 0,
  SGCM_MODEL_LINEARISED = 1,
  /* Example III (Sec. 5.3): n = 3, m = 1,
   *   x1' = -x1 + x2,  x2' = -x2 + g,  x3' = (q + 2 x2 g) g + s u,
   *   cost 0.5 * integral of (g^2 + u^2) dt, no final cost,
   * with s = 1 + x1^2 + x2^2, g = x3 / s, q = -2 x1^2 + 2 x1 x2 - 2 x2^2;
   * u* = -s lambda3.  J, B, q_w, r_w and p_w are ignored.  FP64 and the
   * trapezoid only; no plans or batches (SGCM_EUNSUPPORTED).  Continuation
   * K > 0 runs in the initial state: stage k = 1..K solves the BVP from
   * (k / K) x0, the first from the zero trajectory and each later one from
   * the previous stage's solution (Newton's iteration from the linearised
   * step stalls at corners of the box for some horizons); statuses and
   * iteration counts as for the two-control continuation.  x0 and lambda0
   * have 3 columns, u0 one, traj (N+1) x 6.  With the time variable as a
   * grid dimension see sgcm_solve_bvps_tx. */
  SGCM_MODEL_EXAMPLE3 = 2
} sgcm_model;

typedef enum { SGCM_FP64 = 0, SGCM_FP32 = 1 } sgcm_precision;

/* Collocation formula of the BVP (both members of the Lobatto IIIA family):
 *   SGCM_TRAPEZOID  the two-point formula, y_k - y_{k-1} = (h/2)(Phi_{k-1} + Phi_k),
 *                   second order;
 *   SGCM_LOBATTO4   the four-point formula the paper solves its BVPs with
 *                   (Sec. 3.1, Sec. 5.1): on each interval the collocation
 *                   points t_k + c_j h, c = (0, (5 - sqrt 5)/10, (5 + sqrt 5)/10, 1),
 *                   two interior stages per interval, order 6 at the mesh
 *                   points; the error is controlled by the caller by mesh
 *                   doubling (the difference of the solutions on N and 2N
 *                   intervals estimates 63/64 of the coarse one's error).
 *                   FP64 only; no plans or batches (SGCM_EUNSUPPORTED). */
typedef enum { SGCM_TRAPEZOID = 0, SGCM_LOBATTO4 = 1 } sgcm_scheme;

/* The optimal-control problem of Sec. 2 and its discretisation.
 * Cost: integral over [0,T] of 0.5 (q_w x^T x + r_w u^T u) dt
 *       + 0.5 p_w x(T)^T x(T).
 * Discretisation: collocation by the problem's scheme (trapezoid: the
 * two-point Lobatto IIIA formula; or the four-point formula, see
 * sgcm_scheme) on N uniform intervals of [0, T]; Newton's method from the zero
 * trajectory; its first step, the solve of the problem linearised about the
 * origin (the LQR initial guess), is not counted and is taken in full; then
 * at iteration it = 0, 1, ...: NONFINITE if the residual F is not finite,
 * CONVERGED if max|F| <= tol, MAXITER if it == max_iter, else a damped Newton
 * step Y + t d: the first of t = 1, 1/2, ..., 2^-H whose residual is finite
 * and satisfies max|F(Y + t d)| <= (1 - 1e-4 t) max|F(Y)|, else t = 2^-H
 * (the full step whenever it passes; H = 0 is plain Newton).  The paper fixes
 * no solver internals (Sec. 3.1); this globalisation is the library's.
 * Continuation (two controls, K > 0): the linearisation about the origin of
 * a two-torque body loses a controllable direction (the torques span a
 * plane), and Newton's iteration from its solution fails over most of a box
 * of initial states.  The BVP is then solved in K + 1 stages: stage
 * k = 0..K-1 solves the three-control problem with B_k = [B_1 B_2 s_k b3],
 * s_k = 1 - k / K, b3 = B_1 x B_2 / |B_1 x B_2| (a virtual torque normal to the
 * plane, of decreasing authority), the first stage from the zero trajectory
 * as above and each later stage, and the final stage K (the problem itself),
 * from the previous stage's solution, starting with its test.  A stage that
 * does not converge ends the continuation with its status; iters is the
 * total over the stages and max_iter applies to each. */
typedef struct sgcm_problem {
  int32_t model;     /* sgcm_model                                            */
  int32_t n;         /* state dimension: 6 (3 for SGCM_MODEL_EXAMPLE3)        */
  int32_t m;         /* number of controls: 1, 2 or 3                         */
  double J[3];       /* diagonal of the inertia matrix, all > 0               */
  double B[9];       /* 3 x m input matrix, column-major: B[i + 3*j]          */
  double q_w;        /* running state weight   (>= 0)                         */
  double r_w;        /* running control weight (> 0)                          */
  double p_w;        /* final state weight     (>= 0)                         */
  double T;          /* horizon (> 0)                                         */
  int32_t N;         /* number of mesh intervals, 1 <= N <= 65536             */
  double tol;        /* Newton tolerance on max|F| (>= 0)                     */
  int32_t max_iter;  /* Newton iterations after the first step, 0..1000       */
  int32_t precision; /* sgcm_precision of the Newton linear solve: SGCM_FP64,
                        or SGCM_FP32 for the inexact Newton whose linear solve
                        runs in FP32 while the residual, the update and the
                        stopping test stay FP64                               */
  int32_t max_halvings; /* backtracking cap H of each counted Newton step,
                        0..60 (0: full steps; see below)                      */
  int32_t continuation; /* two controls: K > 0 continuation stages (0..64; see
                        below); ignored for one or three controls; for
                        SGCM_MODEL_EXAMPLE3 stages in the initial state    */
  int32_t scheme;    /* sgcm_scheme of the collocation                       */
  int32_t sweep_batch;   /* tile of the trapezoidal solve: intervals per
                        backward-sweep batch, 8, 10, 12 or 16 (0: 8)         */
  int32_t forward_chunk; /* tile of the trapezoidal solve: intervals per
                        forward-pass chunk, 8 or 12 (0: 12).  The tiles
                        change only the time, never a result (bit for bit);
                        other values return SGCM_EUNSUPPORTED; the
                        four-point formula ignores them                     */
} sgcm_problem;

/* ---- library ------------------------------------------------------------- */

/* Static message for a status code; never NULL. */
const char* sgcm_strerror(int code);

/* ABI version (major * 10000 + minor * 100 + patch). */
int sgcm_version(void);

/* ---- characteristic BVP (Sec. 3.1, eq. hamchar and eq. optuv) -------------- */

/* Bytes of device workspace sgcm_solve_bvps needs for n_bvps problems
 * (written to *bytes).  Returns SGCM_EINVAL for an invalid problem. */
int sgcm_solve_bvps_workspace(const sgcm_problem* p, int64_t n_bvps, size_t* bytes);

/* Solve the characteristic BVP of eq. hamchar from every initial state:
 *   x' = (dH/dlambda)^T,  lambda' = -(dH/dx)^T  at u* = argmin_u H,
 *   x(0) = x0,  lambda(T) = (dh/dx)^T(x(T)),
 * with H = L + lambda^T f and, for the models here,
 * u* = -(1/r_w) B^T J^{-1} lambda_w.  Outputs follow eq. optuv at t = 0.
 *   x0       device, n_bvps x 6 initial states (read only)
 *   lambda0  device, n_bvps x 6: the costate lambda(0)
 *   u0       device, n_bvps x m: the feedback u*(0, x0) = u*(x0, lambda(0))
 *   V        device, n_bvps, or NULL: the cost z(T) + h(x(T)), z integrated
 *            by the scheme's quadrature on the mesh (the trapezoidal rule, or
 *            the Lobatto weights over each interval's four points)
 *   traj     device, n_bvps x (N+1) x 12, or NULL: (x_k, lambda_k), t_k = kT/N
 *            (the mesh values; not the interior Lobatto stages)
 *   status   device, n_bvps (sgcm_bvp_status)
 *   iters    device, n_bvps: Newton iterations after the first step
 *   workspace, ws_bytes: device scratch of at least
 *            sgcm_solve_bvps_workspace() bytes, 256-byte aligned; its
 *            contents on entry are ignored.
 * n_bvps == 0 is a valid no-op.  Outputs of a non-converged BVP are those of
 * the last iterate.  The call is stream-ordered on `stream`.  For
 * n_bvps <= 4096 the BVPs are handed to workgroups in decreasing order of
 * |x0|_1 (a predictor of their Newton iterations, so that the longest start
 * first); each BVP's outputs do not depend on that order.
 * First steps: the first Newton step is linear in the initial state (the
 * residual at Y = 0 is [-x0; 0; 0] and the Jacobian does not depend on x0).
 * With the trapezoid and n_bvps >= 64 the call therefore computes the first
 * steps of the six unit initial states first, in the workspace (at Y = 0
 * every interval has the same equations, so they are made by doubling, in
 * about log2 N dependent steps), and forms every BVP's step as their
 * combination; the results are those of sgcm_solve_bvps_plan with a plan of
 * the same problem, bit for bit, and differ from a BVP's own first step by
 * rounding only.  If those six steps are not finite (a singular linearised
 * system), every BVP takes its own. */
int sgcm_solve_bvps(const sgcm_problem* p, int64_t n_bvps, const double* x0,
                    double* lambda0, double* u0, double* V, double* traj,
                    int32_t* status, int32_t* iters, void* workspace,
                    size_t ws_bytes, void* stream);

/* The time variable as a dimension of the sparse grid (Sec. 3.3 after
 * Steps I-III; Sec. 5.3): the characteristic BVPs from the points
 * (t0, x0) of a grid in (t, x), each over [t0, T] with x(t0) = x0 and the
 * final condition at T = p->T, on p->N uniform intervals of [t0, T].  For the
 * autonomous models here this is the BVP of the horizon T - t0 from x0, so
 * V(t0, x0), lambda(t0) and u*(t0, x0) are the values from which the (t, x)
 * interpolant of the value function and of the feedback is built (with
 * sgcm_build_interpolant on the grid in (t, x)).
 *   tx       device, n_bvps x (1 + n): rows (t0, x0), t0 <= T; a row with
 *            t0 > T or a non-finite t0 gets SGCM_BVP_NONFINITE
 *   (other arguments, workspace and outputs as for sgcm_solve_bvps; the
 *   outputs are at t0, and traj holds the mesh values of [t0, T])
 * A row with t0 = T is the final condition itself (lambda = 0, V = 0 for
 * Example III): the mesh has zero width and the first step solves it.
 * Supported for SGCM_MODEL_EXAMPLE3 (others: SGCM_EUNSUPPORTED). */
int sgcm_solve_bvps_tx(const sgcm_problem* p, int64_t n_bvps, const double* tx, double* lambda0, double* u0,
                       double* V, double* traj, int32_t* status, int32_t* iters, void* workspace,
                       size_t ws_bytes, void* stream);

/* Device scratch, in bytes, that the library holds per device for
 * sgcm_solve_bvps_static. */
#define SGCM_STATIC_SCRATCH_BYTES (64u << 20)

/* sgcm_solve_bvps without a workspace argument and without any allocation,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * workspace is a device array of SGCM_STATIC_SCRATCH_BYTES that the library
 * holds on each device it runs on until the process ends (its address is
 * looked up on the first call on a device).  A call whose workspace
 * (sgcm_solve_bvps_workspace of the same problem and count) exceeds it
 * returns SGCM_EUNSUPPORTED before any device work: at N = 256 that allows
 * about 180 BVPs per call.  Arguments, outputs and the other errors as for
 * sgcm_solve_bvps.  Every call on a device uses the same array: calls that
 * overlap on one device (other streams, other threads) race and give wrong
 * results; order them.  No part of the array needs clearing between calls
 * (the solver ignores the workspace's contents on entry). */
int sgcm_solve_bvps_static(const sgcm_problem* p, int64_t n_bvps, const double* x0, double* lambda0,
                           double* u0, double* V, double* traj, int32_t* status, int32_t* iters,
                           void* stream);

/* The right-hand side of eq. hamchar at n_points states y = (x, lambda) and
 * its Jacobian (the per-mesh-point blocks the Newton solve is built from):
 *   y     device, n_points x 12
 *   phi   device, n_points x 12:  [ f(x, u*) ; -(dH/dx)^T(x, lambda, u*) ]
 *   dphi  device, n_points x 12 x 12 (row-major d phi_i / d y_j), or NULL. */
int sgcm_characteristic_rhs(const sgcm_problem* p, int64_t n_points, const double* y,
                            double* phi, double* dphi, void* stream);

/* ---- solve plans: the first Newton step by superposition --------------- */

/* Newton's iteration starts with one step from Y = 0: the collocation
 * solution of the BVP of eq. hamchar linearised about the origin (the initial
 * guess).  For both models the right-hand side vanishes at the origin, so at
 * Y = 0 the residual is [-x0; 0; 0] and the Jacobian does not depend on x0:
 * that step is linear in x0, Y1(x0) = sum_j x0_j Y1(e_j).  A plan holds the
 * problem and the steps Y1(e_j) of the six unit initial states, and
 * sgcm_solve_bvps_plan forms each BVP's first step from them instead of
 * solving it: the same iterates as sgcm_solve_bvps up to rounding, with one
 * serial linear solve fewer per BVP. */
typedef struct sgcm_plan sgcm_plan;

/* Create a plan for problem p (copied).  The six steps are computed on `stream`
 * in FP64 whatever p->precision (which applies to the solves with the plan),
 * and the call synchronizes the stream.  With continuation they are the first
 * steps of its first stage.  On success *out owns 6 x (N+1) x 12
 * doubles of device memory on the current device.  Returns SGCM_EINVAL for an
 * invalid problem or out == NULL, SGCM_ENOMEM, SGCM_EDEVICE, and
 * SGCM_EUNSUPPORTED when the linearised step is not finite (a singular
 * linearised system; then sgcm_solve_bvps reports that per BVP). */
int sgcm_plan_create(const sgcm_problem* p, void* stream, sgcm_plan** out);

/* sgcm_solve_bvps for the plan's problem, each BVP's first Newton step formed
 * from the plan.  Arguments, workspace (sgcm_solve_bvps_workspace of the
 * plan's problem), outputs and errors as for sgcm_solve_bvps; SGCM_EINVAL
 * also when the current device is not the plan's.  The plan is only read:
 * calls with one plan may run concurrently. */
int sgcm_solve_bvps_plan(const sgcm_plan* plan, int64_t n_bvps, const double* x0,
                         double* lambda0, double* u0, double* V, double* traj,
                         int32_t* status, int32_t* iters, void* workspace,
                         size_t ws_bytes, void* stream);

void sgcm_plan_destroy(sgcm_plan* plan);

/* ---- batches of BVPs with mixed meshes and horizons --------------------- */

/* Plan for n_bvps BVPs of one problem whose mesh size N and horizon T differ
 * per BVP (the problem's own N and T are ignored).  The plan holds device
 * tables (per-BVP N and mesh width, workspace offsets, the processing order
 * and a work counter) on the device current at creation, so that
 * sgcm_solve_bvps_batch allocates nothing and can be captured in a HIP graph.
 * Created and destroyed on the host; not thread-safe to use concurrently on
 * two streams (the persistent schedule shares one counter). */
typedef struct sgcm_batch sgcm_batch;

/* Schedule of a batch:
 *   order:        0 = BVPs in the given order; 1 = larger N * T first
 *   slots_per_cu: 0 = one workgroup per BVP; 1..8 = one persistent launch of
 *                 slots_per_cu workgroups per compute unit, each taking the
 *                 next BVP of the order from a device work counter. */
typedef struct sgcm_schedule {
  int32_t order;
  int32_t slots_per_cu;
} sgcm_schedule;

/* N, T: host arrays of n_bvps (>= 1) mesh sizes (1..65536) and horizons
 * (finite, > 0); sched: NULL for {order 1, slots_per_cu 0}.  A problem with
 * continuation stages returns SGCM_EUNSUPPORTED (a batch is one launch).  Like a solve
 * plan, the batch forms each BVP's first Newton step from the first steps of
 * the six unit initial states of its (N, T), for every (N, T) shared by at
 * least 8 BVPs: creation solves those (FP64, one small launch per such
 * (N, T) on the null stream, synchronized); the other BVPs, and a group
 * whose linearised step is singular or not finite, solve their own first
 * steps.  On success *out owns device memory of about 32 bytes per BVP and
 * 6 x (N+1) x 12 doubles per such (N, T), on the current device. */
int sgcm_batch_create(const sgcm_problem* p, int64_t n_bvps, const int32_t* N, const double* T,
                      const sgcm_schedule* sched, sgcm_batch** out);

/* Bytes of device workspace sgcm_solve_bvps_batch needs. */
int sgcm_batch_workspace(const sgcm_batch* b, size_t* bytes);

/* Solve every BVP of the plan from x0 (device, n_bvps x 6); outputs as in
 * sgcm_solve_bvps (lambda0 n x 6, u0 n x m, V n or NULL, status n, iters n,
 * indexed in the given order), without trajectories.  workspace: at least
 * sgcm_batch_workspace() bytes, 256-byte aligned.  Must be called with the
 * plan's device current.  Results do not depend on the schedule. */
int sgcm_solve_bvps_batch(const sgcm_batch* b, const double* x0, double* lambda0, double* u0,
                          double* V, int32_t* status, int32_t* iters, void* workspace,
                          size_t ws_bytes, void* stream);

void sgcm_batch_destroy(sgcm_batch* b);

/* ---- sparse grid (Sec. 3.2) --------------------------------------------- */

/* Opaque grid: the Smolyak sparse grid G^q = U_{|i| <= q} dX^{i_1} x .. x
 * dX^{i_d} on the nested CGL (Clenshaw-Curtis) sets of eq. CGL,
 * X^1 = {1/2}, X^i = {(1 - cos((k-1) pi / 2^{i-1})) / 2 : k = 1..2^{i-1}+1},
 * with q = level + d, mapped affinely from [0,1]^d to the box [lo, hi].
 *
 * Canonical node order (used by every array indexed by node): every 1-D
 * point has an integer id, numbered by the level at which it first appears
 * and, within a level, by increasing coordinate (level 1: id 0 = 1/2;
 * level 2: id 1 = 0, id 2 = 1; level i >= 3: ids 2^{i-2}+1 .. 2^{i-1}).  A
 * node's key is its tuple of d ids; nodes are sorted lexicographically by key. */
typedef struct sgcm_grid sgcm_grid;

/* Create the grid (host-side tables only: no device is needed).
 * 1 <= d <= 8, 0 <= level <= 5, lo[j] < hi[j]. */
int sgcm_grid_create(int32_t d, int32_t level, const double* lo, const double* hi,
                     sgcm_grid** out);

/* Make the grid's device tables on the current device: node coordinates,
 * level lists, 1-D point and scale tables, child offsets, the node maps of
 * the lower-level grids and a build staging buffer of M x 3 doubles (about
 * 30 M + 4 d M bytes in all).  This call allocates (hipMalloc) and copies the
 * tables on `stream` (stream-ordered; the host tables belong to the grid and
 * stay valid); it does nothing if the tables are already on this device.  It
 * must precede sgcm_build_interpolant and the sgcm_eval_feedback calls on a
 * device, which then allocate nothing and never synchronise.  Not to be
 * called concurrently with a build or an evaluation of the same grid.
 * Returns SGCM_EINVAL for a NULL grid, SGCM_ENOMEM, SGCM_EDEVICE. */
int sgcm_grid_upload(sgcm_grid* g, void* stream);

/* Number of nodes M, or -1 for a NULL grid. */
int64_t sgcm_grid_size(const sgcm_grid* g);

/* Host copies of the node coordinates (M x d, box coordinates) and keys
 * (M x d point ids), canonical order. */
int sgcm_grid_nodes(const sgcm_grid* g, double* nodes_host);
int sgcm_grid_keys(const sgcm_grid* g, int32_t* keys_host);

/* Free the grid and its device tables (device tables are freed on the
 * device they were made on, after the work queued on it).  NULL is a no-op. */
void sgcm_grid_destroy(sgcm_grid* g);

/* ---- interpolant (Sec. 3.3, eq. interpo) ----------------------------------- */

/* The grid's tables must be on the current device (sgcm_grid_upload), else
 * the calls below return SGCM_EINVAL; they allocate nothing.
 *
 * Hierarchical surpluses of eq. interpo: for levels |i| = d..q in order,
 * w = f(node) - I^{|i|-1}(f)(node), with the tensor-product Lagrange basis on
 * X^{i_1} x .. x X^{i_d}.
 *   values   device, M x m node values f (canonical order), read only
 *   surplus  device, M x m (canonical order); may not alias values
 * 1 <= m <= 64.  Every value must be finite: the node values of BVP
 * solutions whose status is not SGCM_BVP_CONVERGED are the last Newton
 * iterate and are not to be interpolated (the Python binding refuses them
 * with SGCM_ENOTCONVERGED).  For d = 6 and m <= 3 the lower levels'
 * surpluses are staged in the grid's device buffer, so builds with the same
 * grid on one device must not overlap (use one stream, or order them). */
int sgcm_build_interpolant(const sgcm_grid* g, int32_t m, const double* values,
                           double* surplus, void* stream);

/* The on-line step: evaluate the interpolant I^q(f)(x) = sum over nodes of
 * w * prod_j a^{i_j}(xi_j) at n_q query states (Sec. 3.3, Step III and the
 * text after it), xi = (x - lo) / (hi - lo).  Queries outside the box are
 * evaluated by the same polynomial (no clamping).
 *   surplus  device, M x m from sgcm_build_interpolant
 *   xq       device, n_q x d query states
 *   uq       device, n_q x m results
 *   precision  SGCM_FP64 (FP32 evaluation is sgcm_eval_feedback_f32, with
 *            FP32 arrays; SGCM_FP32 here returns SGCM_EUNSUPPORTED)
 * n_q == 0 is a valid no-op. */
int sgcm_eval_feedback(const sgcm_grid* g, int32_t m, const double* surplus, int64_t n_q,
                       const double* xq, double* uq, int32_t precision, void* stream);

/* The same evaluation in FP32 (the reduced-precision variant of the on-line
 * step): surplus (M x m), xq (n_q x d) and uq (n_q x m) are FP32 device
 * arrays; the 1-D Lagrange basis values, their products and the sum over the
 * nodes are computed in FP32 (the map to the unit cube in FP64, then rounded).
 * Supported for d = 6, levels 1..5 and m <= 3, else SGCM_EUNSUPPORTED.  The
 * error against the FP64 evaluation is that of FP32 rounding in a sum of M
 * terms (about 1e-6 of max|u| on the rigid-body feedback). */
int sgcm_eval_feedback_f32(const sgcm_grid* g, int32_t m, const float* surplus, int64_t n_q,
                           const float* xq, float* uq, void* stream);

/* ---- total-error estimate (Sec. 4.3) ---------------------------------------- */

/* The error of the interpolant at n sample states against BVP solutions more
 * accurate than those at the grid nodes (the Monte Carlo estimate of
 * e_interp + e_bvp of Sec. 4.3).  The reference at a sample is the Richardson
 * extrapolation of two solutions of a formula of order p (order), on N and
 * 2N intervals of the same horizon: ref = (2^p fine - coarse) / (2^p - 1),
 * which removes the h^p term of the error (p = 2 for the trapezoid, whose
 * error expands in even powers of h; p = 6 for the four-point Lobatto IIIA
 * formula at the mesh points).
 *   order    p, 1..16
 *   interp   device, n x m: the interpolant at the samples (sgcm_eval_feedback)
 *   coarse   device, n x m: the same quantity solved on N intervals
 *   fine     device, n x m: solved on 2N intervals
 *   ref      device, n x m out: the extrapolated reference
 *   err      device, n out: max over the m components of |interp - ref|
 *   stats    device, 5 out: [0] max of err, [1] RMS of err, [2] max over
 *           samples and components of |fine - ref| (the extrapolation's
 *           correction to the fine solution, an estimate of its error),
 *           [3] the mean absolute error (mean of err), [4] the mean relative
 *           error, mean of err / max(max_c |ref|, 1e-8) (Sec. 5.1, Table 1)
 * Row-major arrays; no output may overlap an input.  A NaN in any input
 * propagates to its err entry and to stats.  n == 0 writes zeros to stats.
 * 1 <= m <= 64.  One workgroup does the whole call, in stream order. */
int sgcm_total_error(int64_t n, int32_t m, int32_t order, const double* interp, const double* coarse,
                     const double* fine, double* ref, double* err, double* stats, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SGCM_H */

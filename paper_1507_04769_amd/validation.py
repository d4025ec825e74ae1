"""Monte Carlo estimate of the total error of the feedback interpolant on the
device (Sec. 4.3).

The interpolant is built from solutions at the grid nodes, so at a state x its
error against the true solution is e_interp + e_bvp.  It is measured at sample
states against a reference that is much more accurate than the node
solutions.  As in the paper, the reference comes from the four-point Lobatto
IIIA formula with error control (Sec. 4.3, Sec. 5.1): the sample states are
solved on N_r and 2 N_r intervals, the two solutions are extrapolated at the
formula's order (6), and N_r doubles until the extrapolation's correction to
the finer solution, the estimate of its error, is within the reference
tolerance (the paper sets 1e-7 or 1e-9).  The trapezoid with an order-2
extrapolation remains available.  The paper samples 1280 random states and
reports the mean absolute error and its relative form (Table 1).

Every step runs in libsgcm: the reference solves (sgcm_solve_bvps), the
evaluation of the interpolant (sgcm_eval_feedback) and the comparison
(sgcm_total_error); this module orders the calls and reads the correction on
the host to decide the doubling.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass

import paper_1507_04769_amd as S

N_SAMPLES = 1280  # random states of the paper's estimate (Sec. 4.3)
SAMPLE_SEED = 43  # seed of the uniform sample in the state box
REF_TOL = 1e-7    # the reference's error tolerance (the paper's 1e-7 of Sec. 5.1)
MAX_REF = 2048    # largest mesh of the reference solves


@dataclass
class TotalError:
    """Per-sample results (device tensors) and the solves behind them."""
    ref_u: "object"     # n x m extrapolated reference feedback u(0, x)
    err_u: "object"     # n: max over components of |I(u)(x) - ref_u|
    stats_u: "object"   # 5: max err, RMS err, max |u_fine - ref_u|, MAE, relative MAE
    ref_V: "object"     # n x 1 extrapolated reference value V(0, x), or None
    err_V: "object"     # n, or None
    stats_V: "object"   # 5, or None
    status: "object"    # 2 x n: status of the solves on N_r and 2 N_r intervals (all
                        # CONVERGED: the estimator raises SGCM_ENOTCONVERGED otherwise)
    iters: "object"     # 2 x n
    n_ref: int = 0      # the accepted N_r
    correction: float = 0.0  # the accepted reference's estimated error (max over u and V)


class Estimator:
    """The reference solves for one problem: the four-point Lobatto IIIA
    formula (scheme S.LOBATTO4, extrapolated at order 6) from n_ref intervals
    with error control, or the trapezoid (S.TRAPEZOID, order 2, solve plans
    made once) on n_ref and 2 n_ref intervals."""

    def __init__(self, problem: S.Problem, n_ref: int, scheme: int = S.LOBATTO4, ref_tol: float = REF_TOL,
                 max_ref: int = MAX_REF, stream=None):
        if n_ref < 1:
            raise ValueError("n_ref must be positive")
        if scheme not in (S.TRAPEZOID, S.LOBATTO4):
            raise ValueError("unknown scheme")
        self.problem = dataclasses.replace(problem, scheme=scheme, precision=S.FP64)
        self.n_ref = int(n_ref)
        self.scheme = scheme
        self.order = 6 if scheme == S.LOBATTO4 else 2
        self.ref_tol = float(ref_tol)
        self.max_ref = int(max_ref)
        self.plans = {}
        if scheme == S.TRAPEZOID:  # fixed meshes, first steps from plans
            for n in (self.n_ref, 2 * self.n_ref):
                self.plans[n] = S.Plan(dataclasses.replace(self.problem, N=n), stream)

    def _solve(self, n: int, xs, want_V: bool, stream):
        p = dataclasses.replace(self.problem, N=n)
        return S.solve_bvps(p, xs, want_V=want_V, stream=stream, plan=self.plans.get(n))

    def __call__(self, grid: S.Grid, surplus_u, xs, surplus_V=None, stream=None) -> TotalError:
        """Estimate at the states xs (n x 6, device) the error of the
        interpolant with surplus surplus_u (M x m: the feedback u(0, x)) and,
        if given, of the one with surplus_V (M x 1: the value V(0, x))."""
        import torch
        want_V = surplus_V is not None
        u_int = S.eval_feedback(grid, surplus_u, xs, stream=stream)
        V_int = S.eval_feedback(grid, surplus_V, xs, stream=stream) if want_V else None
        n_r = self.n_ref
        c = self._solve(n_r, xs, want_V, stream)
        while True:
            f = self._solve(2 * n_r, xs, want_V, stream)
            ref_u, err_u, st_u = S.total_error(u_int, c.u0, f.u0, stream, self.order)
            ref_V = err_V = st_V = None
            if want_V:
                ref_V, err_V, st_V = S.total_error(V_int, c.V.view(-1, 1), f.V.view(-1, 1), stream, self.order)
            corr = float(st_u[2].item()) if not want_V else max(float(st_u[2].item()), float(st_V[2].item()))
            if self.scheme == S.TRAPEZOID or corr <= self.ref_tol or 4 * n_r > self.max_ref:
                break
            n_r *= 2
            c = f
        status = torch.stack([c.status, f.status])
        bad = int((status != S.CONVERGED).sum().item())
        if bad:  # a reference that did not converge is no reference
            raise S.SgcmError(S.SGCM_ENOTCONVERGED, "total-error reference (%d of %d solves)" % (bad, status.numel()))
        return TotalError(ref_u, err_u, st_u, ref_V, err_V, st_V, status, torch.stack([c.iters, f.iters]), n_r, corr)

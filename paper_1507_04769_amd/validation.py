"""Monte Carlo estimate of the total error of the feedback interpolant on the
device (Sec. 4.3).

The interpolant is built from trapezoidal solutions on N intervals at the grid
nodes, so at a state x its error against the true solution is
e_interp + e_bvp.  It is measured at sample states against a reference that is
much more accurate than the node solutions: the Richardson extrapolation of
trapezoidal solutions on N_r and 2 N_r intervals of the same horizon
((4 f_2N - f_N) / 3, accurate to O(h^4); the paper uses an error-controlled
collocation solver instead).  The paper samples 1280 random states.

Every step runs in libsgcm: the reference solves (sgcm_solve_bvps_plan, one
plan per mesh), the evaluation of the interpolant (sgcm_eval_feedback) and the
comparison (sgcm_total_error); this module orders the calls.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass

import paper_1507_04769_amd as S

N_SAMPLES = 1280  # random states of the paper's estimate (Sec. 4.3)
SAMPLE_SEED = 43  # seed of the uniform sample in the state box


@dataclass
class TotalError:
    """Per-sample results (device tensors) and the solves behind them."""
    ref_u: "object"     # n x m extrapolated reference feedback u(0, x)
    err_u: "object"     # n: max over components of |I(u)(x) - ref_u|
    stats_u: "object"   # 3: max err, RMS err, max |u_fine - ref_u|
    ref_V: "object"     # n x 1 extrapolated reference value V(0, x), or None
    err_V: "object"     # n, or None
    stats_V: "object"   # 3, or None
    status: "object"    # 2 x n: status of the solves on N_r and 2 N_r intervals
    iters: "object"     # 2 x n


class Estimator:
    """The reference solves for one problem: plans for N_r and 2 N_r
    intervals, made once (each solves the six unit-state first steps)."""

    def __init__(self, problem: S.Problem, n_ref: int, stream=None):
        if n_ref < 1:
            raise ValueError("n_ref must be positive")
        self.problem = problem
        self.n_ref = int(n_ref)
        self.coarse = S.Plan(dataclasses.replace(problem, N=self.n_ref), stream)
        self.fine = S.Plan(dataclasses.replace(problem, N=2 * self.n_ref), stream)

    def __call__(self, grid: S.Grid, surplus_u, xs, surplus_V=None, stream=None) -> TotalError:
        """Estimate at the states xs (n x 6, device) the error of the
        interpolant with surplus surplus_u (M x m: the feedback u(0, x)) and,
        if given, of the one with surplus_V (M x 1: the value V(0, x))."""
        import torch
        c = S.solve_bvps(self.coarse.problem, xs, want_V=surplus_V is not None, stream=stream, plan=self.coarse)
        f = S.solve_bvps(self.fine.problem, xs, want_V=surplus_V is not None, stream=stream, plan=self.fine)
        u_int = S.eval_feedback(grid, surplus_u, xs, stream=stream)
        ref_u, err_u, st_u = S.total_error(u_int, c.u0, f.u0, stream)
        ref_V = err_V = st_V = None
        if surplus_V is not None:
            V_int = S.eval_feedback(grid, surplus_V, xs, stream=stream)
            ref_V, err_V, st_V = S.total_error(V_int, c.V.view(-1, 1), f.V.view(-1, 1), stream)
        return TotalError(ref_u, err_u, st_u, ref_V, err_V, st_V, torch.stack([c.status, f.status]),
                          torch.stack([c.iters, f.iters]))

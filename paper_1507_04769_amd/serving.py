"""Continuous-batching request loop for the hot path (the serving direction).

Requests arrive over time (a seeded Poisson stream): BVP-solve requests (a
few initial states of the three- or two-wheel model on a mesh of N intervals)
and feedback-query requests (states to evaluate against an interpolant kept
resident on the device, in FP64 or FP32).  The loop

  * admits arrived requests into a pending list;
  * merges pending requests with the same key (model and N for solves;
    interpolant and precision for queries) into one launch: a solve launch
    concatenates the initial states of several requests into one
    sgcm_solve_bvps call, a query launch the states of several requests into
    one evaluation call;
  * starts a launch whenever one of its streams is free and the device
    memory of the launches in flight stays within an HBM budget (admission by
    footprint: states, outputs and workspace of the launch), so that requests
    arriving while others run are admitted as slots and memory free up and
    their work overlaps on the device;
  * caps the streams one class of work may hold at once (two-wheel solves,
    whose continuation can run for hundreds of Newton iterations, take all
    but one), so that short work (queries, three-wheel solves) always finds
    a stream instead of queueing behind long launches;
  * retires launches as their completion events fire and hands every request
    its slice of the outputs.

Completions are event driven: one waiter thread per stream watches the
completion event of each launch of its stream in launch order (launches on
one stream complete in order; the event is queried every 50 us, since a
blocking wait in the runtime delayed the launches issued meanwhile on other
streams), then copies the launch's outputs to the host and hands the launch
to the loop, which sleeps until a completion or the next arrival.  The output
copies are issued only once the launch's kernels have completed: the runtime
carries out the copies of all streams in the order they were issued, so an
output copy queued behind a two-wheel solve (tens of ms) held up the input
copy, and so the kernels, of every launch issued after it on any stream
(queries waited up to 90 ms for a kernel of 0.1 ms).  Every output of
a request depends only on that request's inputs (BVPs and query points are
independent), so a request's results are the same alone and in any mix; the
tests check this bitwise.  Latency = completion - arrival on the host clock.
"""
from __future__ import annotations

import dataclasses
import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np

import paper_1507_04769_amd as S
from paper_1507_04769_amd import workloads as W


@dataclass
class SolveRequest:
    rid: int
    arrival: float      # seconds after the stream starts
    x0: np.ndarray      # n x 6 initial states
    N: int              # mesh intervals
    m: int = 3          # wheels: 3 or 2
    T: float = 20.0     # horizon
    out: dict = field(default=None, repr=False)
    done: float = None

    def key(self):
        return ("solve", self.m, self.N, self.T)


@dataclass
class QueryRequest:
    rid: int
    arrival: float
    xq: np.ndarray      # n x 6 states
    level: int          # resident interpolant (grid level)
    fp32: bool = False
    out: np.ndarray = field(default=None, repr=False)
    done: float = None

    def key(self):
        return ("query", self.level, self.fp32)


def problem(m: int, N: int, T: float = 20.0) -> S.Problem:
    """The served problem: three wheels, or two wheels reached by the
    virtual-torque continuation (four stages, at most 100 iterations each)."""
    if m == 2:
        return S.Problem(m=2, J=W.J_DIAG, B=W.input_matrix(2), q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, T=T, N=N,
                         tol=W.TOL, max_iter=W.UNDERACTUATED_MAX_ITER, max_halvings=W.MAX_HALVINGS,
                         continuation=W.UNDERACTUATED_CONTINUATION)
    return S.Problem(m=m, J=W.J_DIAG, B=W.input_matrix(m), q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, T=T, N=N,
                     tol=W.TOL, max_iter=W.MAX_ITER, max_halvings=W.MAX_HALVINGS)


class Interpolant:
    """A feedback interpolant resident on the device (FP64 and FP32 surplus)."""

    def __init__(self, level: int, surplus64):
        self.level = level
        self.grid = S.Grid(6, level, W.BOX_LO, W.BOX_HI)
        self.grid.upload()  # the grid's device tables, made before any request is served
        self.w64 = surplus64
        self.w32 = surplus64.float().contiguous()


def build_interpolant(level: int, N: int = 64):
    """Interpolant of u(0) of the three-wheel problem on the level-`level` grid
    (solved on the device)."""
    import torch
    g = S.Grid(6, level, W.BOX_LO, W.BOX_HI)
    sol = S.solve_bvps(problem(3, N), torch.tensor(g.nodes(), device="cuda"))
    return Interpolant(level, S.build_feedback_interpolant(g, sol))


@dataclass
class _Launch:
    reqs: list
    stream: object
    event: object       # the launch's kernels have completed
    nbytes: int
    dev_outs: tuple     # device outputs, copied to the host once `event` fires
    cls: str = ""
    outs: tuple = ()    # host outputs


def work_class(key) -> str:
    """Class of a launch key for the stream caps: "query", "solve" (three
    wheels) or "solve-2wheel"."""
    if key[0] == "query":
        return "query"
    return "solve-2wheel" if key[1] == 2 else "solve"


def request_size(r) -> int:
    return len(r.x0) if isinstance(r, SolveRequest) else len(r.xq)


def footprint(key, n: int) -> int:
    """Device bytes a launch of n states (solve) or points (query) holds:
    inputs, outputs and, for a solve, the solver workspace."""
    if key[0] == "solve":
        m, N, T = key[1], key[2], key[3]
        return S.sgcm_solve_bvps_workspace(problem(m, N, T), n) + n * 8 * (6 + 6 + m + 1) + n * 4 * 2
    return n * (4 if key[2] else 8) * (6 + 3)


class Admission:
    """Which pending requests start next (host-side policy).

    The oldest pending request whose class holds fewer streams than its cap
    leads (first come, first served within a class, so nothing starves);
    later pending requests with the same key join it while the merged launch
    stays within its size cap and the device memory of all launches in
    flight within the budget.  If the leading request does not fit next to
    the launches in flight, nothing starts until memory frees up; a request
    larger than the whole budget starts alone on an idle device.
    stream_caps: class (`work_class`) -> most streams it may hold at once;
    size_caps: class -> most states of one merged launch (below max_bvps or
    max_points); classes not named are not capped."""

    def __init__(self, hbm_budget: int, max_bvps: int = 2048, max_points: int = 1 << 20,
                 merge: bool = True, footprint=footprint, stream_caps: dict | None = None,
                 size_caps: dict | None = None):
        self.budget = int(hbm_budget)
        self.max_bvps = max_bvps
        self.max_points = max_points
        self.merge = merge
        self.footprint = footprint
        self.caps = dict(stream_caps or {})
        self.size_caps = dict(size_caps or {})

    def select(self, pending: list, used: int, busy: dict | None = None, avail=None):
        """(key, chosen requests, merged size, bytes) or None.  busy: class ->
        streams it holds now; avail: the classes that have a free stream now
        (None: all)."""
        busy = busy or {}
        lead = None
        for j, r in enumerate(pending):
            c = work_class(r.key())
            if avail is not None and c not in avail:
                continue
            if c not in self.caps or busy.get(c, 0) < self.caps[c]:
                lead = j
                break
        if lead is None:
            return None
        key = pending[lead].key()
        cap = self.max_bvps if key[0] == "solve" else self.max_points
        cap = min(cap, self.size_caps.get(work_class(key), cap))
        chosen, n = [pending[lead]], request_size(pending[lead])
        if used > 0 and used + self.footprint(key, n) > self.budget:
            return None
        if self.merge:
            for r in pending[lead + 1:]:
                if r.key() != key:
                    continue
                k = request_size(r)
                if n + k > cap or used + self.footprint(key, n + k) > self.budget:
                    break
                chosen.append(r)
                n += k
        return key, chosen, n, self.footprint(key, n)


def solve_plan(key) -> S.Plan:
    """The solve plan of a solve key ("solve", m, N, T) (made on the default
    stream, which it synchronizes)."""
    return S.Plan(problem(key[1], key[2], key[3]))


class Server:
    def __init__(self, interpolants: dict, n_streams: int = 4, hbm_budget: int = 1 << 30,
                 max_bvps: int = 2048, max_points: int = 1 << 20, merge: bool = True, plans: dict | None = None,
                 stream_caps: dict | None = None, size_caps: dict | None = None):
        """interpolants: level -> resident Interpolant; n_streams: launches in
        flight at once; hbm_budget: device bytes the launches in flight may
        hold; max_bvps / max_points: size cap of one merged launch;
        merge=False serves one request per launch; plans: solve key -> solve
        plan (each solve launch forms its first Newton steps from its key's
        plan; a missing plan is made at the key's first launch);
        stream_caps: class -> most streams it may hold (default: two-wheel
        solves all streams but one, at least one); size_caps: class
        -> most states of one launch (default: none)."""
        import torch
        self.plans = {} if plans is None else dict(plans)
        self.interp = interpolants
        if stream_caps is None:
            stream_caps = {"solve-2wheel": max(1, n_streams - 1)}
        self.admit = Admission(hbm_budget, max_bvps, max_points, merge, stream_caps=stream_caps,
                               size_caps=size_caps)
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.dev = torch.device("cuda")

    def _launch(self, key, reqs, n, stream) -> _Launch:
        import torch
        if key[0] == "solve" and key not in self.plans:
            self.plans[key] = solve_plan(key)  # before the launch stream is entered
        with torch.cuda.stream(stream):
            if key[0] == "solve":
                m, N, T = key[1], key[2], key[3]
                p = problem(m, N, T)
                xh = torch.from_numpy(np.concatenate([r.x0 for r in reqs])).pin_memory()
                x = xh.to(self.dev, non_blocking=True)
                ws = torch.empty((max(S.sgcm_solve_bvps_workspace(p, n), 256) + 255) // 256 * 32,
                                 dtype=torch.float64, device=self.dev)
                lam = torch.empty((n, 6), dtype=torch.float64, device=self.dev)
                u0 = torch.empty((n, m), dtype=torch.float64, device=self.dev)
                V = torch.empty((n,), dtype=torch.float64, device=self.dev)
                st = torch.empty((n,), dtype=torch.int32, device=self.dev)
                it = torch.empty((n,), dtype=torch.int32, device=self.dev)
                S.sgcm_solve_bvps_plan(self.plans[key], x, lam, u0, V, None, st, it, ws, stream)
                outs = (lam, u0, V, st, it)
                keep = (xh, x, ws)
            else:
                itp = self.interp[key[1]]
                fp32 = key[2]
                xq = np.concatenate([r.xq for r in reqs])
                xh = torch.from_numpy(xq.astype(np.float32) if fp32 else xq).pin_memory()
                x = xh.to(self.dev, non_blocking=True)
                if fp32:
                    uq = torch.empty((n, itp.w32.shape[1]), dtype=torch.float32, device=self.dev)
                    S.sgcm_eval_feedback_f32(itp.grid, itp.w32, x, uq, stream)
                else:
                    uq = torch.empty((n, itp.w64.shape[1]), dtype=torch.float64, device=self.dev)
                    S.sgcm_eval_feedback(itp.grid, itp.w64, x, uq, S.FP64, stream)
                outs = (uq,)
                keep = (xh, x)
            ev = torch.cuda.Event(blocking=True)  # a host wait on it sleeps instead of spinning
            ev.record(stream)
        L = _Launch(reqs, stream, ev, footprint(key, n), outs, work_class(key))
        L.keep = keep  # device buffers stay referenced until the launch retires
        return L

    def _retire(self, L: _Launch, now: float):
        if L.reqs[0].key()[0] == "solve":
            lam, u0, V, st, it = (t.numpy() for t in L.outs)
            i = 0
            for r in L.reqs:
                k = len(r.x0)
                r.out = {"lambda0": lam[i:i + k].copy(), "u0": u0[i:i + k].copy(), "V": V[i:i + k].copy(),
                         "status": st[i:i + k].copy(), "iters": it[i:i + k].copy()}
                r.done = now
                i += k
        else:
            uq = L.outs[0].numpy()
            i = 0
            for r in L.reqs:
                k = len(r.xq)
                r.out = uq[i:i + k].copy()
                r.done = now
                i += k

    @staticmethod
    def _wait(event):
        """Return in the calling (waiter) thread once the event has fired.
        It is queried every 50 us: a blocking hipEventSynchronize in the
        waiter threads delayed the launches the loop issued meanwhile on
        other streams."""
        while not event.query():
            time.sleep(50e-6)

    def _complete(self, L: _Launch):
        """In the launch's waiter thread: wait for its kernels, then copy its
        outputs to the host on its own stream (idle by then) and wait for the
        copies."""
        import torch
        self._wait(L.event)
        with torch.cuda.stream(L.stream):
            L.outs = tuple(t.to("cpu", non_blocking=True) for t in L.dev_outs)
            copied = torch.cuda.Event()
            copied.record(L.stream)
        self._wait(copied)

    def run(self, requests: list, realtime: bool = True) -> dict:
        """Serve the requests (sorted by arrival).  realtime: inject each
        request at its arrival time on the host clock; else all at once."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending, inflight = [], []
        free = list(self.streams)
        used = peak_used = peak_shared = peak_inflight = 0
        busy = {}
        i = 0
        launches = 0
        done = queue.Queue()  # launches whose completion event has fired
        todo = {id(st): queue.Queue() for st in self.streams}

        def wait_stream(q):
            while True:
                L = q.get()
                if L is None:
                    return
                try:
                    self._complete(L)
                except BaseException as e:  # handed to the loop, which raises it
                    done.put((L, e))
                    return
                done.put((L, time.perf_counter()))

        waiters = [threading.Thread(target=wait_stream, args=(todo[id(st)],), daemon=True) for st in self.streams]
        for th in waiters:
            th.start()
        t0 = time.perf_counter()
        try:
            while i < len(reqs) or pending or inflight:
                now = time.perf_counter() - t0
                while i < len(reqs) and (not realtime or reqs[i].arrival <= now):
                    pending.append(reqs[i])
                    i += 1
                while free and pending:
                    g = self.admit.select(pending, used, busy)
                    if g is None:
                        break
                    key, chosen, n, _ = g
                    L = self._launch(key, chosen, n, free.pop(0))
                    for r in chosen:
                        pending.remove(r)
                    inflight.append(L)
                    todo[id(L.stream)].put(L)
                    busy[L.cls] = busy.get(L.cls, 0) + 1
                    used += L.nbytes
                    launches += 1
                    peak_used = max(peak_used, used)
                    peak_inflight = max(peak_inflight, len(inflight))
                    if len(inflight) > 1:
                        peak_shared = max(peak_shared, used)
                # sleep until a launch completes or the next request arrives
                timeout = None
                if realtime and i < len(reqs):
                    timeout = max(0.0, reqs[i].arrival - (time.perf_counter() - t0))
                if not inflight:
                    if timeout:
                        time.sleep(timeout)
                    continue
                try:
                    item = done.get(timeout=timeout)
                except queue.Empty:
                    continue
                while item is not None:
                    L, t_done = item
                    if isinstance(t_done, BaseException):
                        raise t_done
                    self._retire(L, t_done - t0)
                    inflight.remove(L)
                    free.append(L.stream)
                    busy[L.cls] -= 1
                    used -= L.nbytes
                    try:
                        item = done.get_nowait()
                    except queue.Empty:
                        item = None
        finally:
            for st in self.streams:
                todo[id(st)].put(None)
            for th in waiters:
                th.join()
        wall = time.perf_counter() - t0
        lat = np.array([r.done - (r.arrival if realtime else 0.0) for r in reqs]) * 1e3
        cls = np.array([work_class(r.key()) for r in reqs])
        by_class = {c: {"requests": int(np.sum(cls == c)),
                        "p50": float(np.percentile(lat[cls == c], 50)),
                        "p99": float(np.percentile(lat[cls == c], 99))}
                    for c in ("query", "solve", "solve-2wheel") if np.any(cls == c)}
        n_bvps = sum(len(r.x0) for r in reqs if isinstance(r, SolveRequest))
        n_pts = sum(len(r.xq) for r in reqs if isinstance(r, QueryRequest))
        return {"requests": len(reqs), "launches": launches, "wall_s": wall,
                "peak_inflight": peak_inflight, "peak_inflight_bytes": peak_used,
                "peak_shared_bytes": peak_shared,
                "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                               "max": float(lat.max()), "by_class": by_class},
                "throughput": {"requests_per_s": len(reqs) / wall, "bvps_per_s": n_bvps / wall,
                               "evals_per_s": n_pts / wall}}


def request_stream(n: int, rate: float, seed: int, levels=(3, 4), max_states: int = 512,
                   max_points: int = 100_000, meshes=(64, 128, 256, 512)) -> list:
    """A seeded Poisson stream of n requests at `rate` per second: half solve
    requests (1..max_states states uniform in the box, N from `meshes`, T = 20;
    one in four on the two-wheel model), half query requests (1..max_points
    states uniform in the box against one of `levels`, one in two in FP32)."""
    g = np.random.default_rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate, size=n))
    out = []
    for k in range(n):
        if g.random() < 0.5:
            m = 2 if g.random() < 0.25 else 3
            ns = int(g.integers(1, max_states + 1))
            x0 = W.uniform_in_box(ns, seed=int(g.integers(1 << 30)))
            out.append(SolveRequest(k, float(t[k]), x0, int(g.choice(meshes)), m, 20.0))
        else:
            npts = int(np.exp(g.uniform(0.0, np.log(max_points))))
            xq = W.uniform_in_box(max(npts, 1), seed=int(g.integers(1 << 30)))
            out.append(QueryRequest(k, float(t[k]), xq, int(g.choice(levels)), bool(g.random() < 0.5)))
    return out


def solve_alone(r: SolveRequest) -> dict:
    """The request solved on its own: one call with its key's solve plan, as
    the server solves it."""
    import torch
    sol = S.solve_bvps(problem(r.m, r.N, r.T), torch.tensor(r.x0, device="cuda"), plan=solve_plan(r.key()))
    torch.cuda.synchronize()
    return {k: getattr(sol, k).cpu().numpy() for k in ("lambda0", "u0", "V", "status", "iters")}


def query_alone(r: QueryRequest, itp: Interpolant) -> np.ndarray:
    import torch
    if r.fp32:
        out = S.eval_feedback_f32(itp.grid, itp.w32, torch.tensor(r.xq, device="cuda"))
    else:
        out = S.eval_feedback(itp.grid, itp.w64, torch.tensor(r.xq, device="cuda"))
    torch.cuda.synchronize()
    return out.cpu().numpy()

"""Continuous-batching solve server on one GPU.

Requests (a grid, a geometry, a source) arrive over time.  The server keeps
the set of problems being solved on the device and advances all of them
together, one V-cycle (or refinement step) per ``tomg_batch_step``; between
two steps it retires problems that reached the tolerance and admits queued
requests, so a request that arrives while others are being solved joins the
next step instead of waiting for the batch to drain.  One batched launch
serves one level-0 operator form and one set of level transfers, so a step
advances the problems in groups: the on-the-fly eq. 18 operator or a stored
stencil (Neumann edges, flux form), and the semi-coarsened levels.

Memory.  Every geometry the server holds (being solved, or idle and kept for
a later warm re-solve) costs its library workspace plus its solution array;
a request is admitted only if that footprint, plus the transient input
arrays of its setup, fits in the budget after idle geometries have been
evicted, least recently used first.  Admission is first-come first-served:
a request that does not fit stops admission (later requests do not overtake
it), except that a request whose geometry is still being solved is passed
over until that solve ends.

Cold setups are queued without waiting for the device: the geometry checks
of a setup (folded map, non-finite input, singular coarsest matrix) come
back with the request's first step, whose residual is then non-finite; the
server asks the backend for the reason, reports it in the completion and
drops the geometry.

Pipelining.  With a backend that can queue a step without waiting for it
(``launch``/``collect``; ``TomgBackend`` uses ``tomg_batch_launch``), a
server step queues the batched step, then admits the requests that arrived
meanwhile (problem creation, input evaluation and setups, all queued on the
same stream behind the step), then waits for the step's residuals.  The
newly admitted requests join the next step.  Only idle geometries are
evicted or re-used during admission, so nothing the running step reads is
touched.  ``pipeline=False`` gives the serial order (admit, step, wait).

Warm re-solves.  A request marked warm whose geometry is resident and idle
skips the coefficient setup and the hierarchy build: only the right-hand
side is recomputed (``tomg_update_rhs``), and the iteration starts from the
geometry's last solution.  If the geometry has been evicted the request is
served cold.

Inputs.  A request that carries map and source descriptors is set up by
``tomg_setup_coeffs_desc`` (and re-sourced by ``tomg_update_rhs_desc``): the
setup kernel evaluates the map, its Jacobian and the charge density at each
node, so admission launches a handful of library kernels and moves no input
arrays.  Other requests hand the library device arrays from ``geometry()``
and ``source()``.

The arithmetic of each problem does not depend on the others in the batch or
on when it joined: a request's result is bitwise the result of solving it
alone from the same initial guess.

The server is host logic only; every solver step runs in the library's
kernels through the backend (``TomgBackend``).
"""

from __future__ import annotations

import math
import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field
from typing import Callable, Hashable, List, Optional

TOMG_OK, TOMG_ENOCONV, TOMG_ENONFINITE = 0, -4, -5


@dataclass
class Request:
    """One solve request.

    ``geometry()`` returns the device arrays of the map (dict with xp, yp,
    jac, mask, phi0; None where absent) and ``source()`` the charge density
    rho' at the nodes; both are called only when needed (cold start, or a new
    right-hand side).  ``geom`` identifies the geometry: a warm request with
    the key of a resident geometry re-uses its hierarchy and last solution."""
    rid: int
    geom: Hashable
    nx: int
    ny: int
    dx: float
    dy: float
    geometry: Callable[[], dict]
    source: Callable[[], object]
    warm: bool = False
    arrival: float = 0.0
    xi0: float = 0.0
    eta0: float = 0.0
    neumann: int = 0      # edges with a zero normal derivative (TOMG_NEU_* bits)
    flux: bool = False    # the symmetric flux form of the operator
    semi_levels: int = 0  # leading coarsenings that halve one axis only
    semi_axis: str = "x"  # the axis they halve
    # the same request as descriptors (keyword arguments of the library's
    # map_desc and source_desc): a backend that takes them evaluates the map
    # and the source in its setup kernel, with no input arrays
    map_desc: Optional[dict] = None
    source_desc: Optional[dict] = None

    @property
    def stored_form(self) -> bool:
        """True when the problem's level-0 operator is a stored stencil."""
        return bool(self.neumann) or bool(self.flux)

    @property
    def shape(self):
        """What a problem's workspace depends on: a problem created for one
        request can be set up again for another of the same shape."""
        return (self.nx, self.ny, self.dx, self.dy, self.xi0, self.eta0, self.neumann,
                bool(self.flux), self.semi_levels, self.semi_axis)

    @property
    def step_kind(self):
        """Requests of one kind share a batched step: the same level-0
        operator form and the same semi-coarsened levels."""
        return (self.stored_form, self.semi_levels, self.semi_axis if self.semi_levels else "")


@dataclass
class Completion:
    rid: int
    status: int
    cycles: int
    rel: float
    arrival: float
    admitted: float
    done: float
    warm_start: bool          # started from a resident geometry's last solution
    queue_depth: int = 0      # requests still queued when this one was admitted
    hbm_used: int = 0         # bytes the server held once this request was admitted
    #                           (its geometries, this request's included)
    phi: object = None        # copy of the solution (keep_results=True)
    phi_start: object = None  # copy of the initial guess (keep_results=True)
    error: str = ""           # why a request failed before its first step

    @property
    def latency(self):
        return self.done - self.arrival

    @property
    def ok(self):
        return self.status == TOMG_OK


@dataclass
class _Resident:
    key: Hashable
    problem: object
    phi: object
    nbytes: int
    busy: bool = False
    shape: object = None  # Request.shape of the geometry it was set up for


@dataclass
class _Active:
    req: Request
    res: _Resident
    admitted: float
    warm_start: bool
    fresh: bool = True
    cycles: int = 0
    rel: float = math.inf
    phi_start: object = None
    queue_depth: int = 0
    hbm_used: int = 0


class TomgBackend:
    """The library as seen by the server: problem creation and setup, warm
    right-hand-side updates and the batched step."""

    reuses = True  # create() can set up an evicted problem of the same shape again

    def __init__(self, precision="fp32_ir", nu1=2, nu2=2, ir_inner_cycles=2, device=None,
                 descriptors=True):
        import torch

        import paper_2602_01888_amd as tomg
        self.tomg, self.torch = tomg, torch
        self.descriptors = descriptors  # set requests that carry them up from descriptors
        self.kw = dict(precision=precision, nu1=nu1, nu2=nu2, ir_inner_cycles=ir_inner_cycles)
        self.device = torch.device("cuda") if device is None else torch.device(device)

    def footprint(self, req: Request) -> int:
        cfg = self.tomg.make_config(req.nx, req.ny, req.dx, req.dy, req.xi0, req.eta0,
                                    neumann=req.neumann, flux=req.flux,
                                    semi_levels=req.semi_levels, semi_axis=req.semi_axis,
                                    **self.kw)
        return self.tomg.workspace_bytes(cfg) + 8 * req.nx * req.ny

    def transient(self, req: Request) -> int:
        if self._by_desc(req):  # evaluated in the setup kernel: no input arrays
            return 0
        # coordinates, analytic partials or mask, initial guess and source
        return 8 * req.nx * req.ny * 8

    def _by_desc(self, req: Request) -> bool:
        return self.descriptors and req.map_desc is not None and req.source_desc is not None

    def create(self, req: Request, reuse=None):
        """Problem with its coefficient setup queued (checks deferred): a new
        one, or `reuse` (an evicted problem of the same shape, whose
        workspace the new setup overwrites); returns (problem, phi)."""
        p = reuse if reuse is not None else self.tomg.Problem(
            req.nx, req.ny, req.dx, req.dy, req.xi0, req.eta0, device=self.device,
            neumann=req.neumann, flux=req.flux, semi_levels=req.semi_levels,
            semi_axis=req.semi_axis, **self.kw)
        if self._by_desc(req):
            with self.torch.cuda.stream(p.stream):
                phi = self.torch.empty((req.ny, req.nx), dtype=self.torch.float64,
                                       device=self.device)
            p.setup_desc(self.tomg.map_desc(**req.map_desc),
                         self.tomg.source_desc(**req.source_desc), phi_init=phi, check=False)
            return p, phi
        g = req.geometry()
        rho = req.source()
        if g.get("jac") is not None:
            p.setup_coeffs(rho, jac=g["jac"], mask=g.get("mask"), check=False)
        else:
            p.setup_coeffs(rho, xp=g["xp"], yp=g["yp"], mask=g.get("mask"), check=False)
        return p, g["phi0"].clone()

    def diagnose(self, problem):
        """(status, message) for a problem whose step gave a non-finite
        residual: the deferred setup checks if they failed, else
        non-finite values in the iteration."""
        try:
            problem.setup_check()
        except self.tomg.TomgError as e:
            return e.status, str(e)
        return TOMG_ENONFINITE, "non-finite residual"

    def new_source(self, problem, req: Request):
        if problem.from_map and self._by_desc(req):
            problem.update_rhs_desc(self.tomg.source_desc(**req.source_desc))
        else:
            problem.update_rhs(req.source())

    def step(self, problems, phis, fresh):
        return self.tomg.batch_step(problems, phis, fresh)

    def launch(self, problems, phis, fresh):
        """Queues one batched step (tomg_batch_launch) and returns a handle for
        collect(): the residuals travel to pinned host memory behind the step,
        and an event marks their arrival."""
        torch = self.torch
        stream = problems[0].stream
        n = len(problems)
        with torch.cuda.stream(stream):
            dev = torch.empty(n, dtype=torch.float64, device=self.device)
            self.tomg.batch_launch(problems, phis, fresh, dev)
            host = torch.empty(n, dtype=torch.float64, pin_memory=True)
            host.copy_(dev, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev, host, dev

    def collect(self, handle):
        ev, host, _ = handle
        ev.synchronize()
        return host.tolist()

    def copy(self, phi):
        return phi.clone()


class Server:
    def __init__(self, backend, budget_bytes: int = 64 << 30, rel_tol: float = 1e-10,
                 max_cycles: int = 100, max_active: int = 256, keep_results: bool = False,
                 clock: Callable[[], float] = time.perf_counter, pipeline: bool = True):
        self.backend = backend
        # with a backend that can queue a step without waiting for it, the
        # next step's admissions are prepared on the host while the device
        # runs the current one
        self.pipeline = bool(pipeline) and hasattr(backend, "launch")
        self.budget = int(budget_bytes)
        self.rel_tol = rel_tol
        self.max_cycles = max_cycles
        self.max_active = max_active
        self.keep = keep_results
        self.clock = clock
        self.queue: deque = deque()
        self.active: List[_Active] = []
        self.resident: "OrderedDict[Hashable, _Resident]" = OrderedDict()  # LRU order
        self.used = 0
        self.stats = {"admitted": 0, "warm": 0, "cold": 0, "evicted": 0, "steps": 0,
                      "rejected": 0, "reused": 0}

    # -- queue ------------------------------------------------------------
    def submit(self, req: Request):
        self.queue.append(req)

    @property
    def idle(self):
        return not self.active and not self.queue

    # -- memory -----------------------------------------------------------
    def _evict_for(self, need: int, dropped: Optional[list] = None) -> bool:
        """Evicts idle geometries (least recently used first) until `need`
        more bytes fit; False if they cannot be made to fit.  The (shape,
        problem) of each evicted geometry is appended to `dropped`."""
        if self.used + need <= self.budget:
            return True
        idle = [r for r in self.resident.values() if not r.busy]
        free = sum(r.nbytes for r in idle)
        if self.used - free + need > self.budget:
            return False
        for r in idle:
            if self.used + need <= self.budget:
                break
            if dropped is not None:
                dropped.append((r.shape, r.problem))
            self._drop(r)
            self.stats["evicted"] += 1
        return True

    def _drop(self, r: _Resident):
        del self.resident[r.key]
        self.used -= r.nbytes
        r.problem = r.phi = None

    # -- admission ---------------------------------------------------------
    def _admit(self, now: float, done: list):
        passed = deque()
        while self.queue and len(self.active) < self.max_active:
            req = self.queue.popleft()
            res = self.resident.get(req.geom)
            if res is not None and res.busy:
                passed.append(req)  # its geometry is being solved: try again later
                continue
            if req.warm and res is not None:
                self.resident.move_to_end(req.geom)
                res.busy = True
                try:
                    self.backend.new_source(res.problem, req)
                except Exception as e:  # a failed update leaves the geometry usable
                    res.busy = False
                    done.append(self._failed(req, now, e))
                    continue
                act = _Active(req, res, now, warm_start=True)
                self.stats["warm"] += 1
            else:
                if res is not None:  # a cold request rebuilds its geometry
                    self._drop(res)
                need = self.backend.footprint(req)
                if need + self.backend.transient(req) > self.budget:
                    done.append(self._failed(req, now, MemoryError(
                        f"request needs {need} bytes, budget {self.budget}")))
                    self.stats["rejected"] += 1
                    continue
                dropped = []
                if not self._evict_for(need + self.backend.transient(req), dropped):
                    self.queue.appendleft(req)  # first come, first served: wait
                    break
                # a geometry evicted for this request that had the same shape
                # gives its problem (and workspace) to it instead of a new one
                reuse = None
                if getattr(self.backend, "reuses", False):
                    reuse = next((pb for sh, pb in dropped if sh == req.shape), None)
                try:
                    if reuse is not None:
                        prob, phi = self.backend.create(req, reuse=reuse)
                        self.stats["reused"] += 1
                    else:
                        prob, phi = self.backend.create(req)
                except Exception as e:
                    done.append(self._failed(req, now, e))
                    continue
                res = _Resident(req.geom, prob, phi, need, busy=True, shape=req.shape)
                self.resident[req.geom] = res
                self.used += need
                act = _Active(req, res, now, warm_start=False)
                self.stats["cold"] += 1
            act.queue_depth = len(self.queue) + len(passed)
            act.hbm_used = self.used
            if self.keep:
                act.phi_start = self.backend.copy(res.phi)
            self.active.append(act)
            self.stats["admitted"] += 1
        while passed:
            self.queue.appendleft(passed.pop())

    def _failed(self, req, now, exc):
        status = getattr(exc, "status", -1)
        return Completion(req.rid, status, 0, math.nan, req.arrival, now, now, False,
                          error=str(exc))

    # -- one step ------------------------------------------------------------
    def _groups(self, acts):
        """One batched step per kind of request (level-0 operator form, on
        the fly or stored, and semi-coarsened levels): the positions in
        `acts` of each non-empty group, in order of first appearance."""
        out = OrderedDict()
        for k, a in enumerate(acts):
            out.setdefault(a.req.step_kind, []).append(k)
        return list(out.values())

    def _args(self, acts, grp):
        return ([acts[k].res.problem for k in grp], [acts[k].res.phi for k in grp],
                [acts[k].fresh for k in grp])

    def step(self) -> List[Completion]:
        """Admits what fits, advances every active problem by one step and
        returns the requests that completed.  Pipelined, the requests that
        arrive meanwhile are admitted (their setups queued) while the step
        runs on the device, and join the next step."""
        done: List[Completion] = []
        if not self.pipeline or not self.active:
            self._admit(self.clock(), done)
        if not self.active:
            return done
        acts = list(self.active)
        rels = [math.nan] * len(acts)
        groups = self._groups(acts)
        if self.pipeline:
            handles = [self.backend.launch(*self._args(acts, g)) for g in groups]
            self._admit(self.clock(), done)
            outs = [self.backend.collect(h) for h in handles]
        else:
            outs = [self.backend.step(*self._args(acts, g)) for g in groups]
        for grp, out in zip(groups, outs):
            for k, r in zip(grp, out):
                rels[k] = r
        t = self.clock()
        self.stats["steps"] += 1
        joined = self.active[len(acts):]  # admitted while the step ran
        keep = []
        for a, r in zip(acts, rels):
            if a.fresh:
                a.fresh = False
            else:
                a.cycles += 1
            a.rel = r
            err = ""
            if not math.isfinite(r):
                st, err = TOMG_ENONFINITE, "non-finite residual"
                diagnose = getattr(self.backend, "diagnose", None)
                if diagnose is not None:
                    st, err = diagnose(a.res.problem)
            elif r <= self.rel_tol:
                st = TOMG_OK
            elif a.cycles >= self.max_cycles:
                st = TOMG_ENOCONV
            else:
                keep.append(a)
                continue
            c = Completion(a.req.rid, st, a.cycles, r, a.req.arrival, a.admitted, t,
                           a.warm_start, a.queue_depth, a.hbm_used, error=err)
            if self.keep:
                c.phi = self.backend.copy(a.res.phi)
                c.phi_start = a.phi_start
            a.res.busy = False
            if err:  # a failed setup or a diverged iterate is not kept for re-use
                self._drop(a.res)
            else:
                self.resident.move_to_end(a.res.key)
            done.append(c)
        self.active = keep + joined
        return done

    # -- drivers ---------------------------------------------------------------
    def drain(self) -> List[Completion]:
        """Steps until every submitted request has completed."""
        out = []
        while not self.idle:
            out += self.step()
        return out

    def run_open_loop(self, requests: List[Request], t0: Optional[float] = None,
                      sleep=time.sleep) -> List[Completion]:
        """Submits each request when the clock passes t0 + request.arrival
        (requests sorted by arrival) and steps until all have completed;
        completion times and arrivals are reported on the same clock."""
        t0 = self.clock() if t0 is None else t0
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        for r in pending:
            r.arrival = t0 + r.arrival
        out = []
        total = len(pending)
        while len(out) < total:
            now = self.clock()
            while pending and pending[0].arrival <= now:
                self.submit(pending.popleft())
            if self.idle:
                if pending:
                    sleep(max(0.0, pending[0].arrival - self.clock()))
                continue
            out += self.step()
        return out


def percentile(xs, q):
    """q-th percentile (0..100) by linear interpolation between order statistics."""
    s = sorted(xs)
    if not s:
        return math.nan
    k = (len(s) - 1) * q / 100.0
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    return s[lo] + (s[hi] - s[lo]) * (k - lo)

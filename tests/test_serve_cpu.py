"""Host logic of the continuous-batching server (admission, memory budget,
eviction, warm re-solves, retirement, latency) with a fake backend: no GPU,
no solver arithmetic.  The fake problem's relative residual falls by a
fixed factor per step, so cycle counts are known in advance."""

import math

import pytest

from paper_2602_01888_amd import serve as S


class FakeProblem:
    def __init__(self, req, rate):
        self.req = req
        self.rate = rate
        self.rhs_updates = 0


class FakeBackend:
    def __init__(self, rate=0.1, bytes_per_node=10, fail_on=()):
        self.rate = rate
        self.bpn = bytes_per_node
        self.created = []
        self.steps = []
        self.fail_on = set(fail_on)

    def footprint(self, req):
        return self.bpn * req.nx * req.ny

    def transient(self, req):
        return 0

    def create(self, req):
        if req.rid in self.fail_on:
            raise RuntimeError("bad geometry")
        self.created.append(req.rid)
        p = FakeProblem(req, self.rate)
        return p, {"rel": 1.0}

    def new_source(self, problem, req):
        problem.rhs_updates += 1

    def step(self, problems, phis, fresh):
        self.steps.append([p.req.rid for p in problems])
        out = []
        for p, phi, f in zip(problems, phis, fresh):
            if f:
                phi["rel0"] = phi["rel"]
            else:
                phi["rel"] *= p.rate
            out.append(phi["rel"])
        return out

    def copy(self, phi):
        return dict(phi)


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1.0
        return self.t


def req(rid, n=10, geom=None, warm=False, arrival=0.0):
    return S.Request(rid, geom if geom is not None else f"g{rid}", n, n, 0.1, 0.1,
                     geometry=lambda: {}, source=lambda: None, warm=warm, arrival=arrival)


def test_cycles_and_completion_order():
    be = FakeBackend(rate=0.1)
    s = S.Server(be, budget_bytes=10 ** 6, rel_tol=2e-3, clock=Clock())
    s.submit(req(0))
    s.submit(req(1))
    done = s.drain()
    # first step evaluates norms only, then 3 cycles: 1e-1, 1e-2, 1e-3
    assert [c.rid for c in done] == [0, 1]
    assert all(c.ok and c.cycles == 3 for c in done)
    assert len(be.steps) == 4 and be.steps[0] == [0, 1]


def test_late_arrival_joins_next_step():
    be = FakeBackend(rate=0.1)
    s = S.Server(be, budget_bytes=10 ** 6, rel_tol=2e-3, clock=Clock())
    s.submit(req(0))
    s.step()
    s.step()
    s.submit(req(1))
    s.step()
    assert be.steps[-1] == [0, 1]  # admitted while 0 is still iterating


def test_memory_budget_is_first_come_first_served():
    be = FakeBackend(rate=0.1, bytes_per_node=10)
    # budget fits two 10x10 problems (1000 B each) but not three
    s = S.Server(be, budget_bytes=2500, rel_tol=2e-3, clock=Clock())
    for k in range(3):
        s.submit(req(k))
    s.step()
    assert be.steps[0] == [0, 1]
    assert [r.rid for r in s.queue] == [2]
    done = s.drain()
    assert sorted(c.rid for c in done) == [0, 1, 2]
    assert s.stats["evicted"] >= 1  # an idle geometry made room for request 2
    assert s.used <= 2500


def test_no_overtaking_when_head_does_not_fit():
    be = FakeBackend(rate=0.1, bytes_per_node=10)
    s = S.Server(be, budget_bytes=2500, rel_tol=2e-3, clock=Clock())
    s.submit(req(0, n=10))   # 1000 B
    s.submit(req(1, n=14))   # 1960 B: does not fit beside 0
    s.submit(req(2, n=5))    # 250 B: would fit, but must not overtake 1
    s.step()
    assert be.steps[0] == [0]
    assert [r.rid for r in s.queue] == [1, 2]


def test_request_larger_than_budget_is_rejected():
    be = FakeBackend(bytes_per_node=10)
    s = S.Server(be, budget_bytes=500, clock=Clock())
    s.submit(req(0, n=10))
    (c,) = s.step()
    assert not c.ok and "budget" in c.error
    assert s.idle


def test_warm_request_reuses_resident_geometry():
    be = FakeBackend(rate=0.1)
    s = S.Server(be, budget_bytes=10 ** 6, rel_tol=2e-3, clock=Clock())
    s.submit(req(0, geom="A"))
    (c0,) = s.drain()
    s.submit(req(1, geom="A", warm=True))
    (c1,) = s.drain()
    assert be.created == [0]                 # no second setup
    assert c1.warm_start and not c0.warm_start
    assert s.resident["A"].problem.rhs_updates == 1
    # warm start from the last solution: already below tolerance after the norms
    assert c1.cycles == 0 and c1.ok


def test_warm_request_after_eviction_is_served_cold():
    be = FakeBackend(rate=0.1, bytes_per_node=10)
    s = S.Server(be, budget_bytes=1500, rel_tol=2e-3, clock=Clock())
    s.submit(req(0, geom="A"))
    s.drain()
    s.submit(req(1, geom="B"))  # evicts A
    s.drain()
    s.submit(req(2, geom="A", warm=True))
    (c,) = s.drain()
    assert not c.warm_start and be.created == [0, 1, 2]


def test_busy_geometry_is_passed_over_not_blocking():
    be = FakeBackend(rate=0.1)
    s = S.Server(be, budget_bytes=10 ** 6, rel_tol=2e-3, clock=Clock())
    s.submit(req(0, geom="A"))
    s.step()
    s.submit(req(1, geom="A", warm=True))  # A is busy
    s.submit(req(2, geom="B"))
    s.step()
    assert be.steps[-1] == [0, 2]
    assert [r.rid for r in s.queue] == [1]
    done = s.drain()
    assert sorted(c.rid for c in done) == [0, 1, 2]


def test_nonconvergence_and_nonfinite():
    be = FakeBackend(rate=0.5)
    s = S.Server(be, budget_bytes=10 ** 6, rel_tol=1e-9, max_cycles=5, clock=Clock())
    s.submit(req(0))
    (c,) = s.drain()
    assert c.status == S.TOMG_ENOCONV and c.cycles == 5

    class NanBackend(FakeBackend):
        def step(self, problems, phis, fresh):
            return [math.nan for _ in problems]
    s = S.Server(NanBackend(), budget_bytes=10 ** 6, clock=Clock())
    s.submit(req(1))
    (c,) = s.drain()
    assert c.status == S.TOMG_ENONFINITE


def test_failed_setup_is_reported_and_others_continue():
    be = FakeBackend(rate=0.1, fail_on={1})
    s = S.Server(be, budget_bytes=10 ** 6, rel_tol=2e-3, clock=Clock())
    for k in range(3):
        s.submit(req(k))
    done = s.drain()
    by = {c.rid: c for c in done}
    assert not by[1].ok and "bad geometry" in by[1].error
    assert by[0].ok and by[2].ok


def test_max_active():
    be = FakeBackend(rate=0.1)
    s = S.Server(be, budget_bytes=10 ** 6, rel_tol=2e-3, max_active=2, clock=Clock())
    for k in range(5):
        s.submit(req(k))
    s.step()
    assert len(be.steps[0]) == 2
    assert len(s.drain()) == 5


def test_open_loop_latency():
    class T:
        t = 0.0
    t = T()

    def clock():
        return t.t

    def sleep(dt):
        t.t += dt

    class TimedBackend(FakeBackend):
        def step(self, problems, phis, fresh):
            t.t += 0.01  # every step takes 10 ms
            return super().step(problems, phis, fresh)

    s = S.Server(TimedBackend(rate=0.1), budget_bytes=10 ** 6, rel_tol=2e-3, clock=clock)
    reqs = [req(0, arrival=0.0), req(1, arrival=1.0)]
    done = s.run_open_loop(reqs, t0=0.0, sleep=sleep)
    lat = {c.rid: c.latency for c in done}
    # four steps of 10 ms each (norms + 3 cycles), no queueing
    assert lat[0] == pytest.approx(0.04) and lat[1] == pytest.approx(0.04)


def test_percentile():
    xs = list(range(101))
    assert S.percentile(xs, 50) == 50 and S.percentile(xs, 99) == 99
    assert S.percentile([1.0, 2.0], 50) == 1.5


class _Queued:
    """Mixin: launch/collect over the backend's step (a pipelined backend)."""

    def launch(self, problems, phis, fresh):
        return self.step(problems, phis, fresh)

    def collect(self, handle):
        return handle


@pytest.mark.parametrize("pipelined", [False, True])
def test_deferred_setup_failure_is_diagnosed_and_dropped(pipelined):
    """A setup whose checks fail on the device shows up as a non-finite first
    residual; the server reports the backend's diagnosis and does not keep
    the geometry for warm re-use (serial and pipelined server)."""
    class DeferredBackend(FakeBackend):
        def step(self, problems, phis, fresh):
            out = super().step(problems, phis, fresh)
            return [math.nan if p.req.rid == 1 else r for p, r in zip(problems, out)]

        def diagnose(self, problem):
            return -3, f"det J <= 0 in request {problem.req.rid}"

    cls = type("QueuedDeferred", (_Queued, DeferredBackend), {}) if pipelined else DeferredBackend
    be = cls(rate=0.1)
    s = S.Server(be, budget_bytes=10 ** 6, rel_tol=2e-3, clock=Clock())
    assert s.pipeline == pipelined
    for k in range(3):
        s.submit(req(k))
    by = {c.rid: c for c in s.drain()}
    assert by[1].status == -3 and "request 1" in by[1].error and by[1].cycles == 0
    assert by[0].ok and by[2].ok
    assert "g1" not in s.resident and "g0" in s.resident and "g2" in s.resident
    assert s.used == sum(r.nbytes for r in s.resident.values())


def test_operator_forms_step_in_separate_batches():
    """Requests with a stored level-0 stencil (Neumann edges, flux form) and
    on-the-fly ones are advanced in one backend step per form; each request
    keeps its own sequence of residuals."""
    be = FakeBackend(rate=0.1)
    s = S.Server(be, budget_bytes=10 ** 6, rel_tol=2e-3, clock=Clock())
    r0, r1, r2, r3 = req(0), req(1), req(2), req(3)
    r1.neumann = 4 | 8
    r3.flux = True
    for r in (r0, r1, r2, r3):
        s.submit(r)
    done = s.drain()
    assert sorted(c.rid for c in done) == [0, 1, 2, 3] and all(c.ok for c in done)
    assert all(c.cycles == 3 for c in done)
    # every server step made two backend steps: on the fly, then stored
    assert be.steps[:2] == [[0, 2], [1, 3]]
    assert all(set(a) in ({0, 2}, {1, 3}) for a in be.steps)


def test_serving_stream_default_kinds_unchanged():
    """The annulus kind is opt-in: the default stream draws circle and
    sinusoidal geometries exactly as before (one integer draw of 2)."""
    import workloads as w
    a = w.serving_stream(50, rate=100.0, seed=3)
    b = w.serving_stream(50, rate=100.0, seed=3, kinds=("circle", "sinusoidal"))
    assert a == b
    assert {d["kind"] for d in a} == {"circle", "sinusoidal"}
    c = w.serving_stream(50, rate=100.0, seed=3, kinds=("circle", "annulus"))
    assert [d["kind"] == "circle" for d in c] == [d["kind"] == "circle" for d in a]


def test_evicted_problem_of_the_same_shape_is_reused():
    """Under memory pressure a geometry evicted for a cold request hands its
    problem to the request when the shapes match (no new problem); the
    accounting is unchanged."""
    class Reusing(FakeBackend):
        reuses = True

        def create(self, req, reuse=None):
            p, phi = super().create(req)
            p.reused_from = None if reuse is None else reuse.req.rid
            return p, phi

    be = Reusing(rate=0.1, bytes_per_node=10)
    s = S.Server(be, budget_bytes=10 * 100 * 2, rel_tol=2e-3, clock=Clock())
    s.submit(req(0))             # shape 10 x 10: 1000 bytes
    s.submit(req(1))
    s.drain()                    # both idle and resident: budget full
    s.submit(req(2))             # same shape: evicts geometry 0 and reuses its problem
    s.submit(req(3, n=5))        # other shape: evicts geometry 1, new problem
    s.drain()
    assert s.stats["reused"] == 1 and s.stats["evicted"] == 2
    res = {r.key: r for r in s.resident.values()}
    assert res["g2"].problem.reused_from == 0
    assert res["g3"].problem.reused_from is None
    assert s.used == 1000 + 250


class PipeBackend(FakeBackend):
    """A backend that queues a step (launch) and waits for it later
    (collect); the log records the order of the calls."""

    def __init__(self, **kw):
        super().__init__(**kw)
        self.log = []

    def create(self, req):
        self.log.append(("create", req.rid))
        return super().create(req)

    def launch(self, problems, phis, fresh):
        self.log.append(("launch", [p.req.rid for p in problems]))
        return self.step(problems, phis, fresh)

    def collect(self, handle):
        self.log.append(("collect",))
        return handle


def _mixed_stream(n):
    out = []
    for k in range(n):
        warm = k % 3 == 2
        out.append(req(k, n=10 + 2 * (k % 4), geom=f"g{k % 5}", warm=warm, arrival=0.1 * k))
    return out


def test_pipelined_admission_runs_while_the_step_is_in_flight():
    be = PipeBackend(rate=0.1)
    s = S.Server(be, budget_bytes=10 ** 6, rel_tol=2e-3, clock=Clock())
    assert s.pipeline
    s.submit(req(0))
    s.step()  # idle server: admit, then launch
    s.submit(req(1))
    s.step()
    # request 1 was created between the launch and the collect of the step
    # that advanced request 0, and joined the step after it
    k = be.log.index(("create", 1))
    assert be.log[k - 1] == ("launch", [0]) and be.log[k + 1] == ("collect",)
    s.step()
    assert be.steps[-1] == [0, 1]


def test_pipelined_server_gives_the_serial_results():
    def run(backend, pipeline):
        s = S.Server(backend, budget_bytes=4000, rel_tol=2e-3, clock=Clock(), pipeline=pipeline,
                     max_active=4)
        done = []
        for r in _mixed_stream(24):
            s.submit(r)
            done += s.step()
        done += s.drain()
        return {c.rid: (c.status, c.cycles, c.rel, c.warm_start) for c in done}, s.stats

    serial, st_serial = run(FakeBackend(rate=0.2), False)
    piped, st_piped = run(PipeBackend(rate=0.2), True)
    assert sorted(serial) == sorted(piped) == list(range(24))
    assert serial == piped
    assert st_serial["evicted"] > 0 and st_piped["evicted"] > 0


def test_serial_backend_is_not_pipelined():
    s = S.Server(FakeBackend(), budget_bytes=10 ** 6, pipeline=True)
    assert not s.pipeline
    s = S.Server(PipeBackend(), budget_bytes=10 ** 6, pipeline=False)
    assert not s.pipeline


def test_completion_records_queue_depth_and_hbm_in_use():
    """Each completion carries the queue depth and the bytes the server held
    when its request was admitted (the per-request serving record)."""
    be = FakeBackend(rate=0.1, bytes_per_node=10)
    s = S.Server(be, budget_bytes=10 ** 6, rel_tol=2e-3, max_active=2, clock=Clock())
    for k in range(5):
        s.submit(req(k))
    done = {c.rid: c for c in s.drain()}
    assert done[0].queue_depth == 4 and done[0].hbm_used == 1000
    assert done[1].queue_depth == 3 and done[1].hbm_used == 2000
    # later requests are admitted once the first two retire (their
    # geometries stay resident: the server holds their bytes too)
    assert done[2].queue_depth <= 2 and done[2].hbm_used >= 3000
    assert all(c.admitted >= c.arrival for c in done.values())


def test_one_step_group_per_kind():
    """Requests on semi-coarsened levels (per axis and count) and requests
    with a stored level-0 stencil are each stepped in a batch of their own;
    the groups follow the order in which their kinds first appear."""
    be = FakeBackend(rate=0.1)
    s = S.Server(be, budget_bytes=10 ** 6, rel_tol=2e-3, clock=Clock())
    rs = [req(k) for k in range(6)]
    rs[1].semi_levels = 2
    rs[3].semi_levels, rs[3].semi_axis = 2, "y"
    rs[4].semi_levels = 2
    rs[5].neumann = 1  # a Neumann west edge: stored level-0 stencil
    assert rs[0].step_kind != rs[1].step_kind != rs[3].step_kind != rs[5].step_kind
    for r in rs:
        s.submit(r)
    s.step()
    assert be.steps == [[0, 2], [1, 4], [3], [5]]
    # With no semi-coarsening the axis does not split a group.
    r6, r7 = req(6), req(7)
    r7.semi_axis = "y"
    assert r6.step_kind == r7.step_kind

"""Batched execution (tomg_solve_batch): every problem's result is bitwise
the result of solving it alone (same cycles, same iterate; the residual norm
may differ in the last bits since a batched pass sums it over other blocks),
in both precisions, and a problem that fails leaves the others untouched."""

import numpy as np
import pytest

import oracle
from oracle import direct
import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tomg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_01888_amd as t
    return t


def mixed_batch(count, sides=(65, 129, 257)):
    return w.batch_mixed(count, base_seed=2000, sides=sides)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_batch_equals_alone(tomg, precision):
    probs = mixed_batch(14) + [w.perturbed_circle(129, seed=5), w.manufactured_sinusoidal(65)]
    print(f"[batch] {len(probs)} problems {precision}", flush=True)
    ps, ds = zip(*[tomg.setup_from_grid(q, precision=precision) for q in probs])
    phis = [d["phi0"].clone() for d in ds]
    res = tomg.solve_batch(list(ps), phis, rel_tol=1e-10, max_cycles=60)
    assert all(r.ok for r in res), res
    for p, d, phi, r in zip(ps, ds, phis, res):
        alone = d["phi0"].clone()
        ra = p.solve(alone, rel_tol=1e-10, max_cycles=60)
        # same iterate; the batched norm sums its partials in another order
        assert ra.cycles == r.cycles and abs(ra.rel - r.rel) <= 1e-12 * ra.rel
        assert bool((alone == phi).all())


@pytest.mark.parametrize("nu", [(1, 1), (2, 1), (1, 3), (2, 2)])
def test_chained_inner_cycles_equal_batched(tomg, nu):
    """With a stored level-0 stencil a problem solved alone runs its FP32
    inner cycles chained (the level-0 up pass of a cycle and the down pass of
    the next in one launch, nu2 + nu1 sweeps); a batch runs them as separate
    passes.  Both are the same relaxations in the same order: bitwise equal
    iterates, for 2, 3 and 4 chained sweeps."""
    probs = [w.polar_semi_annulus(65, neumann=True), w.perturbed_circle(129, seed=6)]
    probs[1].neumann = 4 | 2  # Neumann south and east edges
    print(f"[chained] nu {nu}", flush=True)
    kw = dict(precision="fp32_ir", nu1=nu[0], nu2=nu[1], ir_inner_cycles=3)
    ps, ds = zip(*[tomg.setup_from_grid(q, **kw) for q in probs])
    phis = [d["phi0"].clone() for d in ds]
    res = tomg.solve_batch(list(ps), phis, rel_tol=1e-10, max_cycles=100)
    assert all(r.ok for r in res), res
    for p, d, phi, r in zip(ps, ds, phis, res):
        alone = d["phi0"].clone()
        ra = p.solve(alone, rel_tol=1e-10, max_cycles=100)
        assert ra.cycles == r.cycles
        assert bool((alone == phi).all())


def test_batch_matches_oracle(tomg):
    probs = mixed_batch(6)
    ps, ds = zip(*[tomg.setup_from_grid(q) for q in probs])
    phis = [d["phi0"].clone() for d in ds]
    res = tomg.solve_batch(list(ps), phis, rel_tol=1e-10)
    for q, phi, r in zip(probs, phis, res):
        s = oracle.setup(q)
        st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
        ref = direct.direct_solve(st, s["dir"], s["f"], q.phi0)
        g = phi.cpu().numpy()
        assert np.max(np.abs(g - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_failing_problem_does_not_poison_the_batch(tomg):
    good = mixed_batch(4)
    slow = w.polar_semi_annulus(65, ny=33)  # needs ~140 cycles with point smoothing
    probs = good[:2] + [slow] + good[2:]
    ps, ds = zip(*[tomg.setup_from_grid(q) for q in probs])
    phis = [d["phi0"].clone() for d in ds]
    res = tomg.solve_batch(list(ps), phis, rel_tol=1e-10, max_cycles=30)
    assert res[2].status == tomg.TOMG_ENOCONV and res[2].cycles == 30
    for k in (0, 1, 3, 4):
        assert res[k].ok
        alone = ds[k]["phi0"].clone()
        ra = ps[k].solve(alone, rel_tol=1e-10)
        assert ra.cycles == res[k].cycles and bool((alone == phis[k]).all())


def test_single_problem_batch_and_empty(tomg):
    q = w.manufactured_sinusoidal(129)
    p, d = tomg.setup_from_grid(q)
    phi = d["phi0"].clone()
    (r,) = tomg.solve_batch([p], [phi])
    assert r.ok
    assert tomg.solve_batch([], []) == []


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_batch_launch_equals_batch_step(tomg, precision):
    """tomg_batch_launch queues the step of tomg_batch_step: over a few steps
    with problems joining late (fresh) the residuals land at the inputs'
    positions and equal batch_step's, and the iterates are bitwise equal."""
    import torch
    probs = mixed_batch(6) + [w.perturbed_circle(129, seed=7)]
    print(f"[batch_launch] {len(probs)} problems {precision}", flush=True)
    a = [tomg.setup_from_grid(q, precision=precision) for q in probs]
    b = [tomg.setup_from_grid(q, precision=precision) for q in probs]
    pa, pb = [p for p, _ in a], [p for p, _ in b]
    fa = [d["phi0"].clone() for _, d in a]
    fb = [d["phi0"].clone() for _, d in b]
    n = len(probs)
    fresh = [True] * n
    for step in range(4):
        # problems 1 and 4 join at step 2: fresh while the others iterate
        members = [k for k in range(n) if step >= 2 or k not in (1, 4)]
        fr = [fresh[k] for k in members]
        ra = tomg.batch_step([pa[k] for k in members], [fa[k] for k in members], fr)
        out = torch.full((len(members) + 3,), -1.0, dtype=torch.float64, device="cuda")
        tomg.batch_launch([pb[k] for k in members], [fb[k] for k in members], fr, out)
        torch.cuda.synchronize()
        rb = out.cpu().tolist()
        assert rb[len(members):] == [-1.0] * 3  # nothing past the n entries
        assert np.allclose(ra, rb[:len(members)], rtol=1e-12, atol=0), (step, ra, rb)
        for k in members:
            fresh[k] = False
    for x, y in zip(fa, fb):
        assert bool((x == y).all())


def test_batch_launch_errors(tomg):
    import ctypes as C
    import torch
    from paper_2602_01888_amd import _lib
    p, d = tomg.setup_from_grid(w.perturbed_circle(65, seed=1))
    phi = d["phi0"].clone()
    lib = _lib.load()
    hs = (C.c_void_p * 1)(p._h.value)
    ps = (C.c_void_p * 1)(phi.data_ptr())
    fr = (C.c_int32 * 1)(1)
    assert lib.tomg_batch_launch(hs, ps, 1, fr, None) == tomg.TOMG_EINVAL
    assert lib.tomg_batch_launch(hs, ps, -1, fr, None) == tomg.TOMG_EINVAL
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert lib.tomg_batch_launch(hs, ps, 0, fr, C.c_void_p(out.data_ptr())) == tomg.TOMG_OK
    with pytest.raises(tomg.TomgError):
        tomg.batch_launch([p], [phi], [True], torch.zeros(1, dtype=torch.float32, device="cuda"))
    q = tomg.Problem(65, 65, 1 / 64, 1 / 64)  # no setup: state error, nothing queued
    with pytest.raises(tomg.TomgError) as e:
        tomg.batch_launch([q], [phi], [True], out)
    assert e.value.status == tomg.TOMG_ESTATE
    tomg.batch_launch([p], [phi], [True], out)
    torch.cuda.synchronize()
    (r,) = tomg.batch_step([p], [phi.clone()], [True])
    assert abs(out.item() - r) <= 1e-12 * abs(r)

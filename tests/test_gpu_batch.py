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

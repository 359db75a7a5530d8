"""The cycle driver of solve() (Section 3's V-cycle repeated until the
relative residual of the stopping test is met): a problem that has
converged before queues its first cycles right behind the initial norms,
predicted from its last contraction, with no host check between.  Cycles
queued past convergence do nothing, so every solve returns what checking
after every cycle returns: the same cycle count, bitwise the same iterate,
in FP64 and with FP32 inner cycles; a start that already meets the
tolerance runs no cycle, a non-finite start changes nothing, and
max_cycles = 0 runs none."""

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tomg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_01888_amd as t
    return t


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("tol", [1e-6, 1e-10, 1e-12])
def test_repeated_solves_are_bitwise_equal(tomg, precision, tol):
    import torch
    q = w.perturbed_circle(257, seed=3)
    print(f"[queue] {precision} tol {tol:.0e}", flush=True)
    p, d = tomg.setup_from_grid(q, precision=precision)
    fresh, _ = tomg.setup_from_grid(q, precision=precision)
    first = d["phi0"].clone()
    r1 = fresh.solve(first, rel_tol=tol, max_cycles=100)  # no history: checked per group
    assert r1.ok
    p.solve(d["phi0"].clone(), rel_tol=1e-8, max_cycles=100)  # a history at another tolerance
    for _ in range(2):
        phi = d["phi0"].clone()
        r = p.solve(phi, rel_tol=tol, max_cycles=100)
        assert r.ok and r.cycles == r1.cycles and r.rel == r1.rel
        assert torch.equal(phi, first)


def test_queued_start_edge_cases(tomg):
    import torch
    q = w.perturbed_circle(129, seed=4)
    p, d = tomg.setup_from_grid(q)
    phi = d["phi0"].clone()
    r = p.solve(phi, rel_tol=1e-10)
    assert r.ok and r.cycles > 0
    # the converged iterate as the start: no cycle
    again = phi.clone()
    r0 = p.solve(again, rel_tol=1e-8)
    assert r0.ok and r0.cycles == 0 and torch.equal(again, phi)
    # max_cycles = 0 on an unconverged start: no cycle, ENOCONV, phi untouched
    start = d["phi0"].clone()
    rz = p.solve(start, rel_tol=1e-10, max_cycles=0)
    assert rz.status == tomg.TOMG_ENOCONV and rz.cycles == 0
    assert torch.equal(start, d["phi0"])
    # a non-finite start: ENONFINITE, the queued cycles do nothing
    bad = d["phi0"].clone()
    bad[1, 1] = float("nan")  # a free node next to the outer ring
    ref = bad.clone()
    with pytest.raises(tomg.TomgError) as e:
        p.solve(bad, rel_tol=1e-10)
    assert e.value.status == tomg.TOMG_ENONFINITE
    assert torch.equal(torch.nan_to_num(bad), torch.nan_to_num(ref))
    # and the problem still solves afterwards
    phi2 = d["phi0"].clone()
    assert p.solve(phi2, rel_tol=1e-10).cycles == r.cycles
    assert torch.equal(phi2, phi)

"""The residual history of a solve (tomg_residual_history): the relative
residual at the start and after every cycle, for the per-solve records.
Checked against the solve's own report (cycle count, final residual), the
oracle's history of the same problem (its cycles follow the same
arithmetic), and, batched, the same problem solved alone."""

import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_01888_amd as tomg
    return torch, tomg


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_history_of_a_solve(env, precision):
    torch, tomg = env
    q = w.random_sinusoidal(257, 5)
    p, d = tomg.setup_from_grid(q, precision=precision)
    phi = d["phi0"].clone()
    r = p.solve(phi, rel_tol=1e-10)
    h = p.residual_history()
    print(f"[history] {precision}: {r.cycles} cycles, {['%.1e' % v for v in h]}", flush=True)
    assert len(h) == r.cycles + 1
    assert h[0] == 1.0  # the zero-interior start is the stopping test's reference
    assert h[-1] == r.rel
    assert all(b < a for a, b in zip(h, h[1:]))
    if precision == "fp64":
        # the oracle's cycles: the same residuals up to the rounding of a
        # residual computed at 1e-11 of |f| (about 1e-16 / 1e-11 relative)
        ro = oracle.solve_problem(q, rel_tol=1e-10, hist_len=64)
        assert ro["cycles"] == r.cycles
        np.testing.assert_allclose(h, ro["hist"], rtol=1e-6, atol=1e-14)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_batched_history_matches_alone(env, precision):
    torch, tomg = env
    qs = [w.random_sinusoidal(n, s) for n, s in ((129, 1), (257, 2), (65, 3), (513, 4))]
    ps, ds = zip(*[tomg.setup_from_grid(q, precision=precision) for q in qs])
    phis = [d["phi0"].clone() for d in ds]
    res = tomg.solve_batch(list(ps), phis, rel_tol=1e-10)
    hb = [p.residual_history() for p in ps]
    for p, d, r, h in zip(ps, ds, res, hb):
        assert len(h) == r.cycles + 1 and h[-1] == r.rel
        phi = d["phi0"].clone()
        p.solve(phi, rel_tol=1e-10)
        ha = p.residual_history()
        assert len(ha) == len(h)
        # the batched FP64 cycle sums its norm in another order (taller bands)
        np.testing.assert_allclose(h, ha, rtol=1e-12 if precision == "fp64" else 0.0)


def test_history_validates_arguments(env):
    import ctypes as C
    torch, tomg = env
    q = w.random_sinusoidal(65, 1)
    p, d = tomg.setup_from_grid(q)
    lib = p.lib
    assert lib.tomg_residual_history(None, None, 0, None) == tomg.TOMG_EINVAL
    assert lib.tomg_residual_history(p._h, None, 4, None) == tomg.TOMG_EINVAL
    cnt = C.c_int32()
    assert lib.tomg_residual_history(p._h, None, 0, C.byref(cnt)) == tomg.TOMG_OK

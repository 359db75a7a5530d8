"""Sweep counts other than V(2,2): the fused passes are compiled for nu = 1..4
(halo width 4 nu + 2, halo rows 2 nu + 3, register and LDS rings sized by
nu), the tail and the unfused cycle take nu at run time.  One and two
V-cycles against the oracle's cycle with the same nu (mirror mode, 1e-12),
solves with the oracle's cycle count, FP32 inner cycles by the oracle's
residual, and a batch equal to solving alone."""

import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tomg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_01888_amd as t
    return t


def rel_err(a, b):
    return float(np.max(np.abs(np.asarray(a) - b)) / max(np.max(np.abs(b)), 1e-300))


def np_(t):
    return t.detach().cpu().numpy()


def _annulus_neu():
    return w.polar_semi_annulus(129, neumann=True)


CASES = {
    "circle257": lambda: w.perturbed_circle(257, seed=3),
    "rect129x65": lambda: w.manufactured_sinusoidal(129, ny=65),
    "annulus_neumann129": _annulus_neu,
}
NUS = [(1, 1), (3, 3), (4, 4), (1, 2), (3, 1)]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("nu", NUS)
def test_vcycle_and_solve_match_oracle(tomg, name, nu):
    nu1, nu2 = nu
    q = CASES[name]()
    print(f"[nu] {name} V({nu1},{nu2})", flush=True)
    p, d = tomg.setup_from_grid(q, nu1=nu1, nu2=nu2)
    s = oracle.setup(q)
    mg = oracle.MG.from_setup(s, q.dx, q.dy, mask=q.mask, nu1=nu1, nu2=nu2)
    xg = d["phi0"].clone()
    p.vcycle(xg)
    xo = mg.vcycle(q.phi0, s["f"])
    assert rel_err(np_(xg), xo) <= 1e-12
    p.vcycle(xg)
    xo = mg.vcycle(xo, s["f"])
    assert rel_err(np_(xg), xo) <= 1e-12
    phi = d["phi0"].clone()
    res = p.solve(phi, rel_tol=1e-10, max_cycles=400)
    ro = oracle.solve_problem(q, rel_tol=1e-10, max_cycles=400, nu1=nu1, nu2=nu2)
    print(f"  cycles gpu {res.cycles} oracle {ro['cycles']}", flush=True)
    assert res.ok and res.cycles == ro["cycles"]
    assert rel_err(np_(phi), ro["phi"]) <= 1e-10


@pytest.mark.parametrize("nu", [(1, 1), (3, 3), (4, 4)])
def test_mixed_precision_and_batch(tomg, nu):
    import torch
    nu1, nu2 = nu
    probs = [w.perturbed_circle(257, seed=3), w.manufactured_sinusoidal(129),
             w.random_sinusoidal(513, seed=9)]
    for precision in ("fp32_ir", "fp64"):
        ps, ds = zip(*[tomg.setup_from_grid(q, precision=precision, nu1=nu1, nu2=nu2)
                       for q in probs])
        phis = [d["phi0"].clone() for d in ds]
        res = tomg.solve_batch(list(ps), phis, rel_tol=1e-10, max_cycles=200)
        assert all(r.ok for r in res), res
        for q, p, d, phi, r in zip(probs, ps, ds, phis, res):
            alone = d["phi0"].clone()
            ra = p.solve(alone, rel_tol=1e-10, max_cycles=200)
            assert ra.cycles == r.cycles and bool((alone == phi).all())
            s = oracle.setup(q)
            st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
            b0 = oracle.norm2_free(s["dir"], oracle.residual(st, s["dir"], q.phi0, s["f"]))
            rel = oracle.norm2_free(s["dir"], oracle.residual(st, s["dir"], np_(phi),
                                                              s["f"])) / b0
            assert rel <= 1e-10 * (1 + 1e-6), (precision, rel)
    torch.cuda.synchronize()

"""The symmetric flux (energy) form of the operator on the GPU (tomg_config
flux = 1) against the oracle's flux form, through the C-ABI: the level-0
stencil written at setup to a few roundings (1e-13 of the coefficient
scale), the Galerkin hierarchy, smoothing, V-cycles to 1e-12, solves to the
oracle's solution (1e-10) in the same number of cycles; second order on the
manufactured problem; and the 4097 x 4097 conductor problem checked by the
oracle's own residual."""

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


def _circle_se(n):
    q = w.perturbed_circle(n, seed=8)
    q.neumann = 4 | 2
    return q


CASES = {
    "circle257": lambda: w.perturbed_circle(257),
    "sinusoidal129": lambda: w.manufactured_sinusoidal(129),
    "annulus_neumann65": lambda: w.polar_semi_annulus(65, neumann=True),
    "circle129_SE": lambda: _circle_se(129),
    "rect129x65": lambda: w.manufactured_sinusoidal(129, ny=65),  # dx != dy
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("smoother", ["gs4", "zebra_x"])
def test_flux_parity(tomg, name, smoother):
    import torch
    q = CASES[name]()
    print(f"[flux_parity] {name} {smoother}", flush=True)
    kind = oracle.GS4 if smoother == "gs4" else oracle.ZEBRA_X
    p, d = tomg.setup_from_grid(q, flux=True, smoother=smoother)
    s = oracle.setup(q)
    mg = oracle.MG.from_setup(s, q.dx, q.dy, mask=q.mask, flux=True, smoother=kind)
    st0 = mg.stencil(0)
    assert np.max(np.abs(np_(p.export("stencil", 0)) - st0)) <= 1e-13 * np.max(np.abs(st0))
    for l in range(1, mg.num_levels):
        assert np.array_equal(np_(p.export("dir", l)), mg.dirs(l)), l
        assert rel_err(np_(p.export("stencil", l)), mg.stencil(l)) <= 1e-12, l
    rng = np.random.default_rng(5)
    x0 = q.phi0 + np.where(mg.dirs(0) == 0, rng.normal(size=q.phi0.shape), 0.0)
    xg = torch.tensor(x0, device="cuda")
    p.smooth(xg, 2)
    xo = oracle.smooth(st0, mg.dirs(0), x0, s["f"], kind=kind, sweeps=2)
    assert rel_err(np_(xg), xo) <= 1e-12
    xg = d["phi0"].clone()
    p.vcycle(xg)
    xo = mg.vcycle(q.phi0, s["f"])
    assert rel_err(np_(xg), xo) <= 1e-12
    phi = d["phi0"].clone()
    res = p.solve(phi, rel_tol=1e-10, max_cycles=200)
    ro = oracle.solve_problem(q, rel_tol=1e-10, max_cycles=200, flux=True, smoother=kind)
    print(f"  cycles gpu {res.cycles} oracle {ro['cycles']}", flush=True)
    assert res.ok and res.cycles == ro["cycles"]
    assert rel_err(np_(phi), ro["phi"]) <= 1e-10


def test_flux_second_order(tomg):
    errs = []
    for n in (33, 65, 129, 257):
        q = w.manufactured_sinusoidal(n)
        p, d = tomg.setup_from_grid(q, flux=True)
        phi = d["phi0"].clone()
        assert p.solve(phi, rel_tol=1e-13, max_cycles=200).ok
        errs.append(np.max(np.abs(np_(phi) - q.phi_exact)))
    print(f"[flux_order] {errs}", flush=True)
    assert all(3.6 < errs[k] / errs[k + 1] < 4.4 for k in range(3)), errs


def test_flux_fullsize_conductor(tomg):
    n = 4097
    q = w.perturbed_circle(n, seed=0)
    print(f"[flux_fullsize] {n}", flush=True)
    p, d = tomg.setup_from_grid(q, flux=True)
    phi = d["phi0"].clone()
    res = p.solve(phi, rel_tol=1e-10, max_cycles=100)
    print(f"  cycles {res.cycles} rel {res.rel:.3e}", flush=True)
    assert res.ok
    s = oracle.setup(q)
    st = oracle.flux_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
    b0 = oracle.norm2_free(s["dir"], oracle.residual(st, s["dir"], q.phi0, s["f"]))
    rel = oracle.norm2_free(s["dir"], oracle.residual(st, s["dir"], np_(phi), s["f"])) / b0
    assert rel <= 1e-10 * (1 + 1e-3), rel


@pytest.mark.parametrize("name", ["circle257", "circle129_SE"])
def test_flux_mixed_precision(tomg, name):
    """The flux form with FP32 inner cycles on its rounded stored stencil:
    the oracle's FP64 flux-form residual of the result meets the tolerance
    and the result is as close to the flux-form discrete solution as an FP64
    solve stopped at that tolerance."""
    q = CASES[name]()
    print(f"[flux_mixed] {name}", flush=True)
    p, d = tomg.setup_from_grid(q, flux=True, precision="mixed")
    phi = d["phi0"].clone()
    res = p.solve(phi, rel_tol=1e-10, max_cycles=200)
    assert res.ok
    ro = oracle.solve_problem(q, rel_tol=1e-13, max_cycles=200, flux=True)
    s, mg = ro["setup"], ro["mg"]
    b0 = mg.initial_residual(q.phi0, s["f"])
    rel = oracle.norm2_free(s["dir"], oracle.residual(mg.stencil(0), s["dir"], np_(phi),
                                                      s["f"])) / b0
    print(f"  refinement steps {res.cycles} rel {res.rel:.3e} oracle {rel:.3e}", flush=True)
    assert rel <= 1e-10 * (1 + 1e-6), rel
    e10 = rel_err(oracle.solve_problem(q, rel_tol=1e-10, max_cycles=200, flux=True)["phi"],
                  ro["phi"])
    e = rel_err(np_(phi), ro["phi"])
    print(f"  error vs discrete solution {e:.2e} (FP64 at the same tolerance {e10:.2e})",
          flush=True)
    assert e <= max(10 * e10, 1e-12)

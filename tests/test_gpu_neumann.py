"""Neumann edges on the GPU (zero normal derivative, Section 4.1) against the
oracle, through the C-ABI.

The HIP side writes the folded level-0 stencil once at setup and runs the
unfused cycle (one launch per colour, residual-restriction, prolongation)
with operators that cover the ring.  Parity: flags and the folded level-0
stencil to a few roundings (1e-14 of the coefficient scale); the Galerkin
hierarchy, two smoothing sweeps, the residual and V-cycles to 1e-12 (the
bounds of the all-Dirichlet parity tests); the solve reaches the oracle's
solution to 1e-10 with the same cycle count; the paper's semi-annulus
converges at second order to ln(R/r)/ln(R/a)."""

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


def _circle(n, neu, seed=2):
    q = w.perturbed_circle(n, seed=seed)
    q.neumann = neu
    return q


S, N, W, E = 4, 8, 1, 2
CASES = {
    "annulus65": lambda: w.polar_semi_annulus(65, neumann=True),
    "annulus129x65": lambda: w.polar_semi_annulus(129, ny=65, neumann=True),
    "circle65_SE": lambda: _circle(65, S | E),
    "circle129_WES": lambda: _circle(129, W | E | S, seed=5),
    "circle33_all": lambda: _circle(33, W | E | S | N, seed=1),
    # halving stops at 9 x 8 nodes (14 = 2 x 7): 56 coarsest unknowns, more
    # than the one-block Gauss-Jordan inverse holds, so the band LU is used
    "annulus17x15": lambda: w.polar_semi_annulus(17, ny=15, neumann=True),
}


@pytest.mark.parametrize("name", list(CASES))
def test_setup_and_hierarchy_parity(tomg, name):
    q = CASES[name]()
    print(f"[neumann_setup] {name} {q.nx}x{q.ny} edges {q.neumann}", flush=True)
    p, d = tomg.setup_from_grid(q)
    s = oracle.setup(q)
    mg = oracle.MG.from_setup(s, q.dx, q.dy, mask=q.mask)
    assert np.array_equal(np_(p.export("dir")), s["dir"])
    st0 = mg.stencil(0)
    g0 = np_(p.export("stencil", 0))
    assert np.max(np.abs(g0 - st0)) <= 1e-14 * np.max(np.abs(st0))
    assert mg.num_levels == p.num_levels
    if name != "annulus17x15":  # halving reaches the 5 x 5 bound
        assert p.level_shape(p.num_levels - 1)[0] <= 5
    for l in range(1, mg.num_levels):
        assert p.level_shape(l) == mg.shape(l)
        assert np.array_equal(np_(p.export("dir", l)), mg.dirs(l)), l
        assert rel_err(np_(p.export("stencil", l)), mg.stencil(l)) <= 1e-12, l


@pytest.mark.parametrize("name", ["annulus65", "circle65_SE", "circle129_WES"])
@pytest.mark.parametrize("smoother", ["gs4", "jacobi"])
def test_smoother_residual_and_vcycle_parity(tomg, name, smoother):
    import torch
    q = CASES[name]()
    print(f"[neumann_cycle] {name} {smoother}", flush=True)
    p, d = tomg.setup_from_grid(q, smoother=smoother)
    s = oracle.setup(q)
    kind = oracle.GS4 if smoother == "gs4" else oracle.JACOBI
    mg = oracle.MG.from_setup(s, q.dx, q.dy, mask=q.mask, smoother=kind)
    st0, dir0 = mg.stencil(0), mg.dirs(0)
    rng = np.random.default_rng(1)
    x0 = q.phi0 + np.where(dir0 == 0, rng.normal(size=q.phi0.shape), 0.0)
    xg = torch.tensor(x0, device="cuda")
    p.smooth(xg, 2)
    xo = oracle.smooth(st0, dir0, x0, s["f"], kind=kind, sweeps=2, omega=0.8)
    assert rel_err(np_(xg), xo) <= 1e-12
    r = np_(p.residual(xg))
    ro = oracle.residual(st0, dir0, xo, s["f"])
    assert np.max(np.abs(r - ro)) <= 1e-12 * np.max(np.abs(s["f"])) + 1e-12 * np.max(
        np.abs(st0[4])) * np.max(np.abs(xo))
    # V-cycles from the Dirichlet start
    xg = d["phi0"].clone()
    p.vcycle(xg)
    xo = mg.vcycle(q.phi0, s["f"])
    assert rel_err(np_(xg), xo) <= 1e-12
    for l in range(1, mg.num_levels):
        assert rel_err(np_(p.export("x", l)), mg.level_x(l)) <= 1e-11, l
    p.vcycle(xg)
    xo = mg.vcycle(xo, s["f"])
    assert rel_err(np_(xg), xo) <= 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_solve_matches_oracle(tomg, name):
    import torch
    q = CASES[name]()
    print(f"[neumann_solve] {name}", flush=True)
    p, d = tomg.setup_from_grid(q)
    phi = d["phi0"].clone()
    res = p.solve(phi, rel_tol=1e-10, max_cycles=400)
    ro = oracle.solve_problem(q, rel_tol=1e-10, max_cycles=400)
    print(f"  cycles gpu {res.cycles} oracle {ro['cycles']} rel {res.rel:.3e}", flush=True)
    assert res.ok and ro["status"] == 0
    assert res.cycles == ro["cycles"]
    assert res.rel == pytest.approx(ro["rel"], rel=1e-6)
    assert rel_err(np_(phi), ro["phi"]) <= 1e-10
    # residual_norm agrees with the oracle's norm over every free node
    s = ro["setup"]
    mg = ro["mg"]
    a, _ = p.residual_norm(phi)
    ao = oracle.norm2_free(s["dir"], oracle.residual(mg.stencil(0), s["dir"], np_(phi), s["f"]))
    assert a == pytest.approx(ao, rel=1e-9, abs=1e-14 * mg.initial_residual(q.phi0, s["f"]))
    dmask = s["dir"].astype(bool)
    assert np.array_equal(np_(phi)[dmask], q.phi0[dmask])


def test_semi_annulus_second_order(tomg):
    errs = []
    for n in (65, 129, 257):
        q = w.polar_semi_annulus(n, neumann=True)
        p, d = tomg.setup_from_grid(q)
        phi = d["phi0"].clone()
        assert p.solve(phi, rel_tol=1e-12, max_cycles=400).ok
        errs.append(np.max(np.abs(np_(phi) - q.phi_exact)))
    print(f"[neumann_order] errors {errs}", flush=True)
    assert 3.8 < errs[0] / errs[1] < 4.2 and 3.8 < errs[1] / errs[2] < 4.2, errs


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_stored_stencil_problems_batch(tomg, precision):
    """Neumann-edge and flux-form problems (stored level-0 stencils) batch
    together: the batched launches run (batch_step accepts the set), and
    every result is bitwise the one solve() gives alone, with the same cycle
    count."""
    import torch
    specs = [("annulus65", False), ("annulus129x65", False), ("circle65_SE", False),
             ("circle129_WES", False), ("circle65_SE", True), ("circle33_all", True)]
    print(f"[neumann_batch] {len(specs)} problems {precision}", flush=True)
    ps, ds = zip(*[tomg.setup_from_grid(CASES[name](), precision=precision, flux=flux)
                   for name, flux in specs])
    probe = [d["phi0"].clone() for d in ds]
    tomg.batch_step(list(ps), probe, [True] * len(ps))  # raises unless batchable
    phis = [d["phi0"].clone() for d in ds]
    res = tomg.solve_batch(list(ps), phis, rel_tol=1e-10, max_cycles=400)
    assert all(r.ok for r in res), res
    for p, d, phi, r in zip(ps, ds, phis, res):
        alone = d["phi0"].clone()
        ra = p.solve(alone, rel_tol=1e-10, max_cycles=400)
        assert ra.cycles == r.cycles and abs(ra.rel - r.rel) <= 1e-12 * ra.rel
        assert bool((alone == phi).all())
    torch.cuda.synchronize()


def test_stored_and_on_the_fly_problems_do_not_share_a_batch(tomg):
    """One batched launch serves one level-0 operator form."""
    pn, dn = tomg.setup_from_grid(CASES["circle65_SE"]())
    pd, dd = tomg.setup_from_grid(w.perturbed_circle(65, seed=2))
    with pytest.raises(tomg.TomgError) as e:
        tomg.batch_step([pn, pd], [dn["phi0"].clone(), dd["phi0"].clone()], [True, True])
    assert e.value.status == tomg.TOMG_EINVAL


def test_fullsize_semi_annulus(tomg):
    """4097 x 4097 with the Neumann sides, in the configuration the benchmark
    times: the oracle's own residual of the GPU solution meets the stopping
    tolerance, and the error against the closed form is the discretisation
    error (second order from the sizes above: about 2.9e-7 / 256)."""
    n = 4097
    q = w.polar_semi_annulus(n, neumann=True)
    print(f"[neumann_fullsize] {n}", flush=True)
    p, d = tomg.setup_from_grid(q)
    phi = d["phi0"].clone()
    res = p.solve(phi, rel_tol=1e-10, max_cycles=600)
    print(f"  cycles {res.cycles} rel {res.rel:.3e}", flush=True)
    assert res.ok
    x = np_(phi)
    s = oracle.setup(q)
    st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
    b0 = oracle.norm2_free(s["dir"], oracle.residual(st, s["dir"], q.phi0, s["f"]))
    rel = oracle.norm2_free(s["dir"], oracle.residual(st, s["dir"], x, s["f"])) / b0
    assert rel <= 1e-10 * (1 + 1e-3), rel
    res = p.solve(phi, rel_tol=1e-12, max_cycles=600)
    err = np.max(np.abs(np_(phi) - q.phi_exact))
    print(f"  error vs closed form {err:.3e}", flush=True)
    assert err <= 2.5e-9


@pytest.mark.parametrize("name", ["annulus65", "annulus129x65", "circle65_SE", "circle129_WES"])
def test_mixed_precision_neumann(tomg, name):
    """FP32 inner cycles on the rounded stored stencil inside FP64
    refinement: the oracle's FP64 residual of the result meets the stopping
    tolerance, and the result is as close to the discrete solution as an FP64
    solve stopped at that tolerance."""
    q = CASES[name]()
    print(f"[neumann_mixed] {name}", flush=True)
    p, d = tomg.setup_from_grid(q, precision="mixed", ir_inner_cycles=2)
    phi = d["phi0"].clone()
    res = p.solve(phi, rel_tol=1e-10, max_cycles=400)
    print(f"  refinement steps {res.cycles} rel {res.rel:.3e}", flush=True)
    assert res.ok
    ro = oracle.solve_problem(q, rel_tol=1e-13, max_cycles=400)
    s, mg = ro["setup"], ro["mg"]
    b0 = mg.initial_residual(q.phi0, s["f"])
    rel = oracle.norm2_free(s["dir"], oracle.residual(mg.stencil(0), s["dir"], np_(phi),
                                                      s["f"])) / b0
    assert rel <= 1e-10 * (1 + 1e-6), rel
    assert rel == pytest.approx(res.rel, rel=1e-6)
    # as close to the discrete solution as an FP64 solve stopped at the same
    # tolerance (the oracle's own iterate), within a factor 10
    e10 = rel_err(oracle.solve_problem(q, rel_tol=1e-10, max_cycles=400)["phi"], ro["phi"])
    e = rel_err(np_(phi), ro["phi"])
    print(f"  error vs discrete solution {e:.2e} (FP64 at the same tolerance {e10:.2e})",
          flush=True)
    assert e <= max(10 * e10, 1e-12)
    dmask = s["dir"].astype(bool)
    assert np.array_equal(np_(phi)[dmask], q.phi0[dmask])


def test_mixed_precision_limits(tomg):
    """A stored level-0 stencil takes FP32 inner cycles with every smoother
    but the alternating zebra (FP64 only)."""
    mk = tomg.make_config
    assert tomg.workspace_bytes(mk(129, 129, 1.0, 1.0, neumann=S, precision="mixed")) > 0
    assert tomg.workspace_bytes(mk(129, 129, 1.0, 1.0, neumann=S, precision="mixed",
                                   smoother="jacobi")) > 0
    assert tomg.workspace_bytes(mk(129, 129, 1.0, 1.0, neumann=S, precision="mixed",
                                   smoother="zebra_x")) > 0
    assert tomg.workspace_bytes(mk(129, 129, 1.0, 1.0, neumann=S, precision="mixed",
                                   smoother="zebra_xy")) == 0


@pytest.mark.parametrize("smoother", ["jacobi", "zebra_x"])
def test_mixed_precision_neumann_unfused_smoothers(tomg, smoother):
    """Neumann edges with damped Jacobi or x-line smoothing and FP32 inner
    cycles (the unfused cycle on the rounded stored stencil): the oracle's
    FP64 residual of the result meets the tolerance; at a tightened
    tolerance the result is the discrete solution to 1e-10."""
    q = CASES["annulus129x65"]()
    print(f"[neumann_mixed_{smoother}] {q.nx}x{q.ny}", flush=True)
    p, d = tomg.setup_from_grid(q, precision="mixed", smoother=smoother, ir_inner_cycles=2)
    phi = d["phi0"].clone()
    res = p.solve(phi, rel_tol=1e-10, max_cycles=400)
    assert res.ok
    ro = oracle.solve_problem(q, rel_tol=1e-13, max_cycles=400)
    s, mg = ro["setup"], ro["mg"]
    b0 = mg.initial_residual(q.phi0, s["f"])
    rel = oracle.norm2_free(s["dir"], oracle.residual(mg.stencil(0), s["dir"], np_(phi),
                                                      s["f"])) / b0
    assert rel <= 1e-10 * (1 + 1e-6), rel
    e10 = rel_err(np_(phi), ro["phi"])
    phi2 = d["phi0"].clone()
    res2 = p.solve(phi2, rel_tol=1e-13, max_cycles=400)
    assert res2.ok
    e13 = rel_err(np_(phi2), ro["phi"])
    print(f"  steps {res.cycles}/{res2.cycles} error vs discrete solution at 1e-10: {e10:.2e}, "
          f"at 1e-13: {e13:.2e}", flush=True)
    assert e13 <= 1e-10


def test_fullsize_semi_annulus_mixed(tomg):
    """4097 x 4097 with the Neumann sides, FP32 inner cycles: the oracle's
    residual of the result meets the tolerance and the error against the
    closed form is that of the FP64 solve."""
    n = 4097
    q = w.polar_semi_annulus(n, neumann=True)
    print(f"[neumann_fullsize_mixed] {n}", flush=True)
    p, d = tomg.setup_from_grid(q, precision="mixed", ir_inner_cycles=4)
    phi = d["phi0"].clone()
    res = p.solve(phi, rel_tol=1e-10, max_cycles=200)
    print(f"  refinement steps {res.cycles} rel {res.rel:.3e}", flush=True)
    assert res.ok
    s = oracle.setup(q)
    st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
    b0 = oracle.norm2_free(s["dir"], oracle.residual(st, s["dir"], q.phi0, s["f"]))
    rel = oracle.norm2_free(s["dir"], oracle.residual(st, s["dir"], np_(phi), s["f"])) / b0
    assert rel <= 1e-10 * (1 + 1e-3), rel
    err = np.max(np.abs(np_(phi) - q.phi_exact))
    print(f"  error vs closed form {err:.3e}", flush=True)
    assert err <= 5e-7

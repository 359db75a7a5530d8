"""Semi-coarsening on the GPU (semi_levels, semi_axis: the first
coarsenings halve one axis only; an extension of the V-cycle of Section 3)
against the oracle, through the C-ABI.

The HIP side builds the semi-coarsened Galerkin levels with their own
setup kernel and runs the fused level passes with the one-axis transfers
down to the coarsest solve.  Parity at the bounds of the full-coarsening
tests: flags exactly, stencils of every level, two V-cycles and each
level's correction to 1e-12 / 1e-11; the solve reaches the oracle's
solution with the same cycle count; FP32 inner cycles reach the converged
oracle solution to 1e-10; and at 4097 x 4097 the semi-annulus of Section
4.1 meets the oracle's residual in far fewer cycles than full coarsening."""

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
# name: (problem, semi_levels, axis)
CASES = {
    "annulus129_neumann_x2": (lambda: w.polar_semi_annulus(129, neumann=True), 2, "x"),
    "annulus129_x1": (lambda: w.polar_semi_annulus(129), 1, "x"),
    "circle129_y2": (lambda: w.perturbed_circle(129), 2, "y"),
    "circle65_SE_y1": (lambda: _circle(65, S | E), 1, "y"),
    "annulus257x129_neumann_x1": (lambda: w.polar_semi_annulus(257, ny=129, neumann=True), 1,
                                  "x"),
    "circle65_all_x3": (lambda: _circle(65, W | E | S | N, seed=1), 3, "x"),
    # the smallest grids: one pass level above a 5 x 9 or 9 x 3 coarsest grid
    "sinus9_x2": (lambda: w.manufactured_sinusoidal(9), 2, "x"),
    "sinus17x9_y1": (lambda: w.manufactured_sinusoidal(17, ny=9), 1, "y"),
    # cells twice as long along the angle: 74 cycles with full coarsening
    "annulus129x65_neumann_x2": (lambda: w.polar_semi_annulus(129, ny=65, neumann=True), 2,
                                 "x"),
}


def _mg(q, semi, axis, **kw):
    s = oracle.setup(q)
    return s, oracle.MG.from_setup(s, q.dx, q.dy, mask=q.mask, semi=semi,
                                   semi_axis=0 if axis == "x" else 1, **kw)


@pytest.mark.parametrize("name", list(CASES))
def test_semi_hierarchy_parity(tomg, name):
    mk, semi, axis = CASES[name]
    q = mk()
    print(f"[semi_setup] {name} {q.nx}x{q.ny} semi {semi} {axis}", flush=True)
    p, d = tomg.setup_from_grid(q, semi_levels=semi, semi_axis=axis)
    s, mg = _mg(q, semi, axis)
    assert mg.num_levels == p.num_levels
    for l in range(mg.num_levels - 1):
        want = (2, 1) if axis == "x" else (1, 2)
        assert mg.strides(l) == (want if l < semi else (2, 2))
    for l in range(1, mg.num_levels):
        assert p.level_shape(l) == mg.shape(l)
        assert np.array_equal(np_(p.export("dir", l)), mg.dirs(l)), l
        assert rel_err(np_(p.export("stencil", l)), mg.stencil(l)) <= 1e-12, l


@pytest.mark.parametrize("name", list(CASES))
def test_semi_vcycle_parity(tomg, name):
    mk, semi, axis = CASES[name]
    q = mk()
    print(f"[semi_cycle] {name}", flush=True)
    p, d = tomg.setup_from_grid(q, semi_levels=semi, semi_axis=axis)
    s, mg = _mg(q, semi, axis)
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
def test_semi_solve_matches_oracle(tomg, name):
    mk, semi, axis = CASES[name]
    q = mk()
    print(f"[semi_solve] {name}", flush=True)
    p, d = tomg.setup_from_grid(q, semi_levels=semi, semi_axis=axis)
    phi = d["phi0"].clone()
    res = p.solve(phi, rel_tol=1e-10, max_cycles=400)
    ro = oracle.solve_problem(q, rel_tol=1e-10, max_cycles=400, semi=semi,
                              semi_axis=0 if axis == "x" else 1)
    print(f"  cycles gpu {res.cycles} oracle {ro['cycles']} rel {res.rel:.3e}", flush=True)
    assert res.ok and ro["status"] == 0
    assert res.cycles == ro["cycles"]
    assert res.rel == pytest.approx(ro["rel"], rel=1e-6)
    assert rel_err(np_(phi), ro["phi"]) <= 1e-10


@pytest.mark.parametrize("name", ["annulus129_neumann_x2", "circle129_y2"])
def test_semi_fp32_inner_cycles_reach_oracle(tomg, name):
    """FP32 inner cycles on the semi-coarsened hierarchy inside FP64
    refinement: the 1e-13 result is within 1e-10 of the oracle's solution
    converged to 1e-13, and the oracle's FP64 residual of the 1e-10 result
    meets that tolerance."""
    mk, semi, axis = CASES[name]
    q = mk()
    print(f"[semi_fp32] {name}", flush=True)
    p32, d = tomg.setup_from_grid(q, semi_levels=semi, semi_axis=axis, precision="fp32_ir")
    ref = oracle.solve_problem(q, rel_tol=1e-13, max_cycles=400, semi=semi,
                               semi_axis=0 if axis == "x" else 1)
    assert ref["status"] == 0
    b = d["phi0"].clone()
    assert p32.solve(b, rel_tol=1e-10, max_cycles=200).ok
    c = d["phi0"].clone()
    r13 = p32.solve(c, rel_tol=1e-13, max_cycles=400)
    assert r13.ok
    e13 = rel_err(np_(c), ref["phi"])
    print(f"  steps {r13.cycles}: error vs oracle at 1e-13 {e13:.2e}", flush=True)
    assert e13 <= 1e-10
    s, mg = ref["setup"], ref["mg"]
    b0 = mg.initial_residual(q.phi0, s["f"])
    rel = oracle.norm2_free(s["dir"], oracle.residual(mg.stencil(0), s["dir"], np_(b),
                                                      s["f"])) / b0
    assert rel <= 1e-10 * (1 + 1e-6), rel


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_semi_batch_equals_alone(tomg, precision):
    """Problems with the same semi-coarsened levels share the batched
    launches (one transfer kind per level): each result is bitwise its
    solve alone, on grids of several sizes and with Neumann and Dirichlet
    edges; a continuous-batching step takes them too."""
    import torch
    stored = [w.polar_semi_annulus(65, neumann=True), w.polar_semi_annulus(129, neumann=True),
              w.polar_semi_annulus(257, ny=129, neumann=True)]
    onfly = [w.polar_semi_annulus(129), w.perturbed_circle(65, seed=3)]
    for probs in (stored, onfly):
        print(f"[semi_batch] {precision} {[(q.nx, q.ny) for q in probs]}", flush=True)
        ps, ds = zip(*[tomg.setup_from_grid(q, semi_levels=2, precision=precision)
                       for q in probs])
        phis = [d["phi0"].clone() for d in ds]
        res = tomg.solve_batch(list(ps), phis, rel_tol=1e-10, max_cycles=100)
        assert all(r.ok for r in res), res
        for p, d, phi, r in zip(ps, ds, phis, res):
            alone = d["phi0"].clone()
            ra = p.solve(alone, rel_tol=1e-10, max_cycles=100)
            assert ra.cycles == r.cycles
            assert torch.equal(alone, phi)
        step = [d["phi0"].clone() for d in ds]
        rel = tomg.batch_step(list(ps), step, [True] * len(ps))
        assert all(np.isfinite(rel))


def test_semi_mixed_with_full_coarsening_in_one_batch(tomg):
    """Different transfers cannot share launches: tomg_solve_batch solves
    such a set one problem after another, each bitwise as alone, and a
    continuous-batching step refuses it."""
    import torch
    q = w.polar_semi_annulus(65, neumann=True)
    p1, d1 = tomg.setup_from_grid(q, semi_levels=1)
    p2, d2 = tomg.setup_from_grid(q)
    phis = [d1["phi0"].clone(), d2["phi0"].clone()]
    res = tomg.solve_batch([p1, p2], phis, rel_tol=1e-10)
    assert all(r.ok for r in res)
    for p, d, phi in ((p1, d1, phis[0]), (p2, d2, phis[1])):
        a = d["phi0"].clone()
        assert p.solve(a, rel_tol=1e-10).ok
        assert torch.equal(a, phi)
    with pytest.raises(tomg.TomgError) as e:
        tomg.batch_step([p1, p2], [d1["phi0"].clone(), d2["phi0"].clone()], [True, True])
    assert e.value.status == tomg.TOMG_EINVAL


def test_fullsize_semi_annulus_semi_coarsening(tomg):
    """4097 x 4097 semi-annulus with Neumann sides, the radial axis halved
    alone for two levels: the oracle's residual of the GPU solution meets
    the tolerance in at most 9 cycles (full coarsening: 15), and the
    solution is within the discretisation error of ln(R/r)/ln(R/a)."""
    n = 4097
    q = w.polar_semi_annulus(n, neumann=True)
    print(f"[semi_fullsize] {n}", flush=True)
    p, d = tomg.setup_from_grid(q, semi_levels=2, semi_axis="x")
    phi = d["phi0"].clone()
    res = p.solve(phi, rel_tol=1e-10, max_cycles=100)
    print(f"  cycles {res.cycles} rel {res.rel:.3e}", flush=True)
    assert res.ok and res.cycles <= 9
    s = oracle.setup(q)
    st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
    b0 = oracle.norm2_free(s["dir"], oracle.residual(st, s["dir"], q.phi0, s["f"]))
    rel = oracle.norm2_free(s["dir"], oracle.residual(st, s["dir"], np_(phi), s["f"])) / b0
    assert rel <= 1e-10 * (1 + 1e-3), rel
    assert np.max(np.abs(np_(phi) - q.phi_exact)) <= 1e-6

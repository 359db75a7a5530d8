"""The 201 x 201 grid of Section 4.1 and its family (101, 401, 801): halving
stops at a 26 x 26 coarsest level, which the library inverts through a band
LU factorisation and solves below the fused passes.  Checked against the
oracle (whose 201 x 201 multigrid solution is pinned to SciPy's direct
solution), at second order against the closed form of eq. 28, and batched
with other problems (bitwise the solve alone)."""

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


@pytest.mark.parametrize("neumann", [True, False])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_semi_annulus_201_matches_oracle(env, neumann, precision):
    torch, tomg = env
    print(f"[coarse201] semi-annulus 201 neumann={neumann} {precision}", flush=True)
    q = w.polar_semi_annulus(201, neumann=neumann)
    p, d = tomg.setup_from_grid(q, precision=precision)
    assert p.num_levels == 4 and p.level_shape(3) == (26, 26)
    phi = d["phi0"].clone()
    r = p.solve(phi, rel_tol=1e-12, max_cycles=200)
    assert r.ok, r
    ro = oracle.solve_problem(q, rel_tol=1e-13, max_cycles=300)
    assert ro["status"] == 0
    err = np.max(np.abs(phi.cpu().numpy() - ro["phi"])) / np.max(np.abs(ro["phi"]))
    print(f"  {r.cycles} cycles, error vs oracle {err:.2e}", flush=True)
    assert err < 1e-10


def test_sinusoidal_201_matches_oracle(env):
    """The on-the-fly eq. 18 level-0 operator with the fused passes down to
    the large coarsest level (no single-workgroup tail)."""
    torch, tomg = env
    q = w.manufactured_sinusoidal(201, amp=0.1)
    p, d = tomg.setup_from_grid(q)
    phi = d["phi0"].clone()
    r = p.solve(phi, rel_tol=1e-12)
    assert r.ok and r.cycles < 20, r
    ro = oracle.solve_problem(q, rel_tol=1e-13)
    err = np.max(np.abs(phi.cpu().numpy() - ro["phi"])) / np.max(np.abs(ro["phi"]))
    print(f"[coarse201] sinusoidal 201: {r.cycles} cycles, error vs oracle {err:.2e}", flush=True)
    assert err < 1e-10


def test_semi_annulus_201_family_second_order(env):
    """eq. 28 (Section 4.1, Neumann sides): the maximum error against
    ln(R/r)/ln(R/a) falls by 4 per halving of h over 101 .. 801."""
    torch, tomg = env
    errs = []
    for n in (101, 201, 401, 801):
        q = w.polar_semi_annulus(n, neumann=True)
        p, d = tomg.setup_from_grid(q)
        assert p.level_shape(p.num_levels - 1) == (26, 26)
        phi = d["phi0"].clone()
        r = p.solve(phi, rel_tol=1e-12, max_cycles=200)
        assert r.ok, (n, r)
        errs.append(float(np.max(np.abs(phi.cpu().numpy() - q.phi_exact))))
    print(f"[coarse201] errors {errs}", flush=True)
    for a, b in zip(errs, errs[1:]):
        assert 3.8 < a / b < 4.2, errs


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_201_in_a_batch_equals_alone(env, precision):
    """A 201 x 201 problem batched with problems of the usual hierarchies
    (its coarsest level solved in the batched tail launch): every result is
    bitwise the solve alone."""
    torch, tomg = env
    qs = [w.manufactured_sinusoidal(201, amp=0.08), w.random_sinusoidal(129, 3),
          w.manufactured_sinusoidal(401, amp=0.05), w.random_sinusoidal(257, 4)]
    ps, ds = zip(*[tomg.setup_from_grid(q, precision=precision) for q in qs])
    phis = [d["phi0"].clone() for d in ds]
    res = tomg.solve_batch(list(ps), phis, rel_tol=1e-10)
    for p, d, r, phi in zip(ps, ds, res, phis):
        assert r.ok, r
        alone = d["phi0"].clone()
        ra = p.solve(alone, rel_tol=1e-10)
        assert ra.cycles == r.cycles
        assert torch.equal(alone, phi)


def test_201_descriptor_setup(env):
    """The polar map descriptor on the 201 x 201 grid (Neumann sides)."""
    torch, tomg = env
    n = 201
    q = w.polar_semi_annulus(n, neumann=True)
    p = tomg.Problem(n, n, q.dx, q.dy, q.xi0, q.eta0, neumann=q.neumann)
    phi = torch.empty((n, n), dtype=torch.float64, device="cuda")
    p.setup_desc(tomg.map_desc("polar", value_in=1.0), tomg.source_desc([], [], 1.0),
                 phi_init=phi)
    r = p.solve(phi, rel_tol=1e-12, max_cycles=200)
    assert r.ok
    err = float(np.max(np.abs(phi.cpu().numpy() - q.phi_exact)))
    assert err < 2e-4, err

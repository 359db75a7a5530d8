"""The embedded-body problems of Section 5.2 on the GPU: grid generation
with the map held on an embedded square's outline (tomg_laplace_grid with a
mask; eq. 44 cylinder, eq. 51 deformed body) against the oracle's grid, and
the potential flow of eq. 47 around the body against the oracle's
solution, on the oracle's grid and end to end on the GPU's own grid."""

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


def rel_err(a, b):
    return float(np.max(np.abs(np.asarray(a) - b)) / max(np.max(np.abs(b)), 1e-300))


def gpu_grid(torch, tomg, n, kind):
    xb, yb, outline = w.embedded_body_boundary(n, kind)
    d = 10.0 / (n - 1)
    p = tomg.Problem(n, n, d, d, -5.0, -5.0)
    xp, yp = torch.as_tensor(xb).cuda(), torch.as_tensor(yb).cuda()
    cyc = p.laplace_grid(xp, yp, rel_tol=1e-13, max_cycles=200,
                         mask=torch.as_tensor(outline).cuda())
    return xp, yp, cyc, (xb, yb, outline, d)


@pytest.mark.parametrize("kind", ["cylinder", "arbitrary"])
@pytest.mark.parametrize("n", [129, 257])
def test_embedded_grid_and_flow_match_oracle(env, kind, n):
    torch, tomg = env
    print(f"[embedded] {kind} {n}", flush=True)
    xp, yp, cyc, (xb, yb, outline, d) = gpu_grid(torch, tomg, n, kind)
    rx, ry = oracle.generate_grid(xb, yb, d, d, rel_tol=1e-13, mask=outline)
    assert rel_err(xp.cpu().numpy(), rx) <= 1e-11 and rel_err(yp.cpu().numpy(), ry) <= 1e-11
    held = outline.astype(bool)
    assert np.array_equal(xp.cpu().numpy()[held], xb[held])
    # the flow on the oracle's grid: same discrete problem, same cycle count
    q = w.embedded_flow(rx, ry)
    p, dd = tomg.setup_from_grid(q)
    phi = dd["phi0"].clone()
    res = p.solve(phi, rel_tol=1e-10, max_cycles=200)
    ro = oracle.solve_problem(q, rel_tol=1e-10, max_cycles=200)
    print(f"  grid cycles {cyc}; flow cycles gpu {res.cycles} oracle {ro['cycles']}", flush=True)
    assert res.ok and res.cycles == ro["cycles"]
    assert rel_err(phi.cpu().numpy(), ro["phi"]) <= 1e-10
    # end to end on the GPU's grid, against the oracle end to end
    qg = w.embedded_flow(xp.cpu().numpy(), yp.cpu().numpy())
    pg, dg = tomg.setup_from_grid(qg)
    phg = dg["phi0"].clone()
    assert pg.solve(phg, rel_tol=1e-12, max_cycles=200).ok
    ref = oracle.solve_problem(q, rel_tol=1e-13, max_cycles=200)["phi"]
    assert rel_err(phg.cpu().numpy(), ref) <= 1e-9


def test_cylinder_flow_converges_to_the_unbounded_flow(env):
    """GPU grid and GPU solve with the outer data of psi = y'(1 - R^2/r'^2):
    the error against that closed form falls with the grid spacing (about
    first order: the outline map is singular at the square's corners)."""
    torch, tomg = env
    errs = []
    for n in (129, 257, 513):
        xp, yp, _, _ = gpu_grid(torch, tomg, n, "cylinder")
        q = w.embedded_flow(xp.cpu().numpy(), yp.cpu().numpy(), data="cylinder_exact")
        p, d = tomg.setup_from_grid(q)
        phi = d["phi0"].clone()
        assert p.solve(phi, rel_tol=1e-12, max_cycles=200).ok
        e = phi.cpu().numpy() - q.phi_exact
        errs.append(float(np.sqrt(np.sum(e ** 2)) / n))
    print(f"[embedded_exact] L2 errors {errs}", flush=True)
    assert errs[0] / errs[1] >= 1.7 and errs[1] / errs[2] >= 1.7


def test_fullsize_cylinder_flow(env):
    """4097 x 4097: GPU grid generation and flow solve; the oracle's residual
    of the GPU solution on the GPU's grid meets the tolerance, and the
    stream function keeps the symmetry of the problem."""
    torch, tomg = env
    n = 4097
    print(f"[embedded_fullsize] {n}", flush=True)
    xp, yp, cyc, _ = gpu_grid(torch, tomg, n, "cylinder")
    q = w.embedded_flow(xp.cpu().numpy(), yp.cpu().numpy())
    p, d = tomg.setup_from_grid(q)
    phi = d["phi0"].clone()
    res = p.solve(phi, rel_tol=1e-10, max_cycles=200)
    print(f"  grid cycles {cyc}; flow cycles {res.cycles} rel {res.rel:.3e}", flush=True)
    assert res.ok
    s = oracle.setup(q)
    st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
    b0 = oracle.norm2_free(s["dir"], oracle.residual(st, s["dir"], q.phi0, s["f"]))
    psi = phi.cpu().numpy()
    rel = oracle.norm2_free(s["dir"], oracle.residual(st, s["dir"], psi, s["f"])) / b0
    assert rel <= 1e-10 * (1 + 1e-3), rel
    assert np.max(np.abs(psi + psi[::-1, :])) <= 1e-8
    assert np.max(np.abs(psi - psi[:, ::-1])) <= 1e-8

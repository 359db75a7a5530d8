"""A geometry that moves in time: the perturbation of the perturbed-circle
conductor rotates from one time step to the next.  At every step the map and
its permittivity tensor are rebuilt (setup_coeffs on the same problem), the
potential is solved starting from the previous step's potential, and the
field is recovered (eq. 2); the conclusion names this time-dependent use of
the method.  Each step is checked against the oracle: the relative residual
by the oracle's operator of that step's map, and the field against the
oracle's field of the same potential.  The stopping test does not depend on
the initial guess, so a warm start from the previous step must take fewer
cycles than a cold one."""

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
    from workloads import device as D
    return torch, tomg, D


def _oracle_rel(q, phi):
    """Relative residual by the oracle: the denominator is the residual of
    the start with the Dirichlet values and zeros elsewhere (q.phi0), which
    does not depend on the initial guess."""
    s = oracle.setup(q)
    st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
    b0 = oracle.norm2_free(s["dir"], oracle.residual(st, s["dir"], q.phi0, s["f"]))
    return oracle.norm2_free(s["dir"], oracle.residual(st, s["dir"], phi, s["f"])) / b0


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_moving_conductor_time_steps(env, precision):
    torch, tomg, D = env
    n, tol = 129, 1e-10
    d = 1.0 / (n - 1)
    mp, amps, centres = D.geometry_params("circle", 5)
    p = tomg.Problem(n, n, d, d, precision=precision)
    phi = None
    eps = np.finfo(np.float64).eps
    for step, phase in enumerate((0.0, 0.04, 0.08, 0.12)):
        print(f"[moving] {precision} step {step} phase {phase}", flush=True)
        g = D.circle_geometry(n, mp["acoef"], "cuda", phase=phase)
        rho = D.gaussian_rho(g["xp"], g["yp"], amps, centres)
        p.setup_coeffs(rho, xp=g["xp"], yp=g["yp"], mask=g["mask"])
        if phi is None:
            phi = g["phi0"].clone()
        r = p.solve(phi, rel_tol=tol, max_cycles=100)
        assert r.ok, r
        cold = g["phi0"].clone()
        rc = p.solve(cold, rel_tol=tol, max_cycles=100)
        if step > 0:
            assert r.cycles < rc.cycles, (step, r.cycles, rc.cycles)
        ex, ey = p.field(phi, xp=g["xp"], yp=g["yp"])

        xp, yp = g["xp"].cpu().numpy(), g["yp"].cpu().numpy()
        q = w.GridProblem("moving", n, n, 0.0, 0.0, d, d, xp, yp, rho.cpu().numpy(),
                          g["phi0"].cpu().numpy(), mask=g["mask"].cpu().numpy())
        ph = phi.cpu().numpy()
        rel = _oracle_rel(q, ph)
        assert rel <= tol * (1 + 1e-3), (step, rel, r.rel)
        jac = oracle.jacobian_numeric(xp, yp, d, d)
        rx, ry = oracle.field(ph, jac, d, d)
        for gv, rv in ((ex.cpu().numpy(), rx), (ey.cpu().numpy(), ry)):
            scale = max(np.max(np.abs(rv)), np.max(np.abs(ph)))
            assert np.max(np.abs(gv - rv)) <= 16 * eps / d * scale

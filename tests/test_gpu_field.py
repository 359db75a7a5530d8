"""Field recovery on the GPU (tomg_field, eq. 2) against the oracle's
field of the same potential, element by element, and the recovered field of
a solved problem against the closed-form field.

Tolerance: both sides evaluate the same differences and the same 2x2
inverse; the one-sided edge differences cancel values of size max|phi| down
to h |grad phi|, so fused and separate multiply-adds may round apart by a few
eps max|phi| / h; 16 eps / h relative to max|E'| (and max|phi|) covers it."""

import math

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


def _tol(q, phi, e):
    eps = np.finfo(np.float64).eps
    return 16 * eps / min(q.dx, q.dy) * max(1.0, np.max(np.abs(phi)) / max(np.max(np.abs(e)),
                                                                            1e-300))


CASES = {
    "affine17": lambda: w.affine_map(17, [[1.3, 0.4], [-0.2, 0.9]], shift=(0.3, -0.1)),
    "sinusoidal129": lambda: w.manufactured_sinusoidal(129),
    "circle257": lambda: w.perturbed_circle(257),
    "annulus65x33": lambda: w.polar_semi_annulus(65, ny=33),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("numeric", [False, True])
def test_field_matches_oracle(tomg, name, numeric):
    import torch
    q = CASES[name]()
    if q.jac is None and not numeric:
        pytest.skip("numeric map only")
    print(f"[field] {name} numeric={numeric}", flush=True)
    rng = np.random.default_rng(3)
    phi = (q.phi_exact if q.phi_exact is not None
           else np.sin(3 * q.xp) * np.cos(2 * q.yp) + 0.01 * rng.standard_normal(q.xp.shape))
    p = tomg.Problem.from_grid(q)
    d = tomg.upload(q)
    ph = torch.as_tensor(phi).cuda()
    if numeric:
        ex, ey = p.field(ph, xp=d["xp"], yp=d["yp"])
        jac = oracle.jacobian_numeric(q.xp, q.yp, q.dx, q.dy)
    else:
        ex, ey = p.field(ph, jac=d["jac"])
        jac = q.jac
    rx, ry = oracle.field(phi, jac, q.dx, q.dy)
    ex, ey = ex.cpu().numpy(), ey.cpu().numpy()
    for g, r in ((ex, rx), (ey, ry)):
        err = np.max(np.abs(g - r)) / np.max(np.abs(r))
        assert err <= _tol(q, phi, r), err


def test_solved_annulus_field_is_second_order(tomg):
    errs = []
    for n in (65, 129):
        q = w.polar_semi_annulus(n)
        p, d = tomg.setup_from_grid(q)
        phi = d["phi0"].clone()
        assert p.solve(phi, rel_tol=1e-12, max_cycles=400).ok
        ex, ey = p.field(phi, jac=d["jac"])
        a, R = q.meta["a"], q.meta["R"]
        r = np.hypot(q.xp, q.yp)
        mag = 1.0 / (r * math.log(R / a))
        errs.append(max(np.max(np.abs(ex.cpu().numpy() - mag * q.xp / r)),
                        np.max(np.abs(ey.cpu().numpy() - mag * q.yp / r))))
    print(f"  field errors {errs}", flush=True)
    assert 3.0 <= errs[0] / errs[1] <= 5.0


def test_field_at_benchmark_size(tomg):
    import torch
    q = w.perturbed_circle(4097)
    p, d = tomg.setup_from_grid(q)
    phi = d["phi0"].clone()
    assert p.solve(phi, rel_tol=1e-10).ok
    ex, ey = p.field(phi, xp=d["xp"], yp=d["yp"])
    torch.cuda.synchronize()
    g = phi.cpu().numpy()
    rx, ry = oracle.field(g, oracle.jacobian_numeric(q.xp, q.yp, q.dx, q.dy), q.dx, q.dy)
    for a, r in ((ex.cpu().numpy(), rx), (ey.cpu().numpy(), ry)):
        assert np.max(np.abs(a - r)) / np.max(np.abs(r)) <= _tol(q, g, r)


def test_field_argument_errors(tomg):
    import torch
    q = w.manufactured_sinusoidal(17)
    p = tomg.Problem.from_grid(q)
    phi = torch.zeros((17, 17), dtype=torch.float64, device="cuda")
    with pytest.raises(tomg.TomgError):
        p.field(phi)  # no map

"""Pins of the oracle's coefficient setup (Section 2: eq. 1, 10-15, 11;
numeric Jacobian eq. 39-42) against closed forms and library routines."""

import math
import os

import numpy as np
import pytest

import oracle
import workloads as w

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_facts.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split("=")
            out[k.strip()] = float(v)
    return out


def eps_by_matrix_inverse(J):
    """eps = det J * J^-1 J^-T (eq. 10 with eps' = I) by numpy's 2x2 inverse,
    node by node; independent of the component formulas eq. 12-15."""
    M = np.moveaxis(J.reshape(2, 2, *J.shape[1:]), (0, 1), (-2, -1))
    Minv = np.linalg.inv(M)
    E = np.linalg.det(M)[..., None, None] * (Minv @ np.swapaxes(Minv, -1, -2))
    return E[..., 0, 0], E[..., 0, 1], E[..., 1, 0], E[..., 1, 1], np.linalg.det(M)


def test_identity_map_gives_identity_tensor():
    p = w.identity_map(17)
    exx, exy, eyy, det = oracle.permittivity(p.jac)
    assert np.array_equal(exx, np.ones_like(exx))
    assert np.array_equal(eyy, np.ones_like(eyy))
    assert np.array_equal(exy, np.zeros_like(exy))
    assert np.array_equal(det, np.ones_like(det))


@pytest.mark.parametrize("make", [
    lambda: w.manufactured_sinusoidal(33),
    lambda: w.polar_semi_annulus(33),
    lambda: w.sinh_stretch(33),
    lambda: w.affine_map(9, [[1.3, 0.4], [-0.2, 0.9]]),
])
def test_components_match_matrix_form(make):
    """eq. 12-15 against eq. 10 evaluated with a library matrix inverse."""
    p = make()
    exx, exy, eyy, det = oracle.permittivity(p.jac)
    rxx, rxy, ryx, ryy, rdet = eps_by_matrix_inverse(p.jac)
    for a, b in ((exx, rxx), (exy, rxy), (exy, ryx), (eyy, ryy), (det, rdet)):
        assert np.allclose(a, b, rtol=1e-13, atol=1e-13)


def test_polar_map_closed_form():
    """Polar map eq. 29: eps_xx = xi, eps_yy = 1/xi, eps_xy = 0 (the paper
    states the off-diagonals vanish), det J = xi."""
    g = golden()
    p = w.polar_semi_annulus(65, a=g["semi_annulus.a"], R=g["semi_annulus.R"])
    XI = p.xi0 + p.dx * np.arange(p.nx)[None, :] + 0 * p.xp
    exx, exy, eyy, det = oracle.permittivity(p.jac)
    assert np.allclose(exx, XI, rtol=1e-15, atol=0)
    assert np.allclose(eyy, 1.0 / XI, rtol=1e-15, atol=0)
    assert np.max(np.abs(exy)) <= 1e-15 * np.max(exx) + g["semi_annulus.eps_xy"]
    assert np.allclose(det, XI, rtol=1e-15)
    # paper's spacings for this problem
    assert p.dx == pytest.approx((g["semi_annulus.R"] - g["semi_annulus.a"]) / (p.nx - 1))
    assert p.dy == pytest.approx(math.pi / (p.ny - 1))


def test_sinh_map_closed_form():
    """Stretch eq. 52: eps_xx = cosh(a eta)/cosh(a xi), eps_yy its inverse,
    eps_xy = 0 (stated in Section 5.1), det = s^2 a^2 cosh cosh."""
    g = golden()
    s, al = g["sinh.s"], g["sinh.alpha"]
    p = w.sinh_stretch(int(g["sinh.n"]), s=s, alpha=al, L=g["sinh.L"])
    XI = p.xi0 + p.dx * np.arange(p.nx)[None, :] + 0 * p.xp
    ETA = p.eta0 + p.dy * np.arange(p.ny)[:, None] + 0 * p.xp
    exx, exy, eyy, det = oracle.permittivity(p.jac)
    assert np.allclose(exx, np.cosh(al * ETA) / np.cosh(al * XI), rtol=1e-14)
    assert np.allclose(eyy, np.cosh(al * XI) / np.cosh(al * ETA), rtol=1e-14)
    assert np.all(exy == g["sinh.eps_xy"])
    assert np.allclose(det, s * s * al * al * np.cosh(al * XI) * np.cosh(al * ETA), rtol=1e-14)


def test_sinusoidal_map_det_closed_form():
    """x' = xi + A s, y' = eta + A s: det J = 1 + A pi sin(pi (xi + eta))."""
    p = w.manufactured_sinusoidal(65, amp=0.1)
    XI = np.arange(p.nx)[None, :] * p.dx + 0 * p.xp
    ETA = np.arange(p.ny)[:, None] * p.dy + 0 * p.xp
    _, _, _, det = oracle.permittivity(p.jac)
    assert np.allclose(det, 1 + 0.1 * np.pi * np.sin(np.pi * (XI + ETA)), rtol=0, atol=2e-15)


@pytest.mark.parametrize("make", [lambda: w.manufactured_sinusoidal(65),
                                  lambda: w.perturbed_circle(257)])
def test_det_eps_is_one_and_spd(make):
    """In 2D with eps' = 1, det(eps) = det(J)^2 / det(J)^2 = 1 exactly, and
    eps is symmetric positive definite wherever det J > 0."""
    p = make()
    s = oracle.setup(p)
    d = s["exx"] * s["eyy"] - s["exy"] ** 2
    assert np.max(np.abs(d - 1.0)) <= 1e-13
    assert np.all(s["exx"] > 0) and np.all(s["eyy"] > 0)


def test_eps_phys_scales_tensor():
    p = w.manufactured_sinusoidal(17)
    e1 = oracle.permittivity(p.jac)
    sc = 1.0 + np.random.default_rng(3).uniform(size=p.xp.shape)
    e2 = oracle.permittivity(p.jac, sc)
    for a, b in zip(e1[:3], e2[:3]):
        assert np.allclose(a * sc, b, rtol=1e-15)


def test_numeric_jacobian_is_second_order():
    """eq. 39-42 (one-sided second order on the edges) converge to the
    analytic partials at rate 4 per halving of h."""
    errs = []
    for n in (33, 65, 129):
        p = w.manufactured_sinusoidal(n, amp=0.1)
        Jn = oracle.jacobian_numeric(p.xp, p.yp, p.dx, p.dy)
        errs.append(np.max(np.abs(Jn - p.jac)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


def test_numeric_jacobian_exact_on_quadratic_map():
    """Central and one-sided second-order differences are exact for a map
    that is quadratic in each coordinate."""
    n = 9
    d = 1.0 / (n - 1)
    XI, ETA = np.meshgrid(np.arange(n) * d, np.arange(n) * d)
    xp = XI + 0.3 * XI ** 2 + 0.1 * XI * ETA
    yp = ETA - 0.2 * ETA ** 2 + 0.25 * XI ** 2
    J = oracle.jacobian_numeric(xp, yp, d, d)
    assert np.allclose(J[0], 1 + 0.6 * XI + 0.1 * ETA, atol=1e-13)
    assert np.allclose(J[1], 0.1 * XI, atol=1e-13)
    assert np.allclose(J[2], 0.5 * XI, atol=1e-13)
    assert np.allclose(J[3], 1 - 0.4 * ETA, atol=1e-13)


def test_rhs_sign_and_charge_transform():
    """eq. 11 rho = rho' det J, and f = -rho (div(eps grad phi) = -rho)."""
    p = w.polar_semi_annulus(17)
    rho = np.random.default_rng(1).normal(size=p.xp.shape)
    _, _, _, det = oracle.permittivity(p.jac)
    f = oracle.rhs(rho, det)
    assert np.array_equal(f, -(rho * det))


def test_geometry_check():
    """A folded map (det J < 0 somewhere) is rejected; the square-to-disc map,
    whose det J vanishes only at the four corners, is accepted."""
    p = w.square_to_disc(33, 1.0, "harmonic8")
    s = oracle.setup(p)
    corners = [s["det"][0, 0], s["det"][0, -1], s["det"][-1, 0], s["det"][-1, -1]]
    assert max(abs(c) for c in corners) < 1e-15
    assert s["geometry_ok"]
    q = w.manufactured_sinusoidal(33, amp=0.5)  # 0.5 pi > 1 folds the map
    assert not oracle.setup(q)["geometry_ok"]


def test_disc_domain_reading():
    """Section 4.2.1 prints dx = 0.015625 for N = 257 and b = 2, which fixes
    the computational square as [-b, b]^2."""
    g = golden()
    p = w.square_to_disc(int(g["disc.n"]), g["disc.b"], "source")
    assert p.dx == g["disc.dx"]
    ring = np.zeros(p.xp.shape, bool)
    ring[0, :] = ring[-1, :] = ring[:, 0] = ring[:, -1] = True
    # eq. 44 puts the square's sides on the circle of radius b
    assert np.allclose(np.hypot(p.xp, p.yp)[ring], g["disc.b"], atol=1e-14)
    assert np.allclose(p.phi0[ring], g["disc.boundary_phi"], atol=1e-14)


def test_error_norms_by_hand():
    a = np.array([[0.0, 1.0], [2.0, 3.0]])
    b = np.array([[0.5, 1.0], [1.0, 3.0]])
    linf, l2, l1 = oracle.error_norms(a, b)
    assert linf == 1.0
    assert l2 == pytest.approx(math.sqrt((0.25 + 1.0) / 4))
    assert l1 == pytest.approx(1.5 / 4)

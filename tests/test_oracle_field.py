"""Pins of the oracle's field recovery E' = (J^T)^-1 (-grad phi) (eq. 2):
exactness where the differences are exact (quadratic potentials under affine
maps, including a non-symmetric Jacobian, which tells J^-T from J^-1), and
second-order convergence to the closed-form field of the semi-annulus
(eq. 28-a under the polar map eq. 29)."""

import math

import numpy as np

import oracle
import workloads as w


def test_affine_map_quadratic_potential_is_exact():
    M = np.array([[1.3, 0.4], [-0.2, 0.9]])  # J != J^T
    q = w.affine_map(17, M, shift=(0.3, -0.1))
    x, y = q.xp, q.yp
    phi = x ** 2 - 2 * x * y + 0.5 * y + 3.0
    ex, ey = oracle.field(phi, q.jac, q.dx, q.dy)
    assert np.max(np.abs(ex + (2 * x - 2 * y))) <= 1e-12
    assert np.max(np.abs(ey + (-2 * x + 0.5))) <= 1e-12
    # the transposed inverse matters: J^-1 instead of J^-T is far off
    e1 = -np.gradient(phi, q.dx, axis=1)
    e2 = -np.gradient(phi, q.dy, axis=0)
    Minv = np.linalg.inv(M)
    wrong_x = Minv[0, 0] * e1 + Minv[0, 1] * e2
    assert np.max(np.abs(wrong_x - ex)) > 0.1


def test_identity_map_is_minus_central_gradient():
    q = w.identity_map(9)
    phi = 2 * q.xp ** 2 + q.xp * q.yp - q.yp ** 2
    ex, ey = oracle.field(phi, q.jac, q.dx, q.dy)
    assert np.allclose(ex, -(4 * q.xp + q.yp), atol=1e-13)
    assert np.allclose(ey, -(q.xp - 2 * q.yp), atol=1e-13)


def _annulus_field_error(n):
    q = w.polar_semi_annulus(n)
    a, R = q.meta["a"], q.meta["R"]
    r = np.hypot(q.xp, q.yp)
    ex, ey = oracle.field(q.phi_exact, q.jac, q.dx, q.dy)
    mag = 1.0 / (r * math.log(R / a))  # E' = -grad phi points outwards
    return max(np.max(np.abs(ex - mag * q.xp / r)), np.max(np.abs(ey - mag * q.yp / r)))


def test_semi_annulus_field_is_second_order():
    e1, e2, e3 = (_annulus_field_error(n) for n in (33, 65, 129))
    assert 3.5 <= e1 / e2 <= 4.5 and 3.5 <= e2 / e3 <= 4.5
    assert e3 < 1e-4

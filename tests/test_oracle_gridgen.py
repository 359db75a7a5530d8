"""Pins of the oracle's numerical grid generation (Section 4.2: x' and y'
solve Laplace's equation on the computational grid, eq. 36-37, with the
boundary map of eq. 44 as Dirichlet data) and of the paper's circular-domain
results computed on the generated grids (eq. 43 and eq. 45)."""

import numpy as np

import oracle
import workloads as w


def test_harmonic_quadratic_boundary_gives_the_quadratic_inside():
    # x' = x + 0.1 (x^2 - y^2), y' = y + 0.2 x y are harmonic; the 5-point
    # Laplacian is exact on quadratics, so the discrete solution is the map
    n = 33
    q = w.identity_map(n)
    x, y = q.xp, q.yp
    xt, yt = x + 0.1 * (x ** 2 - y ** 2), y + 0.2 * x * y
    xb, yb = xt.copy(), yt.copy()
    xb[1:-1, 1:-1] = yb[1:-1, 1:-1] = 0.0
    xp, yp = oracle.generate_grid(xb, yb, q.dx, q.dy)
    assert np.max(np.abs(xp - xt)) <= 1e-12 and np.max(np.abs(yp - yt)) <= 1e-12


def _disc_grid(n, b):
    xb, yb = w.disc_boundary(n, b)
    d = 2.0 * b / (n - 1)
    return xb, yb, oracle.generate_grid(xb, yb, d, d)


def test_disc_grid_boundary_symmetry_and_orientation():
    b, n = 2.0, 33
    xb, yb, (xp, yp) = _disc_grid(n, b)
    ring = np.zeros((n, n), bool)
    ring[0] = ring[-1] = ring[:, 0] = ring[:, -1] = True
    assert np.array_equal(xp[ring], xb[ring]) and np.array_equal(yp[ring], yb[ring])
    # eq. 44 on the bottom side: x' = xi / sqrt 2, y' = -b sqrt(1 - xi^2 / (2 b^2))
    xi = np.linspace(-b, b, n)
    assert np.allclose(xb[0], xi / np.sqrt(2)) and np.allclose(yb[0], -b * np.sqrt(1 - xi ** 2 / (2 * b * b)))
    # the map commutes with the swap of the axes: x'(xi, eta) = y'(eta, xi)
    assert np.max(np.abs(xp - yp.T)) <= 1e-12
    # boundary nodes lie on the circle of radius b
    assert np.allclose(np.hypot(xb[ring], yb[ring]), b)
    # a valid, orientation-preserving map away from the four corners
    J = oracle.jacobian_numeric(xp, yp, 2 * b / (n - 1), 2 * b / (n - 1))
    det = J[0] * J[3] - J[1] * J[2]
    corner = np.zeros((n, n), bool)
    corner[0, 0] = corner[0, -1] = corner[-1, 0] = corner[-1, -1] = True
    assert det[~corner].min() > 0


def _solve_on_generated(n, b, kind):
    _, _, (xp, yp) = _disc_grid(n, b)
    q = w.disc_on_grid(xp, yp, b, kind)
    r = oracle.solve_problem(q, rel_tol=1e-12)
    assert r["status"] == 0
    return oracle.error_norms(r["phi"], q.phi_exact)


def test_disc_with_source_on_generated_grid_is_second_order():
    # eq. 43, b = 2 (Section 4.2.1): second order in the global norms; the
    # maximum norm converges more slowly because the map degenerates at the
    # four corners of the square
    e = [_solve_on_generated(n, 2.0, "source") for n in (33, 65, 129)]
    for k in (1, 2):  # L2, L1
        assert 3.5 <= e[0][k] / e[1][k] <= 4.5 and 3.5 <= e[1][k] / e[2][k] <= 4.5
    assert e[0][0] / e[1][0] > 2.5 and e[1][0] / e[2][0] > 2.5


def test_harmonic_on_unit_disc_generated_grid_is_second_order():
    # eq. 45 with n = 8, b = 1 (Section 4.2.2)
    e = [_solve_on_generated(n, 1.0, "harmonic8") for n in (33, 65, 129)]
    assert 3.5 <= e[0][0] / e[1][0] <= 4.5 and 3.5 <= e[1][0] / e[2][0] <= 4.5


def test_sources_give_the_quadratic_map():
    """Grid generation with source terms (the conclusion's adaptive grids):
    x' = xi + a (xi^2 + eta^2) / 4 has lap x' = a, y' = eta + c eta^2 has
    lap y' = 2c; the 5-point Laplacian is exact on quadratics, so with these
    constant sources and the map's boundary values the generated grid is
    the map itself (a wrong sign or a missing h^2 scaling of the source
    breaks this)."""
    n = 33
    q = w.identity_map(n)
    x, y = q.xp, q.yp
    a, c = 0.4, -0.3
    xt, yt = x + a * (x ** 2 + y ** 2) / 4.0, y + c * y ** 2
    xb, yb = xt.copy(), yt.copy()
    xb[1:-1, 1:-1] = yb[1:-1, 1:-1] = 0.0
    px, py = np.full((n, n), a), np.full((n, n), 2.0 * c)
    xp, yp = oracle.generate_grid(xb, yb, q.dx, q.dy, px=px, py=py)
    assert np.max(np.abs(xp - xt)) <= 1e-12 and np.max(np.abs(yp - yt)) <= 1e-12
    # without the sources the interior differs
    x0, _ = oracle.generate_grid(xb, yb, q.dx, q.dy)
    assert np.max(np.abs(x0 - xt)) > 1e-3


def test_source_clusters_nodes():
    """An adaptive grid of the conclusion: along a line x'' = P, so the
    spacing of x' falls where P < 0 and grows where P > 0; a source that
    changes sign from negative to positive across xi = 0.5 clusters the
    nodes there (and the opposite sign spreads them)."""
    n = 65
    q = w.identity_map(n)
    x, y = q.xp, q.yp
    xb, yb = x.copy(), y.copy()
    xb[1:-1, 1:-1] = yb[1:-1, 1:-1] = 0.0
    band = (x - 0.5) * np.exp(-((x - 0.5) / 0.1) ** 2)
    mid = n // 2
    for k, closer in ((40.0, True), (-40.0, False)):
        xp, yp = oracle.generate_grid(xb, yb, q.dx, q.dy, px=k * band)
        dx_mid = xp[mid, mid + 1] - xp[mid, mid]
        dx_far = xp[mid, 9] - xp[mid, 8]
        assert (dx_mid < 0.9 * dx_far) if closer else (dx_mid > 1.1 * dx_far)
        assert np.all(np.diff(xp[mid]) > 0)  # still a valid (monotone) grid line
        assert np.max(np.abs(yp - y)) <= 1e-12

"""Pins of the oracle's symmetric flux (energy) form of the operator, the
alternative discretisation to the expanded eq. 18.

The operator is minus the gradient of a discrete energy (face means of
eps_xx and eps_yy times squared face differences; cell means of eps_xy times
the product of cell-centred differences).  The pins: its matrix is
symmetric and negative definite; it is the 5-point Laplacian for eps = I and
eq. 18 itself for any constant eps; it converges at second order on the
manufactured problem; with a Neumann edge it is the half of the
mirror-doubled Dirichlet problem, as the eq. 18 form is."""

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import direct
import workloads as w


def _stencils(q, neumann=0):
    s = oracle.setup(q)
    dirs = oracle.dirichlet_set(q.nx, q.ny, q.mask, neumann)
    fl = oracle.flux_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, dirs)
    ex = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, dirs)
    return fl, ex, dirs, s


@pytest.mark.parametrize("name", ["circle", "sinusoidal", "annulus_neumann"])
def test_symmetric_and_negative_definite(name):
    q = {"circle": lambda: w.perturbed_circle(33, seed=1),
         "sinusoidal": lambda: w.manufactured_sinusoidal(17, amp=0.15),
         "annulus_neumann": lambda: w.polar_semi_annulus(17, neumann=True)}[name]()
    fl, ex, dirs, _ = _stencils(q, q.neumann)
    A = direct.split(fl, dirs)[0].toarray()
    # a Neumann edge row carries its folded ghost coefficient twice, so the
    # matrix is symmetric once its rows are weighted by the node's share of
    # a cell: 1/2 on a Neumann edge (1/4 at a corner of two)
    wgt = np.ones((q.ny, q.nx))
    wgt[0, :] *= 0.5 if q.neumann & oracle.NEU_S else 1.0
    wgt[-1, :] *= 0.5 if q.neumann & oracle.NEU_N else 1.0
    wgt[:, 0] *= 0.5 if q.neumann & oracle.NEU_W else 1.0
    wgt[:, -1] *= 0.5 if q.neumann & oracle.NEU_E else 1.0
    A = wgt.ravel()[dirs.ravel() == 0][:, None] * A
    assert np.max(np.abs(A - A.T)) <= 1e-13 * np.max(np.abs(A))
    sla.cholesky(-A)  # raises unless -A is positive definite
    if name == "circle":  # the expanded form is not symmetric there
        E = direct.split(ex, dirs)[0].toarray()
        assert np.max(np.abs(E - E.T)) > 1e-6 * np.max(np.abs(E))


def test_identity_map_is_5_point_laplacian():
    q = w.identity_map(17)
    fl, _, dirs, _ = _stencils(q)
    A = direct.split(fl, dirs)[0]
    assert abs(A - direct.five_point_laplacian(17, q.dx)).max() <= 1e-12 / q.dx ** 2


def test_constant_tensor_equals_eq18():
    q = w.affine_map(17, [[1.3, 0.45], [-0.2, 0.9]])
    fl, ex, dirs, _ = _stencils(q)
    free = dirs == 0
    for k in range(9):
        assert np.allclose(fl[k][free], ex[k][free], rtol=1e-13, atol=1e-13 * np.abs(ex[4]).max())


def test_second_order_on_manufactured_solution():
    errs = []
    for n in (17, 33, 65, 129):
        q = w.manufactured_sinusoidal(n)
        r = oracle.solve_problem(q, rel_tol=1e-13, max_cycles=200, flux=True)
        assert r["status"] == 0
        errs.append(np.max(np.abs(r["phi"] - q.phi_exact)))
    ratios = [errs[k] / errs[k + 1] for k in range(3)]
    assert all(3.6 < x < 4.4 for x in ratios[1:]), (errs, ratios)


def test_mirror_extension_with_flux_form():
    n, d = 17, 1.0 / 16
    ys = (np.arange(2 * n - 1) - (n - 1)) * d
    X2, Y2 = np.meshgrid(np.arange(n) * d + 0.3, ys)
    exx = 1.0 + 0.3 * np.cos(np.pi * X2) * np.cos(np.pi * Y2)
    eyy = 1.2 + 0.2 * np.cos(0.5 * np.pi * X2) * np.cos(np.pi * Y2)
    exy = 0.2 * np.sin(np.pi * X2) * np.sin(np.pi * Y2)
    f = np.exp(-((X2 - 0.6) ** 2 + (np.abs(Y2) - 0.4) ** 2) / 0.05)
    g = np.cos(X2) + Y2 * Y2
    dirs2 = oracle.dirichlet_set(n, 2 * n - 1)
    st2 = oracle.flux_stencil(exx, exy, eyy, d, d, dirs2)
    full = direct.direct_solve(st2, dirs2, f, np.where(dirs2 == 1, g, 0.0))
    h = [np.ascontiguousarray(a[n - 1:]) for a in (exx, exy, eyy, f, g)]
    dirs = oracle.dirichlet_set(n, n, None, oracle.NEU_S)
    st = oracle.flux_stencil(h[0], h[1], h[2], d, d, dirs)
    half = direct.direct_solve(st, dirs, h[3], np.where(dirs == 1, h[4], 0.0))
    assert np.max(np.abs(half - full[n - 1:])) <= 1e-12 * np.max(np.abs(full))


def test_flux_multigrid_reaches_direct_solution():
    q = w.perturbed_circle(65, seed=3)
    fl, _, dirs, s = _stencils(q)
    ref = direct.direct_solve(fl, dirs, s["f"], np.where(dirs == 1, q.phi0, 0.0))
    r = oracle.solve_problem(q, rel_tol=1e-13, max_cycles=100, flux=True)
    assert r["status"] == 0 and r["cycles"] < 20
    assert np.max(np.abs(r["phi"] - ref)) <= 1e-9 * np.max(np.abs(ref))

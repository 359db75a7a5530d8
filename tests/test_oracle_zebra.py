"""Pins of the oracle's zebra x-line Gauss-Seidel smoother (an extension for
anisotropic grids, the other half of the Neumann/anisotropy row).

One sweep relaxes the even rows, each solved exactly with its neighbours
held, then the odd rows.  The pins: the sweep equals a block Gauss-Seidel
written here with SciPy's banded solver per row; after a sweep the
equations of the odd rows hold exactly; the multigrid cycle with this
smoother contracts the anisotropic semi-annulus error much faster than the
point smoother (the reason it exists)."""

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import workloads as w


def _problem(name):
    if name == "annulus_neumann":
        return w.polar_semi_annulus(33, neumann=True)
    if name == "circle":
        return w.perturbed_circle(33, seed=4)
    return w.manufactured_sinusoidal(17, ny=9)


@pytest.mark.parametrize("name", ["annulus_neumann", "circle", "sinusoidal17x9"])
def test_zebra_sweep_is_row_block_gauss_seidel(name):
    q = _problem(name)
    s = oracle.setup(q)
    st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
    rng = np.random.default_rng(3)
    x0 = np.where(s["dir"] == 1, q.phi0, rng.normal(size=q.phi0.shape))
    got = oracle.smooth(st, s["dir"], x0, s["f"], kind=oracle.ZEBRA_X, sweeps=1)
    # reference: rows in the order 0, 2, 4, ..., 1, 3, ...; each row solved
    # with scipy.linalg.solve_banded, the other rows held at current values
    x = x0.copy()
    ny, nx = x.shape
    P = {(di, dj): st[(dj + 1) * 3 + (di + 1)] for dj in (-1, 0, 1) for di in (-1, 0, 1)}
    for j in list(range(0, ny, 2)) + list(range(1, ny, 2)):
        ab = np.zeros((3, nx))
        rhs = np.zeros(nx)
        for i in range(nx):
            if s["dir"][j, i]:
                ab[1, i] = 1.0
                rhs[i] = x[j, i]
                continue
            ab[1, i] = P[(0, 0)][j, i]
            if i > 0:
                ab[2, i - 1] = P[(-1, 0)][j, i]
            if i < nx - 1:
                ab[0, i + 1] = P[(1, 0)][j, i]
            r = s["f"][j, i]
            for dj in (-1, 1):
                for di in (-1, 0, 1):
                    if 0 <= j + dj < ny and 0 <= i + di < nx:
                        r -= P[(di, dj)][j, i] * x[j + dj, i + di]
            rhs[i] = r
        x[j] = sla.solve_banded((1, 1), ab, rhs)
    assert np.max(np.abs(got - x)) <= 1e-12 * max(1.0, np.max(np.abs(x)))


def test_odd_rows_exact_after_sweep():
    q = _problem("annulus_neumann")
    s = oracle.setup(q)
    st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
    x0 = np.where(s["dir"] == 1, q.phi0, 0.3)
    x1 = oracle.smooth(st, s["dir"], x0, s["f"], kind=oracle.ZEBRA_X, sweeps=1)
    r = oracle.residual(st, s["dir"], x1, s["f"])
    scale = np.max(np.abs(st[4])) * max(1.0, np.max(np.abs(x1)))
    assert np.max(np.abs(r[1::2])) <= 1e-12 * scale
    assert np.max(np.abs(r[0::2])) > 1e-6 * scale  # the even rows moved on since


def test_zebra_multigrid_beats_point_smoother_on_anisotropic_grid():
    """On the semi-annulus the coupling along xi is 4-27 times the coupling
    along eta; x-line relaxation smooths such errors, so its V(2,2) rate is
    a fraction of the point smoother's."""
    q = w.polar_semi_annulus(129, neumann=True)
    rz = oracle.solve_problem(q, rel_tol=1e-10, max_cycles=200, smoother=oracle.ZEBRA_X,
                              hist_len=40)
    rp = oracle.solve_problem(q, rel_tol=1e-10, max_cycles=200, hist_len=40)
    assert rz["status"] == 0 and rp["status"] == 0
    assert rz["cycles"] <= rp["cycles"] // 2, (rz["cycles"], rp["cycles"])
    assert np.max(np.abs(rz["phi"] - rp["phi"])) <= 1e-8 * np.max(np.abs(rp["phi"]))


@pytest.mark.parametrize("name", ["annulus_neumann", "circle", "sinusoidal17x9"])
def test_zebra_y_half_sweep_is_column_block_gauss_seidel(name):
    """An alternating sweep is an x-line sweep followed by a y-line sweep;
    the y-line part equals column-block Gauss-Seidel (even columns, then
    odd ones) with SciPy's banded solver per column."""
    q = _problem(name)
    s = oracle.setup(q)
    st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
    rng = np.random.default_rng(8)
    x0 = np.where(s["dir"] == 1, q.phi0, rng.normal(size=q.phi0.shape))
    xh = oracle.smooth(st, s["dir"], x0, s["f"], kind=oracle.ZEBRA_X, sweeps=1)
    got = oracle.smooth(st, s["dir"], x0, s["f"], kind=oracle.ZEBRA_XY, sweeps=1)
    x = xh.copy()
    ny, nx = x.shape
    P = {(di, dj): st[(dj + 1) * 3 + (di + 1)] for dj in (-1, 0, 1) for di in (-1, 0, 1)}
    for i in list(range(0, nx, 2)) + list(range(1, nx, 2)):
        ab = np.zeros((3, ny))
        rhs = np.zeros(ny)
        for j in range(ny):
            if s["dir"][j, i]:
                ab[1, j] = 1.0
                rhs[j] = x[j, i]
                continue
            ab[1, j] = P[(0, 0)][j, i]
            if j > 0:
                ab[2, j - 1] = P[(0, -1)][j, i]
            if j < ny - 1:
                ab[0, j + 1] = P[(0, 1)][j, i]
            r = s["f"][j, i]
            for di in (-1, 1):
                for dj in (-1, 0, 1):
                    if 0 <= j + dj < ny and 0 <= i + di < nx:
                        r -= P[(di, dj)][j, i] * x[j + dj, i + di]
            rhs[j] = r
        x[:, i] = sla.solve_banded((1, 1), ab, rhs)
    assert np.max(np.abs(got - x)) <= 1e-12 * max(1.0, np.max(np.abs(x)))


def test_alternating_zebra_on_the_sinh_stretch():
    """The sinh-stretched grid of Section 5.1 is anisotropic in both
    directions (varying with position): x-lines alone do not help, the
    alternating x/y sweep does."""
    q = w.sinh_stretch(129)
    rp = oracle.solve_problem(q, rel_tol=1e-10, max_cycles=200)
    rx = oracle.solve_problem(q, rel_tol=1e-10, max_cycles=200, smoother=oracle.ZEBRA_X)
    rxy = oracle.solve_problem(q, rel_tol=1e-10, max_cycles=200, smoother=oracle.ZEBRA_XY)
    assert rxy["cycles"] <= rp["cycles"] // 2 and rx["cycles"] > rp["cycles"] // 2
    assert np.max(np.abs(rxy["phi"] - rp["phi"])) <= 1e-8 * np.max(np.abs(rp["phi"]))

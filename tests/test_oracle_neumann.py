"""Pins of the oracle's Neumann edges (Section 4.1: a zero normal derivative
on the two straight sides of the semi-annulus).

A free node on the outer ring takes eq. 18 with a mirror ghost layer (the
tensor mirrored, eps_xy with its sign changed; phi mirrored) folded onto the
mirror nodes.  The pins: the closed-form semi-annulus solution is reached at
second order; the discrete Neumann problem equals, exactly, the half of a
doubled all-Dirichlet problem whose data are mirror-symmetric (one edge, and
a corner of two Neumann edges); the Galerkin product and the restriction at
free ring nodes match SciPy's (1/4) P^T A P and P^T; a GS4 sweep leaves zero
residual on its last colour, edge nodes included; the multigrid solution is
SciPy's sparse direct solution."""

import numpy as np
import pytest

import oracle
from oracle import direct
import workloads as w

S, N, W, E = oracle.NEU_S, oracle.NEU_N, oracle.NEU_W, oracle.NEU_E


def test_semi_annulus_neumann_second_order():
    """The paper's setting: Dirichlet arcs, Neumann straight sides; the error
    against ln(R/r)/ln(R/a) falls by 4 per halving of h and matches that of
    the all-Dirichlet version."""
    errs, errs_d = [], []
    for n in (33, 65, 129):
        q = w.polar_semi_annulus(n, neumann=True)
        assert q.neumann == S | N
        r = oracle.solve_problem(q, rel_tol=1e-12, max_cycles=300)
        assert r["status"] == 0
        errs.append(np.max(np.abs(r["phi"] - q.phi_exact)))
        qd = w.polar_semi_annulus(n)
        rd = oracle.solve_problem(qd, rel_tol=1e-12, max_cycles=300)
        errs_d.append(np.max(np.abs(rd["phi"] - qd.phi_exact)))
    assert 3.8 < errs[0] / errs[1] < 4.2 and 3.8 < errs[1] / errs[2] < 4.2, errs
    for a, b in zip(errs, errs_d):
        assert abs(a - b) <= 0.05 * b


def _tensor(X, Y):
    """SPD tensor even in x and y for eps_xx, eps_yy and odd in each for
    eps_xy, so that it is mirror-symmetric across x = 0 and y = 0."""
    exx = 1.0 + 0.3 * np.cos(np.pi * X) * np.cos(np.pi * Y)
    eyy = 1.2 + 0.2 * np.cos(0.5 * np.pi * X) * np.cos(np.pi * Y)
    exy = 0.2 * np.sin(np.pi * X) * np.sin(np.pi * Y)
    return exx, exy, eyy


def _data(X, Y):
    f = np.exp(-((np.abs(X) - 0.6) ** 2 + (np.abs(Y) - 0.4) ** 2) / 0.05)
    g = np.cos(X) + Y * Y
    return f, g


def _solve_direct(exx, exy, eyy, d, dirs, f, g):
    st = oracle.fine_stencil(exx, exy, eyy, d, d, dirs)
    phi_dir = np.where(dirs == 1, g, 0.0)
    return direct.direct_solve(st, dirs, f, phi_dir)


@pytest.mark.parametrize("case", ["edge", "corner"])
def test_mirror_extension_equals_doubled_dirichlet(case):
    """Neumann on y = 0 (edge) or on x = 0 and y = 0 (corner): the discrete
    solution equals the solution of the mirror-doubled problem with
    Dirichlet data all round, restricted to the original half (quarter)."""
    n, d = 17, 1.0 / 16
    # doubled grid: y (and x for the corner) over [-1, 1]
    xs = np.arange(n) * d if case == "edge" else (np.arange(2 * n - 1) - (n - 1)) * d
    ys = (np.arange(2 * n - 1) - (n - 1)) * d
    X2, Y2 = np.meshgrid(xs + (0.3 if case == "edge" else 0.0), ys)
    exx, exy, eyy = _tensor(X2, Y2)
    f, g = _data(X2, Y2)
    dirs2 = oracle.dirichlet_set(X2.shape[1], X2.shape[0])
    full = _solve_direct(exx, exy, eyy, d, dirs2, f, g)
    # the half (quarter) with the mirror line(s) as Neumann edges
    sl = (slice(n - 1, None), slice(None)) if case == "edge" else (slice(n - 1, None),
                                                                   slice(n - 1, None))
    neu = S if case == "edge" else S | W
    h = [np.ascontiguousarray(a[sl]) for a in (exx, exy, eyy, f, g)]
    ny, nx = h[0].shape
    dirs = oracle.dirichlet_set(nx, ny, None, neu)
    assert dirs[0, 1:-1].sum() == 0 and dirs[1:-1, 0].sum() == (0 if case == "corner" else ny - 2)
    half = _solve_direct(h[0], h[1], h[2], d, dirs, h[3], h[4])
    ref = full[sl]
    assert np.max(np.abs(half - ref)) <= 1e-12 * np.max(np.abs(ref))
    # and the oracle's multigrid reaches the same discrete solution
    mg = oracle.MG(h[0], h[1], h[2], d, d, neumann=neu)
    phi, st, _, rel, _ = mg.solve(np.where(dirs == 1, h[4], 0.0), h[3], 1e-13, 200)
    assert st == 0
    assert np.max(np.abs(phi - ref)) <= 1e-10 * np.max(np.abs(ref))


def _neumann_problem(n=33, neu=S | E):
    q = w.perturbed_circle(n, seed=2)
    q.neumann = neu
    return q


def test_galerkin_with_neumann_edges_matches_scipy():
    """(1/4) P^T A P with P restricted to the unknowns; the coarse ring keeps
    free nodes where the fine node under it is free."""
    q = _neumann_problem()
    s = oracle.setup(q)
    st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
    stc, dirc = oracle.galerkin(st, s["dir"], 17, 17)
    # ring kinds: S and E edges free except at corners with Dirichlet edges
    assert dirc[0, 1:-1].sum() == 0 and dirc[1:-1, -1].sum() == 0
    assert dirc[-1].all() and dirc[:, 0].all()
    assert dirc[0, -1] == 0  # S-E corner: both edges Neumann
    A = direct.assemble_full(st).tolil()
    df = s["dir"].ravel().astype(bool)
    dc = dirc.ravel().astype(bool)
    A[np.flatnonzero(df), :] = 0
    Pm = direct.bilinear_P(17, 17, 33, 33).tolil()
    Pm[np.flatnonzero(df), :] = 0
    Pm[:, np.flatnonzero(dc)] = 0
    Pm = Pm.tocsr()
    Ac = (0.25 * (Pm.T @ A.tocsr() @ Pm)).toarray()
    Cs = direct.assemble_full(stc).toarray()
    free = np.flatnonzero(~dc)
    sub = np.ix_(free, free)
    assert np.allclose(Cs[sub], Ac[sub], rtol=1e-13, atol=1e-13 * abs(Ac).max())


def test_restriction_bc_is_quarter_transpose():
    rng = np.random.default_rng(4)
    q = _neumann_problem()
    s = oracle.setup(q)
    st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
    _, dirc = oracle.galerkin(st, s["dir"], 17, 17)
    r = rng.normal(size=(33, 33)) * (s["dir"] == 0)
    e = rng.normal(size=(17, 17)) * (dirc == 0)
    Rr = oracle.restrict_fw_bc(r, dirc)
    Pe = direct.bilinear_P(17, 17, 33, 33) @ e.ravel()
    assert np.sum(Rr * e) == pytest.approx(0.25 * np.sum(r.ravel() * Pe), rel=1e-13)
    ring_dir = np.zeros_like(dirc, bool)
    ring_dir[0, :] = ring_dir[-1, :] = ring_dir[:, 0] = ring_dir[:, -1] = True
    assert np.all(Rr[ring_dir & (dirc == 1)] == 0.0)


def test_gs4_sweep_solves_last_colour_on_edges():
    """After one four-colour sweep the equations of the last colour (odd i,
    odd j) hold exactly -- and so do those of every colour on a Neumann edge
    node as it is relaxed; checked at the last colour, edge nodes included."""
    q = _neumann_problem(33, S | N | E)
    s = oracle.setup(q)
    st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
    rng = np.random.default_rng(9)
    x = rng.normal(size=(33, 33))
    x = np.where(s["dir"] == 1, q.phi0, x)
    x1 = oracle.smooth(st, s["dir"], x, s["f"], oracle.GS4, 1)
    r = oracle.residual(st, s["dir"], x1, s["f"])
    J, I = np.mgrid[0:33, 0:33]
    last = (I % 2 == 1) & (J % 2 == 1) & (s["dir"] == 0)
    assert np.max(np.abs(r[last])) <= 1e-12 * np.max(np.abs(s["f"]))
    # the last colour has no node on the even-indexed edges; the first colour
    # (even, even) does, and its residual is nonzero after later colours
    edge0 = (J == 0) & (I % 2 == 0) & (s["dir"] == 0)
    assert edge0.sum() > 0 and np.max(np.abs(r[edge0])) > 0


@pytest.mark.parametrize("neu", [S | N, S | E, W | E | S])
def test_neumann_multigrid_reaches_direct_solution(neu):
    q = _neumann_problem(65, neu)
    s = oracle.setup(q)
    st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
    ref = direct.direct_solve(st, s["dir"], s["f"], np.where(s["dir"] == 1, q.phi0, 0.0))
    r = oracle.solve_problem(q, rel_tol=1e-13, max_cycles=200, hist_len=30)
    assert r["status"] == 0
    assert np.max(np.abs(r["phi"] - ref)) <= 1e-9 * np.max(np.abs(ref))
    h = r["hist"]
    # the coarse-grid correction works at the free edges: a multigrid rate
    assert max(h[k + 1] / h[k] for k in range(3, 8)) < 0.35

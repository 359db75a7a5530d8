"""Pins of the oracle's semi-coarsening: the transfers and the Galerkin
coarse operator with one axis halved and the other kept (an extension of
the V-cycle of Section 3, eq. 19-24, which halves both axes).

The pins: the coarse stencil of a constant anisotropic operator in closed
form; the stencil-form product against SciPy's (1/(sx sy)) P^T A P with P
built as a Kronecker product; the restriction and prolongation against the
same matrix; and the multigrid: on the semi-annulus of Section 4.1, whose
coupling along the radius (the x axis) is 4 to 27 times the one along the
angle, halving x only converges at a rate independent of the grid and to
the direct solution of the discrete problem."""

import numpy as np
import pytest

import oracle
from oracle import direct
import workloads as w


def _const_stencil(n, a, b, dx, dy, neumann=0):
    exx = np.full((n, n), a)
    eyy = np.full((n, n), b)
    exy = np.zeros((n, n))
    dirs = oracle.dirichlet_set(n, n, None, neumann)
    return oracle.fine_stencil(exx, exy, eyy, dx, dy, dirs), dirs


@pytest.mark.parametrize("axis", [0, 1])
def test_semi_galerkin_closed_form(axis):
    """A = a d_xx + b d_yy (eq. 18 with a constant diagonal tensor).  Halving
    x with linear P and R = P^T / 2 gives, away from the boundary, the
    coarse x operator a [1, -2, 1] / (2 dx)^2 and the y operator
    b [1, -2, 1] / dy^2 spread over x by (1/2) P^T P = [1/8, 3/4, 1/8];
    halving y is the same with the axes exchanged."""
    n, a, b, dx, dy = 33, 1.7, 0.3, 0.05, 0.08
    st, dirs = _const_stencil(n, a, b, dx, dy)
    assert st[4, 5, 5] == pytest.approx(-2 * a / dx**2 - 2 * b / dy**2, rel=1e-14)
    sx, sy = (2, 1) if axis == 0 else (1, 2)
    stc, dirc = oracle.galerkin_s(st, dirs, sx, sy)
    if axis == 0:
        assert stc.shape == (9, n, 17)
        H, h, strong, kept = 2 * dx, dy, a, b
    else:
        assert stc.shape == (9, 17, n)
        H, h, strong, kept = 2 * dy, dx, b, a
    m = np.array([0.125, 0.75, 0.125])      # (1/2) P^T P along the halved axis
    t = np.array([1.0, -2.0, 1.0])
    ref = np.zeros((3, 3))                  # ref[halved offset, kept offset]
    ref[:, 1] += strong / H**2 * t
    ref += kept / h**2 * np.outer(m, t)
    for k in range(9):
        dj, di = k // 3 - 1, k % 3 - 1
        want = ref[di + 1, dj + 1] if axis == 0 else ref[dj + 1, di + 1]
        inner = stc[k, 2:-2, 2:-2]
        assert np.allclose(inner, want, rtol=1e-13, atol=1e-12 * abs(ref).max()), k


@pytest.mark.parametrize("sx,sy", [(2, 1), (1, 2), (2, 2)])
def test_semi_galerkin_matches_scipy_triple_product(sx, sy):
    """Mapped grid with an interior Dirichlet body and two Neumann edges:
    the stencil-form product against (1/(sx sy)) P^T A P from SciPy with P
    restricted to the unknowns, and the coarse Dirichlet set against its
    definition (the coarse ring keeps the kind of the fine node under it;
    elsewhere a node is Dirichlet when its column of P has no free row)."""
    p = w.perturbed_circle(33)
    s = oracle.setup(p)
    neu = oracle.NEU_W | oracle.NEU_N
    dirs = oracle.dirichlet_set(p.nx, p.ny, p.mask, neu)
    st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], p.dx, p.dy, dirs)
    stc, dirc = oracle.galerkin_s(st, dirs, sx, sy)
    nyc, nxc = dirc.shape
    assert (nxc, nyc) == oracle.coarse_shape(33, 33, sx, sy)
    df = dirs.ravel().astype(bool)
    P0 = direct.tensor_P(33, 33, sx, sy)
    colnz = np.asarray(abs(P0[np.flatnonzero(~df)]).sum(axis=0)).ravel()
    ring = np.zeros((nyc, nxc), bool)
    ring[0, :] = ring[-1, :] = ring[:, 0] = ring[:, -1] = True
    under = dirs[::sy, ::sx].astype(bool)
    want = (ring & under) | (colnz == 0).reshape(nyc, nxc)
    assert np.array_equal(dirc.astype(bool), want)
    dc = dirc.ravel().astype(bool)
    Pm = P0.tolil()
    Pm[np.flatnonzero(df), :] = 0
    Pm[:, np.flatnonzero(dc)] = 0
    Pm = Pm.tocsr()
    Ar = direct.assemble_full(st).tolil()
    Ar[np.flatnonzero(df), :] = 0
    Ac = ((Pm.T @ Ar.tocsr() @ Pm) / (sx * sy)).toarray()
    Cs = direct.assemble_full(stc).toarray()
    free = np.flatnonzero(~dc)
    sub = np.ix_(free, free)
    assert np.allclose(Cs[sub], Ac[sub], rtol=1e-13, atol=1e-13 * abs(Ac).max())
    dn = np.flatnonzero(dc)
    assert np.all(stc[4].ravel()[dn] == 1.0)
    assert np.all(Cs[np.ix_(free, dn)] == 0.0)


@pytest.mark.parametrize("sx,sy", [(2, 1), (1, 2)])
def test_semi_transfers_match_matrix(sx, sy):
    """Prolongation = P e at free fine nodes (Dirichlet values untouched);
    restriction = P^T r / (sx sy) at interior coarse nodes and at free ring
    nodes, zero at Dirichlet ring nodes."""
    rng = np.random.default_rng(3)
    nxf, nyf = 17, 13
    nxc, nyc = oracle.coarse_shape(nxf, nyf, sx, sy)
    P0 = direct.tensor_P(nxf, nyf, sx, sy)
    e = rng.normal(size=(nyc, nxc))
    dirf = np.zeros((nyf, nxf), np.uint8)
    dirf[:, 0] = dirf[:, -1] = 1          # Dirichlet left and right, Neumann rows
    x0 = rng.normal(size=(nyf, nxf))
    out = oracle.prolong_add_s(e, x0, dirf, sx, sy)
    want = x0 + (P0 @ e.ravel()).reshape(nyf, nxf)
    keep = dirf.astype(bool)
    assert np.allclose(out[~keep], want[~keep], rtol=1e-15, atol=1e-14)
    assert np.array_equal(out[keep], x0[keep])
    r = rng.normal(size=(nyf, nxf))
    dirc = np.zeros((nyc, nxc), np.uint8)
    dirc[:, 0] = dirc[:, -1] = 1
    fc = oracle.restrict_s(r, sx, sy, dirc)
    ref = ((P0.T @ r.ravel()) / (sx * sy)).reshape(nyc, nxc)
    assert np.allclose(fc[:, 1:-1], ref[:, 1:-1], rtol=1e-14, atol=1e-14)
    assert np.all(fc[:, 0] == 0.0) and np.all(fc[:, -1] == 0.0)
    # without coarse flags the whole ring is zero
    fz = oracle.restrict_s(r, sx, sy)
    assert np.all(fz[0] == 0.0) and np.all(fz[-1] == 0.0)
    assert np.allclose(fz[1:-1, 1:-1], ref[1:-1, 1:-1], rtol=1e-14, atol=1e-14)


def test_semi_level_shapes():
    sh = oracle.levels(4097, 4097, neumann=12, semi=2, semi_axis=0)
    assert sh[:4] == [(4097, 4097), (2049, 4097), (1025, 4097), (513, 2049)]
    assert sh[-1] == (3, 9) and len(sh) == 12
    assert oracle.levels(257, 257, semi=1, semi_axis=1)[:3] == [(257, 257), (257, 129),
                                                                 (129, 65)]
    # a requested semi-coarsening that cannot be made refuses the grid
    assert oracle.levels(9, 9, semi=3, semi_axis=0) == []
    assert oracle.levels(129, 129, semi=0) == oracle.levels(129, 129)


def _annulus(n):
    p = w.polar_semi_annulus(n, neumann=True)
    s = oracle.setup(p)
    return p, s


def _mg(p, s, **kw):
    return oracle.MG.from_setup(s, p.dx, p.dy, mask=p.mask, **kw)


@pytest.mark.parametrize("n", [129, 257])
def test_semi_multigrid_rate_on_semi_annulus(n):
    """Halving only the radial axis (strong coupling) for two levels: the
    V(2,2) cycle contracts the residual by at least 5x per cycle at both
    sizes, where the full coarsening needs about twice as many cycles."""
    p, s = _annulus(n)
    mg = _mg(p, s, semi=2, semi_axis=0)
    assert [mg.strides(l) for l in range(2)] == [(2, 1), (2, 1)]
    assert mg.strides(2) == (2, 2)
    _, st, cyc, rel, hist = mg.solve(p.phi0, s["f"], 1e-10, 40, hist_len=41)
    assert st == 0 and cyc <= 10
    rates = hist[1:] / hist[:-1]
    assert np.median(rates) < 0.2
    full = _mg(p, s)
    _, st2, cyc2, _, _ = full.solve(p.phi0, s["f"], 1e-10, 60)
    assert st2 == 0 and cyc2 >= cyc + 5


@pytest.mark.parametrize("n,ny,neumann", [(65, 33, False), (129, 65, True)])
def test_semi_coarsening_fixes_the_aspect_two_annulus(n, ny, neumann):
    """The semi-annulus on half as many angular nodes (cells twice as long
    along the angle, radial coupling 18-110 times the angular one): point
    smoothing with full coarsening needs 70-140 cycles, with the radial axis
    halved alone for two levels at most 10."""
    p = w.polar_semi_annulus(n, ny=ny, neumann=neumann)
    s = oracle.setup(p)
    full = _mg(p, s)
    _, st0, c0, _, _ = full.solve(p.phi0, s["f"], 1e-10, 400)
    semi = _mg(p, s, semi=2, semi_axis=0)
    _, st2, c2, _, _ = semi.solve(p.phi0, s["f"], 1e-10, 400)
    assert st0 == 0 and st2 == 0
    assert c0 >= 60 and c2 <= 10, (c0, c2)


def test_semi_multigrid_converges_to_direct_solution():
    """The discrete solution does not depend on the hierarchy: at a 1e-13
    residual the semi-coarsened multigrid matches SciPy's sparse LU solve."""
    p, s = _annulus(129)
    mg = _mg(p, s, semi=2, semi_axis=0)
    phi, st, _, _, _ = mg.solve(p.phi0, s["f"], 1e-13, 60)
    assert st == 0
    ref = direct.direct_solve(mg.stencil(0), mg.dirs(0), s["f"], p.phi0)
    assert np.abs(phi - ref).max() <= 1e-11 * np.abs(ref).max()


def test_semi_y_axis_on_transposed_annulus():
    """The semi-annulus with its axes exchanged (radius along y): halving y
    converges like halving x did on the original, to the transposed
    solution."""
    p, s = _annulus(129)
    neu_t = oracle.NEU_W | oracle.NEU_E          # the Neumann rows become columns
    mgx = _mg(p, s, semi=2, semi_axis=0)
    phx, stx, cx, _, _ = mgx.solve(p.phi0, s["f"], 1e-12, 60)
    mgy = oracle.MG(s["eyy"].T, s["exy"].T, s["exx"].T, p.dy, p.dx, neumann=neu_t, semi=2,
                    semi_axis=1)
    assert [mgy.shape(l) for l in range(3)] == [(129, 129), (129, 65), (129, 33)]
    phy, sty, cy, _, _ = mgy.solve(np.ascontiguousarray(p.phi0.T), np.ascontiguousarray(s["f"].T),
                                   1e-12, 60)
    assert stx == 0 and sty == 0 and abs(cx - cy) <= 1
    assert np.abs(phy.T - phx).max() <= 1e-9 * np.abs(phx).max()

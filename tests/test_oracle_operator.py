"""Pins of the oracle's 9-point operator (eq. 17-18), its smoothers and the
multigrid transfer operators (Section 3) against textbook forms, polynomial
exactness and SciPy."""

import numpy as np
import numpy.polynomial.polynomial as P
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from oracle import direct
import workloads as w


def stencil_of(p, mask=None):
    s = oracle.setup(p)
    dirs = oracle.dirichlet_set(p.nx, p.ny, mask if mask is not None else p.mask)
    return oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], p.dx, p.dy, dirs), dirs, s


def test_identity_map_reduces_to_5_point_laplacian():
    """eps = I: the operator is exactly the textbook 5-point Laplacian."""
    n = 17
    p = w.identity_map(n)
    st, dirs, _ = stencil_of(p)
    Aff, _, _, _ = direct.split(st, dirs)
    L5 = direct.five_point_laplacian(n, p.dx)
    assert (abs(Aff - L5)).max() == 0.0
    # the four diagonal coefficients (k6) vanish identically
    for k in (0, 2, 6, 8):
        assert np.all(st[k] == 0.0)


def _poly2(rng):
    return rng.uniform(-1, 1, (3, 3))  # coefficients c[a, b] of x^a y^b


def test_biquadratic_exactness():
    """For biquadratic eps components and a biquadratic phi the central
    differences of eq. 18 are exact, so A phi equals the continuous
    div(eps grad phi) of eq. 16-17 at every free node (derivatives taken
    with numpy's polynomial routines)."""
    rng = np.random.default_rng(5)
    n, dx, dy = 9, 0.13, 0.07
    x = 0.2 + dx * np.arange(n)
    y = -0.1 + dy * np.arange(n)
    X, Y = np.meshgrid(x, y)
    cxx, cxy, cyy, cph = _poly2(rng), _poly2(rng) * 0.3, _poly2(rng), _poly2(rng)
    cxx[0, 0] += 3.0
    cyy[0, 0] += 3.0
    ev = lambda c: P.polyval2d(X, Y, c)
    d = lambda c, ax: P.polyder(c, axis=ax)
    exx, exy, eyy, phi = ev(cxx), ev(cxy), ev(cyy), ev(cph)
    fx, fy = d(cph, 0), d(cph, 1)
    cont = (ev(cxx) * ev(d(fx, 0)) + ev(d(cxx, 0)) * ev(fx)
            + 2 * ev(cxy) * ev(d(fx, 1)) + ev(d(cxy, 0)) * ev(fy) + ev(d(cxy, 1)) * ev(fx)
            + ev(cyy) * ev(d(fy, 1)) + ev(d(cyy, 1)) * ev(fy))
    dirs = oracle.dirichlet_set(n, n)
    st = oracle.fine_stencil(exx, exy, eyy, dx, dy, dirs)
    Aphi = oracle.apply(st, dirs, phi)
    inner = dirs == 0
    scale = np.max(np.abs(cont[inner]))
    assert np.max(np.abs(Aphi[inner] - cont[inner])) <= 1e-11 * scale


def test_operator_second_order_consistency():
    """Truncation error of A against the continuous operator for a smooth
    map and phi decays as h^2."""
    errs = []
    for n in (17, 33, 65):
        p = w.manufactured_sinusoidal(n)
        st, dirs, s = stencil_of(p)
        Aphi = oracle.apply(st, dirs, p.phi_exact)
        tau = Aphi - s["f"]  # A phi_exact - f at free nodes
        errs.append(np.max(np.abs(tau[dirs == 0])))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def test_symmetric_for_affine_map():
    """Constant eps (affine map): the assembled matrix is symmetric."""
    p = w.affine_map(17, [[1.2, 0.35], [-0.25, 0.8]])
    st, dirs, _ = stencil_of(p)
    Aff, _, _, _ = direct.split(st, dirs)
    asym = abs(Aff - Aff.T).max() / abs(Aff).max()
    assert asym <= 1e-15


def test_asymmetry_decays_first_order():
    """For variable eps the expanded (non-conservative) form of eq. 18 is not
    symmetric; the relative asymmetry decays like h."""
    vals = []
    for n in (9, 17, 33):
        p = w.manufactured_sinusoidal(n)
        st, dirs, _ = stencil_of(p)
        Aff, _, _, _ = direct.split(st, dirs)
        vals.append(abs(Aff - Aff.T).max() / abs(Aff).max())
    assert vals[0] > vals[1] > vals[2] > 0
    assert 1.7 < vals[0] / vals[1] < 2.3 and 1.7 < vals[1] / vals[2] < 2.3, vals


def test_operator_rows_annihilate_constants():
    """Every coefficient k1..k6 pairs with a difference, so A applied to a
    constant vanishes at free nodes (row sums are zero)."""
    p = w.perturbed_circle(65)
    st, dirs, _ = stencil_of(p)
    rs = st.sum(axis=0)
    assert np.max(np.abs(rs[dirs == 0])) <= 1e-9 * np.max(np.abs(st[4]))


def test_lexicographic_sweep_is_triangular_solve():
    """One Gauss-Seidel sweep in the paper's order (i outer, j inner) equals
    x_new = (D + L)^-1 (b - U x_old) in that ordering (SciPy triangular
    solve)."""
    p = w.manufactured_sinusoidal(11)
    st, dirs, s = stencil_of(p)
    rng = np.random.default_rng(2)
    x0 = p.phi0.copy()
    x0[dirs == 0] = rng.normal(size=(dirs == 0).sum())
    x1 = oracle.smooth(st, dirs, x0, s["f"], kind=oracle.GS_LEX, sweeps=1)
    Aff, Afd, free, dd = direct.split(st, dirs)
    # order free nodes by (i, j) lexicographically with i outer
    nx = p.nx
    ii, jj = free % nx, free // nx
    order = np.lexsort((jj, ii))
    A = Aff.toarray()[np.ix_(order, order)]
    b = (s["f"].ravel()[free] - Afd @ p.phi0.ravel()[dd])[order]
    xo = x0.ravel()[free][order]
    DL = np.tril(A)
    U = np.triu(A, 1)
    xn = spla.spsolve_triangular(sp.csr_matrix(DL), b - U @ xo, lower=True)
    assert np.allclose(x1.ravel()[free][order], xn, rtol=1e-13, atol=1e-13)


def test_gs4_sweep_is_colour_block_gauss_seidel():
    """One four-colour sweep equals block Gauss-Seidel over the colour
    blocks 0,1,2,3 (colour (i mod 2) + 2 (j mod 2)); inside a block the
    diagonal is all that couples, so each block solve is a division."""
    p = w.perturbed_circle(33)
    st, dirs, s = stencil_of(p)
    rng = np.random.default_rng(4)
    x0 = p.phi0.copy()
    x0[dirs == 0] = rng.normal(size=(dirs == 0).sum())
    x1 = oracle.smooth(st, dirs, x0, s["f"], kind=oracle.GS4, sweeps=1)
    A = direct.assemble_full(st).toarray()
    x = x0.ravel().copy()
    f = s["f"].ravel()
    nx = p.nx
    idx = np.arange(x.size)
    colour = (idx % nx) % 2 + 2 * ((idx // nx) % 2)
    free = dirs.ravel() == 0
    for c in range(4):
        blk = np.flatnonzero((colour == c) & free)
        Ab = A[np.ix_(blk, blk)]
        assert np.count_nonzero(Ab - np.diag(np.diag(Ab))) == 0
        rhs = f[blk] - A[blk] @ x + np.diag(Ab) * x[blk]
        x[blk] = rhs / np.diag(Ab)
    assert np.allclose(x1.ravel(), x, rtol=1e-13, atol=1e-13)


def test_jacobi_sweep():
    p = w.manufactured_sinusoidal(17)
    st, dirs, s = stencil_of(p)
    x0 = p.phi0.copy()
    x1 = oracle.smooth(st, dirs, x0, s["f"], kind=oracle.JACOBI, sweeps=1, omega=0.7)
    r = s["f"] - oracle.apply(st, dirs, x0)
    ref = x0 + np.where(dirs == 0, 0.7 * r / st[4], 0.0)
    assert np.allclose(x1, ref, rtol=1e-14, atol=1e-14)


def test_restriction_is_quarter_transpose_of_prolongation():
    """Full weighting R and bilinear P satisfy <R r, e> = (1/4) <r, P e> for
    r vanishing on the fine ring and e on the coarse ring."""
    rng = np.random.default_rng(7)
    nxf, nyf, nxc, nyc = 17, 9, 9, 5
    r = rng.normal(size=(nyf, nxf))
    r[0, :] = r[-1, :] = r[:, 0] = r[:, -1] = 0
    e = rng.normal(size=(nyc, nxc))
    e[0, :] = e[-1, :] = e[:, 0] = e[:, -1] = 0
    Rr = oracle.restrict_fw(r, nxc, nyc)
    dirf = np.zeros((nyf, nxf), np.uint8)
    Pe = oracle.prolong_add(e, np.zeros((nyf, nxf)), dirf)
    assert np.sum(Rr * e) == pytest.approx(0.25 * np.sum(r * Pe), rel=1e-13)
    # and the same P as the SciPy matrix
    Pm = direct.bilinear_P(nxc, nyc, nxf, nyf)
    assert np.allclose(Pe.ravel(), Pm @ e.ravel(), rtol=1e-15, atol=1e-15)


def test_prolongation_exact_on_bilinear_functions():
    nxc, nyc = 9, 7
    nxf, nyf = 17, 13
    X, Y = np.meshgrid(np.arange(nxc) * 2.0, np.arange(nyc) * 2.0)
    e = 0.3 + 1.7 * X - 0.4 * Y + 0.25 * X * Y
    Xf, Yf = np.meshgrid(np.arange(nxf) * 1.0, np.arange(nyf) * 1.0)
    exact = 0.3 + 1.7 * Xf - 0.4 * Yf + 0.25 * Xf * Yf
    dirf = np.zeros((nyf, nxf), np.uint8)
    dirf[0, :] = 1  # a Dirichlet row is left untouched
    out = oracle.prolong_add(e, np.zeros((nyf, nxf)), dirf)
    assert np.allclose(out[1:], exact[1:], rtol=1e-15, atol=1e-13)
    assert np.all(out[0] == 0.0)


def test_full_weighting_of_smooth_field():
    """FW preserves constants and linear functions at coarse interior nodes."""
    nxf = 17
    Xf, Yf = np.meshgrid(np.arange(nxf) * 1.0, np.arange(nxf) * 1.0)
    r = 2.0 + 0.5 * Xf - 0.25 * Yf
    c = oracle.restrict_fw(r, 9, 9)
    X, Y = np.meshgrid(np.arange(9) * 2.0, np.arange(9) * 2.0)
    ref = 2.0 + 0.5 * X - 0.25 * Y
    assert np.allclose(c[1:-1, 1:-1], ref[1:-1, 1:-1], rtol=1e-15)
    assert np.all(c[0] == 0) and np.all(c[:, -1] == 0)


def test_galerkin_of_laplacian_closed_form():
    """Galerkin coarsening (1/4) P^T A P of the 5-point Laplacian with
    bilinear P gives, away from the boundary, the 9-point stencil
    [[1,2,1],[2,-12,2],[1,2,1]] / (4 H^2) with H = 2h."""
    n = 33
    p = w.identity_map(n)
    st, dirs, _ = stencil_of(p)
    stc, dirc = oracle.galerkin(st, dirs, 17, 17)
    H = 2 * p.dx
    ref = np.array([1, 2, 1, 2, -12, 2, 1, 2, 1]) / (4 * H * H)
    for k in range(9):
        assert np.allclose(stc[k, 2:-2, 2:-2], ref[k], rtol=1e-13), k


def test_galerkin_matches_scipy_triple_product_with_mask():
    """Stencil-form Galerkin product on a masked, mapped grid against SciPy's
    (1/4) P^T A P with P restricted to the unknowns (zero rows at fine
    Dirichlet nodes, columns only for coarse non-Dirichlet nodes)."""
    p = w.perturbed_circle(33)
    st, dirs, _ = stencil_of(p)
    stc, dirc = oracle.galerkin(st, dirs, 17, 17)
    A = direct.assemble_full(st)
    Pm = direct.bilinear_P(17, 17, 33, 33).tolil()
    df = dirs.ravel().astype(bool)
    dc = dirc.ravel().astype(bool)
    Pm[np.flatnonzero(df), :] = 0
    Pm[:, np.flatnonzero(dc)] = 0
    Pm = Pm.tocsr()
    Ar = A.tolil()
    Ar[np.flatnonzero(df), :] = 0  # Dirichlet fine rows carry no equation
    Ac = (0.25 * (Pm.T @ Ar.tocsr() @ Pm)).toarray()
    # coarse Dirichlet nodes: exactly those whose P column is empty or ring
    colnz = np.asarray(abs(direct.bilinear_P(17, 17, 33, 33)[np.flatnonzero(~df)]).sum(axis=0)).ravel()
    ring = np.zeros((17, 17), bool)
    ring[0, :] = ring[-1, :] = ring[:, 0] = ring[:, -1] = True
    assert np.array_equal(dc, ring.ravel() | (colnz == 0))
    Cs = direct.assemble_full(stc).toarray()
    free = np.flatnonzero(~dc)
    sub = np.ix_(free, free)
    assert np.allclose(Cs[sub], Ac[sub], rtol=1e-13, atol=1e-13 * abs(Ac).max())
    # identity rows on coarse Dirichlet nodes; no coupling into them
    dn = np.flatnonzero(dc)
    assert np.all(stc[4].ravel()[dn] == 1.0)
    assert np.all(Cs[np.ix_(free, dn)] == 0.0)


def test_dense_solve_matches_numpy():
    rng = np.random.default_rng(11)
    A = rng.normal(size=(49, 49)) + 10 * np.eye(49)
    b = rng.normal(size=49)
    assert np.allclose(oracle.dense_solve(A, b), np.linalg.solve(A, b), rtol=1e-12)


def test_level_hierarchy():
    assert oracle.levels(129, 129) == [(129, 129), (65, 65), (33, 33), (17, 17), (9, 9)]
    assert len(oracle.levels(4097, 4097)) == 10
    assert oracle.levels(129, 65)[-1] == (9, 5)
    assert oracle.levels(9, 9) == [(9, 9), (5, 5)]
    # 200 = 8 * 25 stops halving at 26 nodes: kept as a large coarsest level
    assert oracle.levels(201, 201)[-1] == (26, 26)
    assert oracle.levels(1001, 1001) == []  # would stop at 126 x 126: refused
    assert oracle.levels(3, 3) == []

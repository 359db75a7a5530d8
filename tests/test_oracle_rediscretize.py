"""Pins of the oracle's rediscretised coarse operator (Section 3 leaves the
coarse operator of eq. 23 open; this option builds eq. 18 on each coarse grid
from the tensor sampled at the coarse nodes, the Dirichlet set sampled
likewise).  Each pin is fixed by something other than the oracle: the
textbook 5-point Laplacian, the closed-form polar tensor, array slicing of
the fine flags, and SciPy's sparse direct solve."""

import numpy as np
import pytest

import oracle
from oracle import direct
import workloads as w


def _mg(prob, **kw):
    s = oracle.setup(prob)
    return s, oracle.MG.from_setup(s, prob.dx, prob.dy, mask=prob.mask,
                                   coarse_op=oracle.REDISCRETIZE, **kw)


def test_identity_map_gives_the_five_point_laplacian_at_2h():
    """Identity map: every coarse level is the textbook 5-point Laplacian
    with the level's own spacing (2h, 4h, ...), exactly."""
    prob = w.identity_map(33)
    s, mg = _mg(prob)
    for l in range(1, mg.num_levels):
        nx, ny = mg.shape(l)
        H = prob.dx * 2 ** l
        st = mg.stencil(l)
        free = mg.dirs(l) == 0
        want = np.array([0, 1, 0, 1, -4, 1, 0, 1, 0], dtype=float) / (H * H)
        for k in range(9):
            assert np.array_equal(st[k][free], np.full(free.sum(), want[k])), (l, k)
        ring = np.ones((ny, nx), bool)
        ring[1:-1, 1:-1] = False
        assert np.array_equal(mg.dirs(l).astype(bool), ring)


def test_polar_map_closed_form():
    """Polar semi-annulus (eq. 29 with analytic J: eps_xx = xi, eps_yy =
    1/xi, eps_xy = 0): eq. 18 on level l at coarse node xi = xi0 + 2^l i dx
    has k1, k3 = xi/H^2 +- 1/(2H), k4 = k5 = 1/(xi K^2), k6 = 0 with H = 2^l
    dx, K = 2^l dy.  A wrong spacing, a wrong sampling index or a dropped
    derivative term changes these."""
    prob = w.polar_semi_annulus(65)
    s, mg = _mg(prob)
    for l in (1, 2, 3):
        nx, ny = mg.shape(l)
        H, K = prob.dx * 2 ** l, prob.dy * 2 ** l
        xi = prob.xi0 + H * np.arange(nx)
        st = mg.stencil(l)[:, 1:-1, 1:-1]
        X = np.broadcast_to(xi[1:-1], st[0].shape)
        ex = {1: 1 / (X * K * K), 3: X / H ** 2 - 1 / (2 * H), 5: X / H ** 2 + 1 / (2 * H),
              7: 1 / (X * K * K), 4: -2 * (X / H ** 2 + 1 / (X * K * K))}
        scale = np.max(np.abs(ex[4]))
        for k in range(9):
            want = ex.get(k, np.zeros_like(X))
            assert np.max(np.abs(st[k] - want)) <= 1e-12 * scale, (l, k)


def test_dirichlet_set_is_sampled():
    """Masked geometry: the coarse Dirichlet set is the fine one sampled at
    the coarse nodes (every 2^l-th node), plus the outer ring."""
    prob = w.perturbed_circle(65, seed=3)
    s, mg = _mg(prob)
    d0 = s["dir"].astype(bool)
    for l in range(1, mg.num_levels):
        nx, ny = mg.shape(l)
        want = d0[:: 2 ** l, :: 2 ** l].copy()
        want[0, :] = want[-1, :] = want[:, 0] = want[:, -1] = True
        assert np.array_equal(mg.dirs(l).astype(bool), want), l


@pytest.mark.parametrize("name", ["circle129", "sinusoidal65", "rect129x65"])
def test_multigrid_reaches_the_direct_solution(name):
    prob = {"circle129": lambda: w.perturbed_circle(129, seed=1),
            "sinusoidal65": lambda: w.manufactured_sinusoidal(65),
            "rect129x65": lambda: w.manufactured_sinusoidal(129, ny=65)}[name]()
    ro = oracle.solve_problem(prob, rel_tol=1e-13, max_cycles=300,
                              coarse_op=oracle.REDISCRETIZE)
    assert ro["status"] == 0
    s = ro["setup"]
    st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], prob.dx, prob.dy, s["dir"])
    ref = direct.direct_solve(st, s["dir"], s["f"], prob.phi0)
    assert np.max(np.abs(ro["phi"] - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_rate_on_the_manufactured_problem():
    """The smooth sinusoidal map: rediscretised V(2,2) cycles converge at a
    grid-independent rate (8-9 cycles to 1e-10, the rate the multigrid
    literature gives for a smooth variable-coefficient operator)."""
    cyc = []
    for n in (33, 65, 129, 257):
        ro = oracle.solve_problem(w.manufactured_sinusoidal(n), rel_tol=1e-10,
                                  coarse_op=oracle.REDISCRETIZE)
        assert ro["status"] == 0
        cyc.append(ro["cycles"])
    assert max(cyc) <= 11 and max(cyc) - min(cyc) <= 2, cyc


def test_rejects_stored_stencil_problems():
    prob = w.polar_semi_annulus(33, neumann=True)
    s = oracle.setup(prob)
    with pytest.raises(ValueError):
        oracle.MG.from_setup(s, prob.dx, prob.dy, coarse_op=oracle.REDISCRETIZE)

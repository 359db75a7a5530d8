"""Pins of the oracle's multigrid solve (Section 3) against direct solves,
and of the whole discretisation against the paper's closed-form solutions
and its second-order claim (Section 4)."""

import math

import numpy as np
import pytest

import oracle
from oracle import direct
import workloads as w


def reference(p):
    s = oracle.setup(p)
    st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], p.dx, p.dy, s["dir"])
    return s, st


@pytest.mark.parametrize("make", [lambda n: w.manufactured_sinusoidal(n),
                                  lambda n: w.perturbed_circle(n),
                                  lambda n: w.random_sinusoidal(n, 3)])
@pytest.mark.parametrize("n", [9, 17, 33])
def test_mg_matches_dense_direct_solve(make, n):
    p = make(n)
    s, st = reference(p)
    ref = direct.dense_solve(st, s["dir"], s["f"], p.phi0)
    r = oracle.solve_problem(p, rel_tol=1e-14, max_cycles=200)
    scale = max(np.max(np.abs(ref)), 1e-300)
    assert np.max(np.abs(r["phi"] - ref)) <= 1e-12 * scale


@pytest.mark.parametrize("make,n", [(w.manufactured_sinusoidal, 129), (w.perturbed_circle, 257)])
def test_mg_matches_sparse_direct_solve(make, n):
    p = make(n)
    s, st = reference(p)
    ref = direct.direct_solve(st, s["dir"], s["f"], p.phi0)
    r = oracle.solve_problem(p, rel_tol=1e-13, max_cycles=200)
    assert r["status"] == 0
    assert np.max(np.abs(r["phi"] - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_paper_ordering_reaches_same_solution():
    """The paper's lexicographic Gauss-Seidel and the four-colour ordering
    are different smoothers of the same discrete system."""
    p = w.perturbed_circle(65)
    a = oracle.solve_problem(p, rel_tol=1e-13, smoother=oracle.GS_LEX)
    b = oracle.solve_problem(p, rel_tol=1e-13, smoother=oracle.GS4)
    c = oracle.solve_problem(p, rel_tol=1e-13, smoother=oracle.JACOBI)
    assert a["status"] == b["status"] == c["status"] == 0
    sc = np.max(np.abs(b["phi"]))
    assert np.max(np.abs(a["phi"] - b["phi"])) <= 1e-11 * sc
    assert np.max(np.abs(c["phi"] - b["phi"])) <= 1e-11 * sc


def test_convergence_is_h_independent():
    """Regression guard: V(2,2) with Galerkin coarse operators contracts the
    residual by a grid-independent factor (well below 0.25 per cycle)."""
    for make in (w.manufactured_sinusoidal, w.perturbed_circle):
        cyc = []
        for n in (129, 257, 513):
            r = oracle.solve_problem(make(n), rel_tol=1e-10)
            assert r["status"] == 0
            cyc.append(r["cycles"])
            assert r["rel"] ** (1.0 / r["cycles"]) < 0.25
        assert max(cyc) - min(cyc) <= 2, cyc


def test_max_cycles_and_warm_start():
    p = w.manufactured_sinusoidal(65)
    r = oracle.solve_problem(p, rel_tol=1e-12, max_cycles=1)
    assert r["status"] == 1 and r["cycles"] == 1 and r["rel"] > 1e-12
    # restarting from the returned iterate continues with the same scaling
    mg, f = r["mg"], r["setup"]["f"]
    phi2, st2, cyc2, rel2, _ = mg.solve(r["phi"], f, 1e-12, 50)
    assert st2 == 0 and rel2 <= 1e-12


def test_zero_problem_converges_immediately():
    p = w.identity_map(17)
    r = oracle.solve_problem(p)
    assert r["status"] == 0 and r["cycles"] == 0 and r["rel"] == 0.0
    assert np.all(r["phi"] == 0.0)


def _orders(errs):
    return [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]


def test_manufactured_solution_second_order():
    """O(dx^2) error decay on the manufactured solution (sinusoidal map,
    amplitude 0.1); at 129^2 the max error is 5.97e-5."""
    errs = {}
    for n in (33, 65, 129, 257):
        p = w.manufactured_sinusoidal(n)
        r = oracle.solve_problem(p, rel_tol=1e-12)
        errs[n] = oracle.error_norms(r["phi"], p.phi_exact)
    for k in range(3):
        o = _orders([errs[n][k] for n in (33, 65, 129, 257)])
        assert all(1.9 < v < 2.1 for v in o), (k, o)
    assert errs[129][0] == pytest.approx(5.97e-5, rel=0.01)


def test_semi_annulus_second_order():
    """Section 4.1 (polar map, a = 2, R = 5, exact ln(R/r)/ln(R/a)): second
    order in L_inf, L_2 and L_1 (Dirichlet data from the exact solution on
    all four sides)."""
    errs = []
    for n in (33, 65, 129):
        p = w.polar_semi_annulus(n)
        r = oracle.solve_problem(p, rel_tol=1e-12, max_cycles=300)
        assert r["status"] == 0
        errs.append(oracle.error_norms(r["phi"], p.phi_exact))
    for k in range(3):
        o = _orders([e[k] for e in errs])
        assert all(1.85 < v < 2.15 for v in o), (k, o)


def test_disc_with_source_second_order():
    """Section 4.2.1: exact phi = (x'^2 + y'^2)/4 on the disc of radius 2
    with a uniform source; second order in the global norms (the corner
    nodes of the square, where det J = 0, cost the max norm a little)."""
    errs = []
    for n in (33, 65, 129):
        p = w.square_to_disc(n, 2.0, "source")
        r = oracle.solve_problem(p, rel_tol=1e-12, max_cycles=300)
        assert r["status"] == 0
        errs.append(oracle.error_norms(r["phi"], p.phi_exact))
    o2 = _orders([e[1] for e in errs])
    o1 = _orders([e[2] for e in errs])
    assert all(1.8 < v < 2.2 for v in o2 + o1), (o2, o1)


def test_disc_harmonic_second_order():
    """Section 4.2.2: exact r^8 sin(8 theta) on the unit disc."""
    errs = []
    for n in (65, 129, 257):
        p = w.square_to_disc(n, 1.0, "harmonic8")
        r = oracle.solve_problem(p, rel_tol=1e-12, max_cycles=300)
        assert r["status"] == 0
        errs.append(oracle.error_norms(r["phi"], p.phi_exact))
    for k in range(3):
        o = _orders([e[k] for e in errs])
        assert all(1.8 < v < 2.2 for v in o), (k, o)


def test_initial_residual_definition():
    """The stopping test divides by ||f - A phi0||_2 over free nodes, with
    phi0 equal to the Dirichlet data and zero on free nodes, whatever the
    iterate passed in."""
    p = w.perturbed_circle(65)
    s, st = reference(p)
    mg = oracle.MG.from_setup(s, p.dx, p.dy, mask=p.mask)
    guess = p.phi0 + np.where(s["dir"] == 0, 0.3, 0.0)
    b0 = mg.initial_residual(guess, s["f"])
    r = oracle.residual(st, s["dir"], p.phi0, s["f"])
    assert b0 == pytest.approx(np.sqrt(np.sum(r[s["dir"] == 0] ** 2)), rel=1e-14)


def test_stopping_test_when_zero_start_solves_the_problem():
    """Zero source and zero boundary data: the discrete solution is exactly
    zero (closed form).  The zero-interior start is converged at once; a
    non-zero warm start is measured against its own residual (the
    denominator ||f - A phi0|| is 0), so the multigrid iterates it down to
    the zero solution instead of returning it unchanged."""
    prob = w.manufactured_sinusoidal(33)
    prob.rho = np.zeros_like(prob.rho)
    prob.phi0 = np.zeros_like(prob.phi0)
    ro = oracle.solve_problem(prob, rel_tol=1e-10)
    assert ro["status"] == 0 and ro["cycles"] == 0 and ro["rel"] == 0.0
    xi, eta = np.meshgrid(np.linspace(0, 1, 33), np.linspace(0, 1, 33))
    x0 = np.sin(np.pi * xi) * np.sin(np.pi * eta)
    x0[0, :] = x0[-1, :] = x0[:, 0] = x0[:, -1] = 0.0  # the Dirichlet data stay 0
    s, mg = ro["setup"], ro["mg"]
    x, st, cyc, rel, hist = mg.solve(x0, s["f"], 1e-10, 100, hist_len=100)
    assert st == 0 and cyc > 0 and rel <= 1e-10
    assert hist[0] == 1.0
    assert np.max(np.abs(x)) <= 1e-8

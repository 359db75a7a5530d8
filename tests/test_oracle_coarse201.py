"""Pins of the oracle's larger coarsest level: the 201 x 201 grid of
Section 4.1 halves to 101, 51 and 26 nodes per side and stops there (25
intervals), so its coarsest direct solve is a 26 x 26 level.  The pins: the
multigrid solution of the semi-annulus (Dirichlet arcs, Neumann straight
sides, as the paper states it) at 201 x 201 is SciPy's sparse direct solution
of the same discrete system; the error against the closed form
ln(R/r)/ln(R/a) (eq. 28) falls at second order over the 201 family of grids
(101, 201, 401); the coarsest level keeps the ring's Neumann unknowns."""

import numpy as np
import pytest

import oracle
from oracle import direct
import workloads as w


def test_201_family_levels():
    assert oracle.levels(201, 201) == [(201, 201), (101, 101), (51, 51), (26, 26)]
    assert oracle.levels(201, 201, neumann=oracle.NEU_S | oracle.NEU_N)[-1] == (26, 26)
    assert oracle.levels(401, 401)[-1] == (26, 26)
    # a coarsest level that stays above 1024 nodes is refused
    assert oracle.levels(1001, 1001) == []
    # grids that halve down to 9 x 9 keep doing so
    assert oracle.levels(129, 129)[-1] == (9, 9)


@pytest.mark.parametrize("neumann", [False, True])
def test_semi_annulus_201_matches_direct_solve(neumann):
    q = w.polar_semi_annulus(201, neumann=neumann)
    r = oracle.solve_problem(q, rel_tol=1e-13, max_cycles=300)
    assert r["status"] == 0, r["rel"]
    mg = r["mg"]
    assert mg.shape(mg.num_levels - 1) == (26, 26)
    s = r["setup"]
    st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
    ref = direct.direct_solve(st, s["dir"], s["f"], q.phi0)
    err = np.max(np.abs(r["phi"] - ref)) / np.max(np.abs(ref))
    assert err < 1e-11, err


def test_semi_annulus_201_family_second_order():
    """eq. 28 on the 201 family: the maximum error falls by 4 per halving of h."""
    errs = []
    for n in (101, 201, 401):
        q = w.polar_semi_annulus(n, neumann=True)
        r = oracle.solve_problem(q, rel_tol=1e-12, max_cycles=300)
        assert r["status"] == 0
        errs.append(np.max(np.abs(r["phi"] - q.phi_exact)))
    assert 3.8 < errs[0] / errs[1] < 4.2 and 3.8 < errs[1] / errs[2] < 4.2, errs

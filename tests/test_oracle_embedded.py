"""Pins of the oracle on the embedded-body problems of Section 5.2: grid
generation with the map held on an embedded square's outline (eq. 44 for
the cylinder, eq. 51 for the deformed body) and the potential flow of eq. 47
around the body."""

import numpy as np

import oracle
from oracle import direct
import workloads as w


def _grid(n, kind, **kw):
    xb, yb, outline = w.embedded_body_boundary(n, kind, **kw)
    d = 10.0 / (n - 1)
    xp, yp = oracle.generate_grid(xb, yb, d, d, mask=outline)
    return xb, yb, outline, xp, yp


def test_held_outline_with_the_identity_map_gives_the_identity():
    # a linear map is discrete-harmonic: with the identity held on the ring
    # and on the outline, every generated node is its own computational node
    n = 33
    xb, yb, outline, xp, yp = _grid(n, "arbitrary", amp=0.0)
    q = w.embedded_flow(xp, yp)
    d = q.dx
    xi = -5.0 + d * np.arange(n)
    X, Y = np.meshgrid(xi, xi)
    assert np.max(np.abs(xp - X)) <= 1e-12 and np.max(np.abs(yp - Y)) <= 1e-12


def test_outline_and_ring_are_held():
    n = 65
    for kind in ("cylinder", "arbitrary"):
        xb, yb, outline, xp, yp = _grid(n, kind)
        held = outline.astype(bool)
        held[0] = held[-1] = held[:, 0] = held[:, -1] = True
        assert np.array_equal(xp[held], xb[held]) and np.array_equal(yp[held], yb[held])
    # the cylinder's outline lies on the circle of radius 2.5
    xb, yb, outline, _, _ = _grid(n, "cylinder")
    o = outline.astype(bool)
    assert np.max(np.abs(np.hypot(xb[o], yb[o]) - 2.5)) <= 1e-14


def test_stream_function_symmetry():
    # both bodies are symmetric about the y axis and their maps odd in y:
    # psi(-x, y) = psi(x, y), psi(x, -y) = -psi(x, y) (eq. 47 with psi0 = -psi1)
    for kind in ("cylinder", "arbitrary"):
        *_, xp, yp = _grid(65, kind)
        r = oracle.solve_problem(w.embedded_flow(xp, yp), rel_tol=1e-13, max_cycles=200)
        psi = r["phi"]
        assert r["status"] == 0
        assert np.max(np.abs(psi - psi[:, ::-1])) <= 1e-12
        assert np.max(np.abs(psi + psi[::-1, :])) <= 1e-12
        # the free stream runs in +x: psi increases upward away from the body
        n = psi.shape[0]
        assert np.all(np.diff(psi[:, 0]) > 0)


def test_multigrid_equals_direct_solve():
    for kind in ("cylinder", "arbitrary"):
        *_, xp, yp = _grid(33, kind)
        q = w.embedded_flow(xp, yp)
        r = oracle.solve_problem(q, rel_tol=1e-13, max_cycles=200)
        s = r["setup"]
        st = oracle.fine_stencil(s["exx"], s["exy"], s["eyy"], q.dx, q.dy, s["dir"])
        ref = direct.direct_solve(st, s["dir"], s["f"], q.phi0)
        assert np.max(np.abs(r["phi"] - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_cylinder_converges_to_the_unbounded_flow():
    """With the outer data of psi = y'(1 - R^2/r'^2) (the flow past a circle
    of radius R = 2.5 in an unbounded stream, zero on the circle) the
    discrete stream function converges to it.  The outline map sends the
    square's corners to points of a smooth circle, so the generated map is
    singular there (det J -> 0) and the errors fall at about first order."""
    errs = []
    for n in (65, 129, 257):
        *_, xp, yp = _grid(n, "cylinder")
        q = w.embedded_flow(xp, yp, data="cylinder_exact")
        r = oracle.solve_problem(q, rel_tol=1e-13, max_cycles=300)
        e = r["phi"] - q.phi_exact
        errs.append((np.max(np.abs(e)), np.sqrt(np.sum(e ** 2)) / n))
    print(errs)
    for (li0, l20), (li1, l21) in zip(errs, errs[1:]):
        assert l20 / l21 >= 1.7 and li1 < li0
    assert errs[-1][1] <= 6e-3

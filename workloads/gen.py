"""Problem generators (inputs only; see the package docstring).

Conventions shared with both solvers:

* node (i, j) has computational coordinates xi_i = xi0 + i*dx (i < nx) and
  eta_j = eta0 + j*dy (j < ny); every node field is a float64 array of shape
  (ny, nx), so element (i, j) is ``a[j, i]`` and x (i) runs fastest in memory;
* ``xp, yp`` are the physical coordinates x'(xi_ij), y'(xi_ij) of the nodes;
* ``jac`` (analytic maps only) is an array (4, ny, nx) holding the partials
  dx'/dxi, dx'/deta, dy'/dxi, dy'/deta (the paper's J_xx, J_xy, J_yx, J_yy);
* ``rho`` is the physical charge density rho' sampled at (xp, yp); the problem
  solved is div'(grad' phi) = -rho' in the physical domain;
* ``mask`` (uint8, or None) marks interior nodes held at a Dirichlet value;
  the outer ring of nodes is Dirichlet except on the edges named by
  ``neumann`` (zero normal derivative there);
* ``phi0`` carries the Dirichlet data on the outer ring and on masked nodes,
  and zero on every free node;
* ``phi_exact`` (when a closed form exists) is the continuous solution at the
  nodes.

Random draws use ``numpy.random.default_rng(seed)`` (PCG64) in the order the
functions below state, so a seed fixes a problem exactly.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class GridProblem:
    name: str
    nx: int
    ny: int
    xi0: float
    eta0: float
    dx: float
    dy: float
    xp: np.ndarray
    yp: np.ndarray
    rho: np.ndarray
    phi0: np.ndarray
    jac: Optional[np.ndarray] = None
    mask: Optional[np.ndarray] = None
    phi_exact: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)
    # edges with a zero normal derivative instead of Dirichlet data, bits
    # 1: i = 0, 2: i = nx-1, 4: j = 0, 8: j = ny-1
    neumann: int = 0

    @property
    def dof(self) -> int:
        return self.nx * self.ny


def _grid(nx, ny, xi0, eta0, dx, dy):
    xi = xi0 + dx * np.arange(nx, dtype=np.float64)
    eta = eta0 + dy * np.arange(ny, dtype=np.float64)
    XI, ETA = np.meshgrid(xi, eta)  # shape (ny, nx), XI varies along axis 1
    return XI, ETA


def _outer_ring(ny, nx):
    ring = np.zeros((ny, nx), dtype=bool)
    ring[0, :] = ring[-1, :] = True
    ring[:, 0] = ring[:, -1] = True
    return ring


def _phi0_from(values, ring_or_dir):
    phi0 = np.zeros_like(values)
    phi0[ring_or_dir] = values[ring_or_dir]
    return phi0


# ----------------------------------------------------------------------------
# Plain maps (used by the oracle's pins)
# ----------------------------------------------------------------------------

def identity_map(n: int, L: float = 1.0, rho=None, name="identity") -> GridProblem:
    """x' = xi, y' = eta on [0, L]^2; rho' given as a callable of (x', y')."""
    d = L / (n - 1)
    XI, ETA = _grid(n, n, 0.0, 0.0, d, d)
    jac = np.zeros((4, n, n))
    jac[0] = 1.0
    jac[3] = 1.0
    r = np.zeros((n, n)) if rho is None else rho(XI, ETA)
    return GridProblem(name, n, n, 0.0, 0.0, d, d, XI.copy(), ETA.copy(), r,
                       np.zeros((n, n)), jac=jac)


def affine_map(n: int, M, shift=(0.0, 0.0), name="affine") -> GridProblem:
    """x' = M @ (xi, eta) + shift on the unit square (constant Jacobian M)."""
    M = np.asarray(M, dtype=np.float64)
    d = 1.0 / (n - 1)
    XI, ETA = _grid(n, n, 0.0, 0.0, d, d)
    xp = M[0, 0] * XI + M[0, 1] * ETA + shift[0]
    yp = M[1, 0] * XI + M[1, 1] * ETA + shift[1]
    jac = np.empty((4, n, n))
    jac[0], jac[1], jac[2], jac[3] = M[0, 0], M[0, 1], M[1, 0], M[1, 1]
    return GridProblem(name, n, n, 0.0, 0.0, d, d, xp, yp, np.zeros((n, n)),
                       np.zeros((n, n)), jac=jac)


def sinusoidal_map(n: int, amp: float, ny: Optional[int] = None):
    """x' = xi + A s, y' = eta + A s with s = sin(pi xi) sin(pi eta) on the
    unit square.  Returns (XI, ETA, xp, yp, jac).  The map is the identity on
    the boundary of the square."""
    ny = n if ny is None else ny
    XI, ETA = _grid(n, ny, 0.0, 0.0, 1.0 / (n - 1), 1.0 / (ny - 1))
    s = np.sin(np.pi * XI) * np.sin(np.pi * ETA)
    a = amp * np.pi * np.cos(np.pi * XI) * np.sin(np.pi * ETA)  # d s/d xi * A
    b = amp * np.pi * np.sin(np.pi * XI) * np.cos(np.pi * ETA)  # d s/d eta * A
    xp = XI + amp * s
    yp = ETA + amp * s
    jac = np.stack([1.0 + a, b, a, 1.0 + b])
    return XI, ETA, xp, yp, jac


def manufactured_sinusoidal(n: int = 129, amp: float = 0.1, ny: Optional[int] = None) -> GridProblem:
    """The 129^2 manufactured-solution workload: sinusoidal map of amplitude
    0.1, phi = sin(pi x') sin(pi y') + x' y', rho' = 2 pi^2 sin(pi x') sin(pi y')
    (so that the physical Laplacian of phi is -rho'), Dirichlet data from phi."""
    ny = n if ny is None else ny
    XI, ETA, xp, yp, jac = sinusoidal_map(n, amp, ny)
    phi = np.sin(np.pi * xp) * np.sin(np.pi * yp) + xp * yp
    rho = 2.0 * np.pi ** 2 * np.sin(np.pi * xp) * np.sin(np.pi * yp)
    ring = _outer_ring(ny, n)
    return GridProblem(f"manufactured_sinusoidal_{n}x{ny}", n, ny, 0.0, 0.0,
                       1.0 / (n - 1), 1.0 / (ny - 1), xp, yp, rho,
                       _phi0_from(phi, ring), jac=jac, phi_exact=phi,
                       meta={"amp": amp})


def polar_semi_annulus(n: int, a: float = 2.0, R: float = 5.0, phi_a: float = 1.0,
                       ny: Optional[int] = None, neumann: bool = False) -> GridProblem:
    """Polar map x' = xi cos(eta), y' = xi sin(eta) with xi in [a, R] and eta in
    [0, pi] (the paper's semi-annulus, Section 4.1, with a = 2, R = 5).
    rho' = 0; exact phi = phi_a ln(R/r)/ln(R/a).  Dirichlet data from the exact
    solution on the whole outer ring, or, with neumann=True, as in the paper:
    Dirichlet data on the arcs r = a, R only and a zero normal derivative on the
    two straight sides eta = 0, pi (the exact solution satisfies both)."""
    ny = n if ny is None else ny
    dx = (R - a) / (n - 1)
    dy = math.pi / (ny - 1)
    XI, ETA = _grid(n, ny, a, 0.0, dx, dy)
    xp = XI * np.cos(ETA)
    yp = XI * np.sin(ETA)
    jac = np.stack([np.cos(ETA), -XI * np.sin(ETA), np.sin(ETA), XI * np.cos(ETA)])
    phi = phi_a * np.log(R / XI) / math.log(R / a)
    ring = _outer_ring(ny, n)
    if neumann:
        ring[1:-1, :] = False
        ring[:, 1:-1] = False
        ring[:, 0] = ring[:, -1] = True
    return GridProblem(f"semi_annulus_{n}" + ("_neumann" if neumann else ""), n, ny, a, 0.0,
                       dx, dy, xp, yp, np.zeros((ny, n)), _phi0_from(phi, ring), jac=jac,
                       phi_exact=phi, meta={"a": a, "R": R}, neumann=12 if neumann else 0)


def sinh_stretch(n: int = 129, s: float = 5.0, alpha: float = 0.6, L: float = 6.0,
                 rho0: float = 100.0, sigma: float = 0.5) -> GridProblem:
    """The stretched grid of Section 5.1: x' = s sinh(alpha xi), y' = s sinh(alpha
    eta) on the computational square [-L/2, L/2]^2, with the Gaussian beam
    rho' = -rho0 exp(-(x'^2 + y'^2)/(2 sigma^2)) centred at the origin.
    Outer boundary phi = 0."""
    d = L / (n - 1)
    XI, ETA = _grid(n, n, -L / 2, -L / 2, d, d)
    xp = s * np.sinh(alpha * XI)
    yp = s * np.sinh(alpha * ETA)
    z = np.zeros_like(XI)
    jac = np.stack([s * alpha * np.cosh(alpha * XI), z, z, s * alpha * np.cosh(alpha * ETA)])
    rho = -rho0 * np.exp(-(xp ** 2 + yp ** 2) / (2 * sigma ** 2))
    return GridProblem(f"sinh_stretch_{n}", n, n, -L / 2, -L / 2, d, d, xp, yp, rho,
                       np.zeros((n, n)), jac=jac, meta={"s": s, "alpha": alpha})


def square_to_disc(n: int, b: float, kind: str) -> GridProblem:
    """Closed-form square-to-disc map on [-b, b]^2:
        x' = xi sqrt(1 - eta^2/(2 b^2)),  y' = eta sqrt(1 - xi^2/(2 b^2)).
    On the four sides of the square it takes exactly the boundary values the
    paper prescribes for its circular-domain grids (eq. 44), so it stands in for
    the Laplace-generated interior map of Section 4.2.  Its Jacobian vanishes
    only at the four corner nodes.

    kind = "source": rho' = -1 in this library's convention (the paper's
    uniform source of Section 4.2.1 is written with the opposite sign),
    exact phi = (x'^2 + y'^2)/4, boundary phi = b^2/4.
    kind = "harmonic8": rho' = 0, exact phi = r^8 sin(8 theta) (Section 4.2.2,
    with b = 1)."""
    d = 2.0 * b / (n - 1)
    XI, ETA = _grid(n, n, -b, -b, d, d)
    sy = np.sqrt(1.0 - ETA ** 2 / (2 * b * b))
    sx = np.sqrt(1.0 - XI ** 2 / (2 * b * b))
    xp = XI * sy
    yp = ETA * sx
    jac = np.stack([sy, -XI * ETA / (2 * b * b * sy), -XI * ETA / (2 * b * b * sx), sx])
    if kind == "source":
        phi = (xp ** 2 + yp ** 2) / 4.0
        rho = -np.ones_like(xp)
    elif kind == "harmonic8":
        r = np.hypot(xp, yp)
        th = np.arctan2(yp, xp)
        phi = r ** 8 * np.sin(8 * th)
        rho = np.zeros_like(xp)
    else:
        raise ValueError(kind)
    ring = _outer_ring(n, n)
    return GridProblem(f"disc_{kind}_{n}", n, n, -b, -b, d, d, xp, yp, rho,
                       _phi0_from(phi, ring), jac=jac, phi_exact=phi, meta={"b": b})


def disc_boundary(n: int, b: float):
    """Boundary data of the numerically generated circular grid of Section
    4.2 (eq. 44) on the computational square [-b, b]^2: returns (xb, yb), node
    arrays holding x'(xi, eta), y'(xi, eta) of eq. 44 on the outer ring and
    zero elsewhere (the interior is found by solving eq. 36-37)."""
    d = 2.0 * b / (n - 1)
    XI, ETA = _grid(n, n, -b, -b, d, d)
    xb, yb = np.zeros((n, n)), np.zeros((n, n))
    # bottom (eta = -b) and top (eta = b): x' = xi / sqrt 2, y' = -+b sqrt(1 - xi^2/(2b^2))
    for row, sgn in ((0, -1.0), (n - 1, 1.0)):
        xb[row] = XI[row] / math.sqrt(2.0)
        yb[row] = sgn * b * np.sqrt(1.0 - XI[row] ** 2 / (2 * b * b))
    # left (xi = -b) and right (xi = b): x' = -+b sqrt(1 - eta^2/(2b^2)), y' = eta / sqrt 2
    for col, sgn in ((0, -1.0), (n - 1, 1.0)):
        xb[:, col] = sgn * b * np.sqrt(1.0 - ETA[:, col] ** 2 / (2 * b * b))
        yb[:, col] = ETA[:, col] / math.sqrt(2.0)
    return xb, yb


def disc_on_grid(xp, yp, b: float, kind: str) -> GridProblem:
    """The circular-domain problems of Section 4.2 on a given (for example
    numerically generated) grid of the square [-b, b]^2, numeric Jacobian.
    kind = "source": rho' = -1 in this library's convention, exact phi =
    (x'^2 + y'^2)/4 (eq. 43); kind = "harmonic8": rho' = 0, exact
    phi = r^8 sin(8 theta) (eq. 45)."""
    n = xp.shape[0]
    d = 2.0 * b / (n - 1)
    if kind == "source":
        phi = (xp ** 2 + yp ** 2) / 4.0
        rho = -np.ones_like(xp)
    elif kind == "harmonic8":
        r = np.hypot(xp, yp)
        th = np.arctan2(yp, xp)
        phi = r ** 8 * np.sin(8 * th)
        rho = np.zeros_like(xp)
    else:
        raise ValueError(kind)
    ring = _outer_ring(n, n)
    return GridProblem(f"generated_disc_{kind}_{n}", n, n, -b, -b, d, d, np.ascontiguousarray(xp),
                       np.ascontiguousarray(yp), rho, _phi0_from(phi, ring), jac=None,
                       phi_exact=phi, meta={"b": b})


def embedded_body_boundary(n: int = 257, kind: str = "cylinder", L: float = 10.0,
                           half: float = 2.5, a: float = 10.0, n_osc: int = 3,
                           amp: Optional[float] = None):
    """Boundary data of the grids of Section 5.2: an embedded body in the
    computational square [-L/2, L/2]^2, which the map leaves fixed on its
    outer ring.  The body is the computational square [-half, half]^2; the
    nodes of its outline carry the body's map:
      kind = "cylinder": the square-to-disc map of eq. 44 (a circle of radius
        half);
      kind = "arbitrary": eq. 51, each side of the square displaced normally by
        amp sin(pi n_osc s) (s in [0, 1] along the side), outward on the
        sides x = half, y = half, inward on x = -half, y = -half; amp defaults
        to a times the spacing of the paper's 257-node grid (a = 10: 0.39),
        kept fixed in physical units at other resolutions.
    Returns (xb, yb, outline): the map on the outer ring (the identity) and on
    the outline (uint8 mask), zero elsewhere; the other nodes are found by
    solving eq. 36-37 (grid generation with the outline held)."""
    d = L / (n - 1)
    k0 = half / d
    if abs(k0 - round(k0)) > 1e-9:
        raise ValueError("the body's square must fall on grid lines")
    XI, ETA = _grid(n, n, -L / 2, -L / 2, d, d)
    ring = _outer_ring(n, n)
    lo, hi = (n - 1) // 2 - int(round(k0)), (n - 1) // 2 + int(round(k0))
    outline = np.zeros((n, n), dtype=bool)
    outline[lo:hi + 1, lo] = outline[lo:hi + 1, hi] = True
    outline[lo, lo:hi + 1] = outline[hi, lo:hi + 1] = True
    xb, yb = np.zeros((n, n)), np.zeros((n, n))
    xb[ring], yb[ring] = XI[ring], ETA[ring]
    xs, ys = XI[outline], ETA[outline]
    if kind == "cylinder":
        b = half
        on_x = np.isclose(np.abs(xs), b)  # the sides xi = -+b (corners included)
        xo = np.where(on_x, np.sign(xs) * b * np.sqrt(1.0 - ys ** 2 / (2 * b * b)),
                      xs / math.sqrt(2.0))
        yo = np.where(on_x, ys / math.sqrt(2.0),
                      np.sign(ys) * b * np.sqrt(1.0 - xs ** 2 / (2 * b * b)))
    elif kind == "arbitrary":
        A = a * (L / 256.0) if amp is None else amp
        sx = np.sin(np.pi * n_osc * (ys + half) / (2 * half))
        sy = np.sin(np.pi * n_osc * (xs + half) / (2 * half))
        xo = np.where(np.isclose(xs, -half), xs - A * sx,
                      np.where(np.isclose(xs, half), xs + A * sx, xs))
        yo = np.where(np.isclose(ys, -half), ys - A * sy,
                      np.where(np.isclose(ys, half), ys + A * sy, ys))
    else:
        raise ValueError(kind)
    xb[outline], yb[outline] = xo, yo
    return xb, yb, outline.astype(np.uint8)


def embedded_flow(xp, yp, L: float = 10.0, half: float = 2.5, psi0: float = -1.0,
                  psi1: float = 1.0, data: str = "eq47") -> GridProblem:
    """The potential-flow problem of Section 5.2 on a generated grid (xp, yp)
    of the computational square [-L/2, L/2]^2: the stream function solves
    Laplace's equation (rho' = 0) with psi = 0 on the body, the computational
    square [-half, half]^2 (its nodes are Dirichlet nodes), and on the outer
    ring
      data = "eq47": the values of eq. 47 -- psi0 on the bottom edge, psi1 on
        the top, varying linearly in y on the inflow and outflow edges;
      data = "cylinder_exact": the unbounded flow past a circle of radius
        half, psi = y' (1 - half^2 / r'^2), which vanishes on the circle the
        cylinder grid maps the body's outline onto; phi_exact holds it at
        every node (a closed form for the whole discrete problem).
    Numeric Jacobian from the node coordinates."""
    n = xp.shape[0]
    d = L / (n - 1)
    XI, ETA = _grid(n, n, -L / 2, -L / 2, d, d)
    ring = _outer_ring(n, n)
    body = (np.abs(XI) <= half + 1e-12) & (np.abs(ETA) <= half + 1e-12)
    phi0 = np.zeros((n, n))
    exact = None
    if data == "eq47":
        phi0[ring] = psi0 + (psi1 - psi0) * (ETA[ring] + L / 2) / L
    elif data == "cylinder_exact":
        r2 = xp ** 2 + yp ** 2
        exact = np.where(body, 0.0, yp * (1.0 - half * half / np.maximum(r2, 1e-300)))
        phi0[ring] = exact[ring]
    else:
        raise ValueError(data)
    return GridProblem(f"embedded_flow_{data}_{n}", n, n, -L / 2, -L / 2, d, d,
                       np.ascontiguousarray(xp), np.ascontiguousarray(yp), np.zeros((n, n)),
                       phi0, jac=None, mask=body.astype(np.uint8), phi_exact=exact,
                       meta={"L": L, "half": half, "psi": (psi0, psi1), "data": data})


# ----------------------------------------------------------------------------
# Benchmark workloads
# ----------------------------------------------------------------------------

def gaussian_sources(xp, yp, amps, centres, sigma):
    """rho'(x') = sum_m A_m exp(-|x' - c_m|^2 / (2 sigma^2))."""
    rho = np.zeros_like(xp)
    inv = 1.0 / (2.0 * sigma * sigma)
    for A, (cx, cy) in zip(amps, centres):
        rho += A * np.exp(-((xp - cx) ** 2 + (yp - cy) ** 2) * inv)
    return rho


def _boundary_radius(theta, acoef):
    k = np.arange(2, 6, dtype=np.float64)
    return 0.2 + 0.03 * np.sum(acoef[None, :] * np.cos(np.outer(theta, k)), axis=1)


def draw_circle(rng):
    """Perturbation coefficients a_2..a_5 of the conductor boundary, drawn
    uniform in [-1, 1] and redrawn until 0.16 <= R(theta) <= 0.34 on 4096
    equispaced angles."""
    tt = np.linspace(0.0, 2 * np.pi, 4096, endpoint=False)
    while True:
        acoef = rng.uniform(-1.0, 1.0, 4)
        Rs = _boundary_radius(tt, acoef)
        if Rs.min() >= 0.16 and Rs.max() <= 0.34:
            return acoef


def draw_circle_sources(rng, acoef, n_gauss):
    """Amplitudes (standard normal) and centres (uniform on the unit square,
    each redrawn while inside the physical conductor) of the Gaussians."""
    amps = rng.standard_normal(n_gauss)
    centres = []
    for _ in range(n_gauss):
        while True:
            c = rng.uniform(0.0, 1.0, 2)
            tc = math.atan2(c[1] - 0.5, c[0] - 0.5)
            if math.hypot(c[0] - 0.5, c[1] - 0.5) > _boundary_radius(np.array([tc]), acoef)[0]:
                break
        centres.append(c)
    return amps, centres


def draw_sinusoidal(rng, n_gauss=4, amp_max=0.15):
    """Map amplitude U(0, amp_max), then the sources (see draw_box_sources)."""
    amp = float(rng.uniform(0.0, amp_max))
    amps, centres = draw_box_sources(rng, n_gauss)
    return amp, amps, centres


def draw_box_sources(rng, n_gauss=4):
    """Amplitudes (standard normal) and centres uniform in [0.1, 0.9]^2."""
    amps = rng.standard_normal(n_gauss)
    centres = rng.uniform(0.1, 0.9, (n_gauss, 2))
    return amps, centres


def perturbed_circle(n: int = 4097, seed: int = 0, n_gauss: int = 8, sigma: float = 0.02,
                     draw_sources: bool = True) -> GridProblem:
    """Perturbed-circle conductor on the unit square (the 4097^2 workload).

    Draw order with rng = default_rng(seed):
      1. a = rng.uniform(-1, 1, 4), redrawn until the boundary radius
         R(theta) = 0.2 + 0.03 sum_{k=2..5} a_k cos(k theta) lies in
         [0.16, 0.34] on 4096 equispaced theta samples;
      2. amplitudes A = rng.standard_normal(n_gauss);
      3. for each source in turn, c = rng.uniform(0, 1, 2), redrawn while it
         lies inside the physical conductor (|c - (1/2, 1/2)| <= R(theta_c)).
    Map (computational -> physical), radial about the centre (1/2, 1/2), with
    r = |xi - centre| and theta its polar angle:
      r' = r                                      for r < 0.15 or r > 0.35,
      r' = 0.15 + (r - 0.15)(R - 0.15)/0.05       for 0.15 <= r <= 0.2,
      r' = R + (r - 0.2)(0.35 - R)/0.15           for 0.2 < r <= 0.35.
    It carries the computational circle r = 0.2 onto the physical perturbed
    circle r' = R(theta).  Nodes with r <= 0.2 form the conductor (Dirichlet
    phi = 1, a staircase in the computational grid); the outer ring is phi = 0.
    The map is numeric: only node coordinates are supplied (no ``jac``)."""
    rng = np.random.default_rng(seed)
    acoef = draw_circle(rng)
    d = 1.0 / (n - 1)
    XI, ETA = _grid(n, n, 0.0, 0.0, d, d)
    ux = XI - 0.5
    uy = ETA - 0.5
    r = np.hypot(ux, uy)
    th = np.arctan2(uy, ux)
    Rth = _boundary_radius(th.ravel(), acoef).reshape(th.shape)
    rp = r.copy()
    inner = (r >= 0.15) & (r <= 0.2)
    outer = (r > 0.2) & (r <= 0.35)
    rp[inner] = 0.15 + (r[inner] - 0.15) * (Rth[inner] - 0.15) / 0.05
    rp[outer] = Rth[outer] + (r[outer] - 0.2) * (0.35 - Rth[outer]) / 0.15
    xp = 0.5 + rp * np.cos(th)
    yp = 0.5 + rp * np.sin(th)
    mask = (r <= 0.2).astype(np.uint8)
    if draw_sources:
        amps, centres = draw_circle_sources(rng, acoef, n_gauss)
        rho = gaussian_sources(xp, yp, amps, centres, sigma)
    else:
        amps, centres = np.zeros(0), []
        rho = np.zeros_like(xp)
    phi0 = np.zeros((n, n))
    phi0[mask.astype(bool)] = 1.0
    return GridProblem(f"perturbed_circle_{n}_s{seed}", n, n, 0.0, 0.0, d, d, xp, yp, rho,
                       phi0, jac=None, mask=mask,
                       meta={"seed": seed, "a": acoef.tolist(), "amps": np.asarray(amps).tolist(),
                             "centres": [list(map(float, c)) for c in centres], "sigma": sigma})


def random_sinusoidal(n: int, seed: int, n_gauss: int = 4, sigma: float = 0.02,
                      amp_max: float = 0.15) -> GridProblem:
    """Sinusoidal-map problem of the batched workload.  Draw order with
    rng = default_rng(seed): amplitude A = rng.uniform(0, amp_max); source
    amplitudes rng.standard_normal(n_gauss); centres rng.uniform(0.1, 0.9,
    (n_gauss, 2)).  Outer phi = 0, no interior mask, analytic Jacobian."""
    rng = np.random.default_rng(seed)
    amp, amps, centres = draw_sinusoidal(rng, n_gauss, amp_max)
    XI, ETA, xp, yp, jac = sinusoidal_map(n, amp)
    rho = gaussian_sources(xp, yp, amps, centres, sigma)
    d = 1.0 / (n - 1)
    return GridProblem(f"sinusoidal_{n}_s{seed}", n, n, 0.0, 0.0, d, d, xp, yp, rho,
                       np.zeros((n, n)), jac=jac,
                       meta={"seed": seed, "amp": amp, "amps": amps.tolist(),
                             "centres": centres.tolist(), "sigma": sigma})


def batch_mixed(count: int = 256, base_seed: int = 1000,
                sides=(65, 129, 257, 513, 1025)):
    """The batched workload: problem p uses seed base_seed + p; its side is
    drawn first with default_rng(seed).integers(len(sides)), then the
    remaining draws follow random_sinusoidal with the same seed offset by one
    (seed + 10**6), so that the side draw does not shift the map draws."""
    out = []
    for p in range(count):
        s = base_seed + p
        side = sides[int(np.random.default_rng(s).integers(len(sides)))]
        out.append(random_sinusoidal(side, s + 10 ** 6))
    return out


def draw_annulus_sources(rng, n_gauss=4):
    """Gaussian sources inside the semi-annulus 2 <= r <= 5, 0 <= theta <= pi:
    amplitudes N(0,1), centres at r ~ U(2.5, 4.5), theta ~ U(0.2, pi - 0.2)
    (drawn in that order per source)."""
    amps, centres = [], []
    for _ in range(n_gauss):
        amps.append(float(rng.normal()))
        r, th = float(rng.uniform(2.5, 4.5)), float(rng.uniform(0.2, math.pi - 0.2))
        centres.append((r * math.cos(th), r * math.sin(th)))
    return np.asarray(amps), centres


def serving_stream(count: int, rate: float, seed: int = 7,
                   sides=(129, 257, 513, 1025, 2049), warm_frac: float = 0.3,
                   kinds=("circle", "sinusoidal")):
    """Request descriptors for the serving workload (no arrays are built here).

    rng = default_rng(seed).  Arrival gaps are exponential with mean 1/rate
    seconds.  For each request, in order: gap; u = rng.uniform() (< warm_frac
    selects a warm re-solve of an already-seen geometry, when one exists);
    for a cold request the side index rng.integers(len(sides)), the geometry
    kind kinds[rng.integers(len(kinds))] (by default perturbed circle or
    sinusoidal map; "annulus" adds the semi-annulus with Neumann sides) and a
    geometry seed rng.integers(2**31); for a warm request the index of the
    earlier geometry rng.integers(number seen so far) and a fresh source seed
    rng.integers(2**31)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    geoms = []
    for k in range(count):
        t += float(rng.exponential(1.0 / rate))
        u = float(rng.uniform())
        if u < warm_frac and geoms:
            g = geoms[int(rng.integers(len(geoms)))]
            reqs.append({"id": k, "t": t, "warm": True, "geom": g["gid"], "side": g["side"],
                         "kind": g["kind"], "geom_seed": g["geom_seed"],
                         "source_seed": int(rng.integers(2 ** 31))})
        else:
            side = sides[int(rng.integers(len(sides)))]
            kind = kinds[int(rng.integers(len(kinds)))]
            gs = int(rng.integers(2 ** 31))
            g = {"gid": len(geoms), "side": side, "kind": kind, "geom_seed": gs}
            geoms.append(g)
            reqs.append({"id": k, "t": t, "warm": False, "geom": g["gid"], "side": side,
                         "kind": kind, "geom_seed": gs, "source_seed": gs})
    return reqs

"""Serving-workload inputs evaluated on the GPU with torch (float64).

A serving request names a geometry (kind, side, geometry seed) and a source
seed.  Its parameters are drawn on the host with the same draws, in the same
order, as ``gen.perturbed_circle`` and ``gen.random_sinusoidal``; the node
arrays (coordinates, analytic partials, mask, Dirichlet data, charge
density) are then evaluated on the device, so that a request needs no
host-to-device copy of its arrays.  Up to rounding of the elementary
functions these are the arrays the numpy generators build.  Like the rest of
this package it holds none of the solver's arithmetic.

Request semantics:
  * cold request: geometry and sources from default_rng(geometry seed), as
    ``gen.perturbed_circle(side, seed)`` (8 sources) or
    ``gen.random_sinusoidal(side, seed)`` (4 sources);
  * warm request: the geometry of an earlier request, with sources drawn
    from default_rng(source seed): ``draw_circle_sources`` for a circle,
    ``draw_box_sources`` for a sinusoidal map.
"""

from __future__ import annotations

import math

import numpy as np
import torch

from .gen import (draw_annulus_sources, draw_box_sources, draw_circle, draw_circle_sources,
                  draw_sinusoidal)

SIGMA = 0.02


def _grid(n, device):
    d = 1.0 / (n - 1)
    v = torch.arange(n, dtype=torch.float64, device=device) * d
    ETA, XI = torch.meshgrid(v, v, indexing="ij")  # (ny, nx), XI varies along axis 1
    return XI, ETA, d


ANNULUS_SIGMA = 0.3


def geometry_params(kind, geom_seed):
    """Host-side draws of a cold request: (map parameters, amps, centres)."""
    rng = np.random.default_rng(geom_seed)
    if kind == "annulus":
        amps, centres = draw_annulus_sources(rng, 4)
        return {}, amps, np.asarray(centres)
    if kind == "circle":
        acoef = draw_circle(rng)
        amps, centres = draw_circle_sources(rng, acoef, 8)
        return {"acoef": acoef}, amps, np.asarray(centres)
    amp, amps, centres = draw_sinusoidal(rng, 4, 0.15)
    return {"amp": amp}, amps, np.asarray(centres)


def source_params(kind, map_params, source_seed):
    """Host-side draws of a warm request's sources."""
    rng = np.random.default_rng(source_seed)
    if kind == "annulus":
        amps, centres = draw_annulus_sources(rng, 4)
        return amps, np.asarray(centres)
    if kind == "circle":
        amps, centres = draw_circle_sources(rng, map_params["acoef"], 8)
        return amps, np.asarray(centres)
    amps, centres = draw_box_sources(rng, 4)
    return amps, np.asarray(centres)


def circle_geometry(n, acoef, device, phase=0.0):
    """Perturbed-circle conductor map (see ``gen.perturbed_circle``):
    dict(xp, yp, mask, phi0).  `phase` rotates the perturbation of the
    conductor boundary, R(theta - phase), for a geometry that moves in time;
    phase 0 is the static map."""
    XI, ETA, d = _grid(n, device)
    ux, uy = XI - 0.5, ETA - 0.5
    r = torch.hypot(ux, uy)
    th = torch.atan2(uy, ux)
    R = torch.full_like(th, 0.2)
    for k, a in zip(range(2, 6), acoef):
        R = R + 0.03 * float(a) * torch.cos(k * (th - phase))
    inner = (r >= 0.15) & (r <= 0.2)
    outer = (r > 0.2) & (r <= 0.35)
    rp = torch.where(inner, 0.15 + (r - 0.15) * (R - 0.15) / 0.05, r)
    rp = torch.where(outer, R + (r - 0.2) * (0.35 - R) / 0.15, rp)
    xp = (0.5 + rp * torch.cos(th)).contiguous()
    yp = (0.5 + rp * torch.sin(th)).contiguous()
    cond = r <= 0.2
    return {"xp": xp, "yp": yp, "jac": None, "mask": cond.to(torch.uint8).contiguous(),
            "phi0": cond.to(torch.float64).contiguous()}


def sinusoidal_geometry(n, amp, device):
    """Sinusoidal map with analytic partials (see ``gen.sinusoidal_map``):
    dict(xp, yp, jac, phi0)."""
    XI, ETA, d = _grid(n, device)
    sx, sy = torch.sin(math.pi * XI), torch.sin(math.pi * ETA)
    s = sx * sy
    a = amp * math.pi * torch.cos(math.pi * XI) * sy
    b = amp * math.pi * sx * torch.cos(math.pi * ETA)
    jac = torch.stack([1.0 + a, b, a, 1.0 + b]).contiguous()
    return {"xp": (XI + amp * s).contiguous(), "yp": (ETA + amp * s).contiguous(), "jac": jac,
            "mask": None, "phi0": torch.zeros_like(XI)}


def gaussian_rho(xp, yp, amps, centres, sigma=SIGMA):
    """rho'(x') = sum_m A_m exp(-|x' - c_m|^2 / (2 sigma^2)) on the device.
    The sources are evaluated together, broadcast over a leading source axis
    (in chunks that keep the temporaries near 2^26 elements), so a request
    costs a few launches rather than a few per source; the source constants
    travel in one asynchronous copy from pinned memory (no host wait)."""
    inv = 1.0 / (2.0 * sigma * sigma)
    vals = [[float(A), float(c[0]), float(c[1])] for A, c in zip(amps, centres)]
    rho = torch.zeros_like(xp)
    if not vals:
        return rho
    k = torch.tensor(vals, dtype=torch.float64)
    if xp.is_cuda:
        k = k.pin_memory().to(xp.device, non_blocking=True)
    per = max(1, (1 << 26) // max(xp.numel(), 1))
    for s in range(0, len(vals), per):
        a, cx, cy = (k[s:s + per, q].view(-1, 1, 1) for q in range(3))
        d2 = (xp - cx).square_().add_((yp - cy).square_())
        rho += (a * d2.mul_(-inv).exp_()).sum(0)
    return rho.contiguous()


def semi_annulus_geometry(n, device):
    """The semi-annulus of Section 4.1 (see ``gen.polar_semi_annulus``):
    x' = xi cos eta, y' = xi sin eta on [2, 5] x [0, pi], analytic partials,
    phi = 1 on the arc r = 2 and 0 on r = 5; the straight sides eta = 0, pi
    are Neumann edges (the request carries them)."""
    dx, dy = 3.0 / (n - 1), math.pi / (n - 1)
    xi = 2.0 + dx * torch.arange(n, dtype=torch.float64, device=device)
    eta = dy * torch.arange(n, dtype=torch.float64, device=device)
    ETA, XI = torch.meshgrid(eta, xi, indexing="ij")
    c, s = torch.cos(ETA), torch.sin(ETA)
    jac = torch.stack([c, -XI * s, s, XI * c]).contiguous()
    phi0 = torch.zeros((n, n), dtype=torch.float64, device=device)
    phi0[:, 0] = 1.0
    return {"xp": (XI * c).contiguous(), "yp": (XI * s).contiguous(), "jac": jac,
            "mask": None, "phi0": phi0}


def map_descriptor(kind, map_params, phase=0.0):
    """Parameters of the same maps for a map descriptor of the library
    (keyword arguments of its ``map_desc``): the perturbed circle about
    (1/2, 1/2) with radii 0.15 < 0.2 < 0.35, perturbation 0.03 sum a_k
    cos(k (theta - phase)) and conductor value 1; the sinusoidal map of
    amplitude amp; the polar semi-annulus with value 1 on its inner arc."""
    if kind == "annulus":
        return {"kind": "polar", "value_in": 1.0}
    if kind == "circle":
        return {"kind": "circle", "centre": (0.5, 0.5), "r_in": 0.15, "r_c": 0.2, "r_out": 0.35,
                "pert": 0.03, "coef": [float(a) for a in map_params["acoef"]],
                "phase": float(phase), "value_in": 1.0}
    return {"kind": "sinusoidal", "amp": float(map_params["amp"])}


def source_descriptor(kind, amps, centres):
    """Keyword arguments of the library's ``source_desc`` for drawn sources."""
    return {"amps": [float(a) for a in amps], "centres": [(float(c[0]), float(c[1]))
                                                          for c in centres],
            "sigma": ANNULUS_SIGMA if kind == "annulus" else SIGMA}


def geometry(kind, n, map_params, device):
    if kind == "annulus":
        return semi_annulus_geometry(n, device)
    if kind == "circle":
        return circle_geometry(n, map_params["acoef"], device)
    return sinusoidal_geometry(n, map_params["amp"], device)


def request_fields(desc, device):
    """Fields of a serving request built from a ``gen.serving_stream``
    descriptor: geometry() and source() evaluate the arrays on `device` when
    the server asks for them; map_desc and source_desc give the same request
    as map and source descriptors."""
    kind, n = desc["kind"], desc["side"]
    mp, amps, centres = geometry_params(kind, desc["geom_seed"])
    if desc["warm"]:
        amps, centres = source_params(kind, mp, desc["source_seed"])
    d = 1.0 / (n - 1)

    held = {}

    def geom():
        held["g"] = geometry(kind, n, mp, device)
        return held["g"]

    sigma = ANNULUS_SIGMA if kind == "annulus" else SIGMA

    def source():
        # a cold request asks for the geometry first: reuse its coordinates
        g = held.pop("g", None) or geometry(kind, n, mp, device)
        return gaussian_rho(g["xp"], g["yp"], amps, centres, sigma)

    out = {"rid": desc["id"], "geom": desc["geom"], "nx": n, "ny": n, "dx": d, "dy": d,
           "geometry": geom, "source": source, "warm": desc["warm"], "arrival": desc["t"],
           "map_desc": map_descriptor(kind, mp),
           "source_desc": source_descriptor(kind, amps, centres)}
    if kind == "annulus":  # [2, 5] x [0, pi], Neumann sides eta = 0, pi
        out.update(dx=3.0 / (n - 1), dy=math.pi / (n - 1), xi0=2.0, eta0=0.0, neumann=4 | 8)
    return out

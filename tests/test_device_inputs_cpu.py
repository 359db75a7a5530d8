"""The serving workload's torch generators (workloads.device) build the same
arrays as the numpy generators, evaluated here on the CPU."""

import numpy as np
import torch

import workloads as w
from workloads import device as D


def test_circle_request_matches_numpy_generator():
    q = w.perturbed_circle(129, seed=5)
    mp, amps, centres = D.geometry_params("circle", 5)
    g = D.circle_geometry(129, mp["acoef"], "cpu")
    assert np.allclose(g["xp"].numpy(), q.xp, rtol=0, atol=1e-15)
    assert np.allclose(g["yp"].numpy(), q.yp, rtol=0, atol=1e-15)
    assert np.array_equal(g["mask"].numpy(), q.mask)
    assert np.array_equal(g["phi0"].numpy(), q.phi0)
    rho = D.gaussian_rho(g["xp"], g["yp"], amps, centres)
    assert np.allclose(rho.numpy(), q.rho, rtol=0, atol=1e-14)


def test_sinusoidal_request_matches_numpy_generator():
    q = w.random_sinusoidal(65, 1234)
    mp, amps, centres = D.geometry_params("sinusoidal", 1234)
    g = D.sinusoidal_geometry(65, mp["amp"], "cpu")
    assert np.allclose(g["jac"].numpy(), q.jac, rtol=0, atol=1e-14)
    assert np.allclose(g["xp"].numpy(), q.xp, rtol=0, atol=1e-15)
    rho = D.gaussian_rho(g["xp"], g["yp"], amps, centres)
    assert np.allclose(rho.numpy(), q.rho, rtol=0, atol=1e-14)
    assert not g["phi0"].any()


def test_warm_sources_follow_their_own_seed():
    mp, _, _ = D.geometry_params("circle", 9)
    a1, c1 = D.source_params("circle", mp, 77)
    a2, c2 = D.source_params("circle", mp, 77)
    assert np.array_equal(a1, a2) and np.array_equal(c1, c2)
    # centres lie outside the physical conductor
    for cx, cy in c1:
        th = np.arctan2(cy - 0.5, cx - 0.5)
        R = 0.2 + 0.03 * sum(a * np.cos(k * th) for k, a in zip(range(2, 6), mp["acoef"]))
        assert np.hypot(cx - 0.5, cy - 0.5) > R
    a3, c3 = D.source_params("sinusoidal", {"amp": 0.1}, 5)
    assert len(a3) == 4 and np.all((c3 >= 0.1) & (c3 <= 0.9))

"""Setup from map and source descriptors (tomg_setup_coeffs_desc,
tomg_update_rhs_desc): the device evaluates the map, its Jacobian (analytic,
or by the differences of eq. 39-42 for the perturbed circle), the Gaussian
charge density and the Dirichlet set node by node.  Checked against the
oracle on the same maps built on the host (coefficients and solution), and
against the array setup of the same request."""

import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_01888_amd as tomg
    from workloads import device as D
    return torch, tomg, D


def host_problem(kind, n, seed):
    """The request's host arrays (the generator the oracle reads)."""
    if kind == "circle":
        return w.perturbed_circle(n, seed)
    if kind == "sinusoidal":
        return w.random_sinusoidal(n, seed)
    from workloads import device as D
    q = w.polar_semi_annulus(n, neumann=True)
    mp, amps, centres = D.geometry_params("annulus", seed)
    q.rho = w.gaussian_sources(q.xp, q.yp, amps, centres, D.ANNULUS_SIGMA)
    return q


def descriptors(tomg, D, kind, seed):
    mp, amps, centres = D.geometry_params("annulus" if kind == "polar" else kind, seed)
    k = "annulus" if kind == "polar" else kind
    return (tomg.map_desc(**D.map_descriptor(k, mp)),
            tomg.source_desc(**D.source_descriptor(k, amps, centres)))


def make_problem(tomg, q, **kw):
    return tomg.Problem(q.nx, q.ny, q.dx, q.dy, q.xi0, q.eta0,
                        neumann=getattr(q, "neumann", 0), **kw)


CASES = [("circle", 129, 3), ("circle", 257, 11), ("sinusoidal", 129, 4),
         ("sinusoidal", 193, 9), ("polar", 129, 2)]


@pytest.mark.parametrize("kind,n,seed", CASES)
def test_desc_setup_matches_oracle(env, kind, n, seed):
    torch, tomg, D = env
    print(f"[desc] setup {kind} n={n} seed={seed}", flush=True)
    q = host_problem(kind, n, seed)
    if kind == "polar":
        assert q.neumann == (tomg.TOMG_NEU_S | tomg.TOMG_NEU_N)
    m, s = descriptors(tomg, D, kind, seed)
    p = make_problem(tomg, q)
    phi = torch.full((q.ny, q.nx), 7.0, dtype=torch.float64, device="cuda")
    p.setup_desc(m, s, phi_init=phi)
    ref = oracle.setup(q)
    # the Dirichlet set and its values are exact
    assert np.array_equal(p.export("dir").cpu().numpy(), ref["dir"])
    # (the host generator takes the outer arc's value from ln(R/r), which
    # rounds to a few 1e-16 at r = R)
    assert np.abs(phi.cpu().numpy() - q.phi0).max() <= 1e-15
    # coefficients: analytic maps to rounding, the numeric Jacobian of the
    # circle to the rounding of its node coordinates amplified by 1/(2h)
    tol = 1e-14 if kind != "circle" else 1e-12
    tensor_scale = max(np.abs(ref["exx"]).max(), np.abs(ref["eyy"]).max())
    for name in ("exx", "exy", "eyy", "det"):
        got = p.export(name).cpu().numpy()
        # (the off-diagonal entry is rounding noise for an orthogonal map:
        # measured against the size of the tensor)
        scale = np.abs(ref[name]).max() if name == "det" else tensor_scale
        err = np.abs(got - ref[name]).max() / scale
        print(f"[desc]   {name} rel err {err:.2e}", flush=True)
        assert err < tol, (name, err)
    f = p.export("rhs").cpu().numpy()
    assert np.abs(f - ref["f"]).max() <= 1e-11 * np.abs(ref["f"]).max() + 1e-300
    # the solution against the oracle's on its own arrays
    r = p.solve(phi, rel_tol=1e-12, max_cycles=100)
    assert r.ok, r
    ro = oracle.solve_problem(q, rel_tol=1e-12)
    ph = ro["phi"]
    err = np.abs(phi.cpu().numpy() - ph).max() / max(np.abs(ph).max(), 1.0)
    print(f"[desc]   solution rel err {err:.2e} ({r.cycles} cycles)", flush=True)
    assert err < 1e-11


@pytest.mark.parametrize("kind", ["circle", "sinusoidal", "polar"])
def test_desc_matches_array_setup(env, kind):
    """Descriptor setup and the array setup of the device-built request give
    the same solve (cycles and solution)."""
    torch, tomg, D = env
    n, seed = 257, 21
    print(f"[desc] vs arrays {kind}", flush=True)
    k = "annulus" if kind == "polar" else kind
    mp, amps, centres = D.geometry_params(k, seed)
    g = D.geometry(k, n, mp, "cuda")
    rho = D.gaussian_rho(g["xp"], g["yp"], amps, centres,
                         D.ANNULUS_SIGMA if k == "annulus" else D.SIGMA)
    if kind == "polar":  # [2, 5] x [0, pi], Neumann sides eta = 0, pi
        dx, dy = 3.0 / (n - 1), np.pi / (n - 1)
        kw = dict(xi0=2.0, neumann=tomg.TOMG_NEU_S | tomg.TOMG_NEU_N)
    else:
        dx = dy = 1.0 / (n - 1)
        kw = {}
    pa = tomg.Problem(n, n, dx, dy, **kw)
    pd = tomg.Problem(n, n, dx, dy, **kw)
    pa.setup_coeffs(rho, xp=g["xp"], yp=g["yp"], jac=g["jac"], mask=g["mask"])
    m, s = descriptors(tomg, D, kind, seed)
    phd = torch.empty_like(rho)
    pd.setup_desc(m, s, phi_init=phd)
    pha = g["phi0"].clone()
    assert torch.equal(pha, phd)
    ra = pa.solve(pha, rel_tol=1e-11)
    rd = pd.solve(phd, rel_tol=1e-11)
    assert ra.ok and rd.ok
    assert abs(ra.cycles - rd.cycles) <= 1
    err = (pha - phd).abs().max().item() / max(pha.abs().max().item(), 1.0)
    print(f"[desc]   {kind}: cycles {ra.cycles}/{rd.cycles}, rel diff {err:.2e}", flush=True)
    assert err < 1e-11


def test_update_rhs_desc(env):
    """A new source on the stored map: the right-hand side equals that of the
    array update on the same map."""
    torch, tomg, D = env
    n = 129
    d = 1.0 / (n - 1)
    mp, amps, centres = D.geometry_params("circle", 5)
    m = tomg.map_desc(**D.map_descriptor("circle", mp))
    s0 = tomg.source_desc(**D.source_descriptor("circle", amps, centres))
    amps2, centres2 = D.source_params("circle", mp, 99)
    s1 = tomg.source_desc(**D.source_descriptor("circle", amps2, centres2))
    p = tomg.Problem(n, n, d, d)
    phi = torch.empty((n, n), dtype=torch.float64, device="cuda")
    p.setup_desc(m, s0, phi_init=phi)
    p.update_rhs_desc(s1)
    f_desc = p.export("rhs")
    g = D.circle_geometry(n, mp["acoef"], "cuda")
    rho2 = D.gaussian_rho(g["xp"], g["yp"], amps2, centres2)
    p.update_rhs(rho2)
    f_arr = p.export("rhs")
    err = (f_desc - f_arr).abs().max().item() / f_arr.abs().max().item()
    assert err < 1e-12, err
    r = p.solve(phi, rel_tol=1e-10)
    assert r.ok


def test_desc_errors(env):
    torch, tomg, D = env
    n = 65
    d = 1.0 / (n - 1)
    p = tomg.Problem(n, n, d, d)
    s = tomg.source_desc([1.0], [(0.3, 0.3)], 0.05)
    # update before any setup, and after an array setup
    with pytest.raises(tomg.TomgError) as e:
        p.update_rhs_desc(s)
    assert e.value.status == tomg.TOMG_ESTATE
    q = w.random_sinusoidal(n, 1)
    dev = tomg.upload(q)
    p.setup_coeffs(dev["rho"], xp=dev["xp"], yp=dev["yp"], jac=dev["jac"])
    with pytest.raises(tomg.TomgError) as e:
        p.update_rhs_desc(s)
    assert e.value.status == tomg.TOMG_ESTATE
    bad = [tomg.map_desc("circle", r_in=0.2, r_c=0.2, r_out=0.35)]
    m = tomg.map_desc("sinusoidal", amp=0.1)
    m.kind = 7
    bad.append(m)
    for m in bad:
        with pytest.raises(tomg.TomgError) as e:
            p.setup_desc(m, s)
        assert e.value.status == tomg.TOMG_EINVAL
    m = tomg.map_desc("sinusoidal", amp=0.1)
    for count, sigma in ((17, 0.05), (-1, 0.05), (1, 0.0)):
        sb = tomg.source_desc([1.0], [(0.3, 0.3)], 0.05)
        sb.count, sb.sigma = count, sigma
        with pytest.raises(tomg.TomgError) as e:
            p.setup_desc(m, sb)
        assert e.value.status == tomg.TOMG_EINVAL
    # a folded sinusoidal map (|amp| pi > 1/2 folds it) fails the geometry check
    with pytest.raises(tomg.TomgError) as e:
        p.setup_desc(tomg.map_desc("sinusoidal", amp=0.5), s)
    assert e.value.status == tomg.TOMG_EGEOMETRY
    # and a good one after it works
    phi = torch.empty((n, n), dtype=torch.float64, device="cuda")
    p.setup_desc(m, s, phi_init=phi)
    assert p.solve(phi, rel_tol=1e-10).ok


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_async_desc_batch(env, precision):
    """Asynchronous descriptor setups of several problems solved as one batch
    (the coarsest inverses run batched in the first step) match the
    synchronous setups solved one by one."""
    torch, tomg, D = env
    print(f"[desc] async batch {precision}", flush=True)
    reqs = [("circle", 129, 1), ("sinusoidal", 257, 2), ("circle", 65, 3),
            ("sinusoidal", 129, 4), ("polar", 129, 5)]
    probs, phis, refs = [], [], []
    for kind, n, seed in reqs:
        q = host_problem(kind, n, seed)
        m, s = descriptors(tomg, D, kind, seed)
        pa = make_problem(tomg, q, precision=precision)
        phi = torch.empty((n, n), dtype=torch.float64, device="cuda")
        pa.setup_desc(m, s, phi_init=phi, check=False)
        probs.append(pa)
        phis.append(phi)
        pr = make_problem(tomg, q, precision=precision)
        ph = torch.empty_like(phi)
        pr.setup_desc(m, s, phi_init=ph)
        assert pr.solve(ph, rel_tol=1e-11).ok
        refs.append(ph)
    res = tomg.solve_batch(probs, phis, rel_tol=1e-11)
    for r, phi, ref in zip(res, phis, refs):
        assert r.ok, r
        err = (phi - ref).abs().max().item() / max(ref.abs().max().item(), 1.0)
        assert err < 1e-9, err


def test_async_desc_setup_reports_a_folded_map_later(env):
    """A descriptor setup queued without the host check (TOMG_SETUP_ASYNC):
    a folded map is reported by setup_check, and the problem works again
    after a good setup."""
    torch, tomg, D = env
    n = 129
    d = 1.0 / (n - 1)
    p = tomg.Problem(n, n, d, d)
    s = tomg.source_desc([1.0], [(0.4, 0.6)], 0.05)
    phi = torch.empty((n, n), dtype=torch.float64, device="cuda")
    p.setup_desc(tomg.map_desc("sinusoidal", amp=0.5), s, phi_init=phi, check=False)
    with pytest.raises(tomg.TomgError) as e:
        p.setup_check()
    assert e.value.status == tomg.TOMG_EGEOMETRY
    p.setup_desc(tomg.map_desc("sinusoidal", amp=0.1), s, phi_init=phi, check=False)
    p.setup_check()
    assert p.solve(phi, rel_tol=1e-10).ok

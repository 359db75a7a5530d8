"""ctypes wrapper of the C oracle (test infrastructure only).

Every function takes and returns numpy float64 arrays of shape (ny, nx)
(stencils: (9, ny, nx)); see ``tomg_oracle.h`` for the conventions and the
paper passages each step follows."""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

GS4, GS_LEX, JACOBI, ZEBRA_X, ZEBRA_XY = 0, 1, 2, 3, 4
# coarse-grid operators: Galerkin product, or eq. 18 rediscretised per level
GALERKIN, REDISCRETIZE = 0, 1
# edges with a homogeneous Neumann condition (bit mask)
NEU_W, NEU_E, NEU_S, NEU_N = 1, 2, 4, 8

_lib = None
_D = C.POINTER(C.c_double)
_U8 = C.POINTER(C.c_uint8)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.ensure_built()
    lib = C.CDLL(path)
    sz, i, d, p = C.c_size_t, C.c_int, C.c_double, C.c_void_p
    sig = {
        "orc_num_threads": (i, []),
        "orc_set_threads": (None, [i]),
        "orc_jacobian_numeric": (i, [i, i, d, d, _D, _D, _D, _D, _D, _D]),
        "orc_field": (None, [i, i, d, d, _D, _D, _D, _D, _D, _D, _D]),
        "orc_permittivity": (None, [sz, _D, _D, _D, _D, _D, _D, _D, _D, _D]),
        "orc_geometry_ok": (i, [i, i, _D]),
        "orc_rhs": (None, [sz, _D, _D, _D]),
        "orc_dirichlet_set": (None, [i, i, _U8, _U8]),
        "orc_dirichlet_set_bc": (None, [i, i, _U8, i, _U8]),
        "orc_fine_stencil": (None, [i, i, d, d, _D, _D, _D, _U8, _D]),
        "orc_flux_stencil": (None, [i, i, d, d, _D, _D, _D, _U8, _D]),
        "orc_apply": (None, [i, i, _D, _U8, _D, _D]),
        "orc_residual": (None, [i, i, _D, _U8, _D, _D, _D]),
        "orc_norm2_free": (d, [i, i, _U8, _D]),
        "orc_smooth": (None, [i, i, _D, _U8, _D, _D, i, i, d]),
        "orc_restrict_fw": (None, [i, i, _D, i, i, _D]),
        "orc_restrict_fw_bc": (None, [i, i, _D, i, i, _U8, _D]),
        "orc_prolong_add": (None, [i, i, _D, i, i, _U8, _D]),
        "orc_galerkin": (None, [i, i, _D, _U8, i, i, _D, _U8]),
        "orc_restrict_s": (None, [i, i, _D, i, i, i, i, _U8, _D]),
        "orc_prolong_add_s": (None, [i, i, _D, i, i, i, i, _U8, _D]),
        "orc_galerkin_s": (None, [i, i, _D, _U8, i, i, i, i, _D, _U8]),
        "orc_levels_semi": (i, [i, i, i, i, C.POINTER(i), C.POINTER(i), C.POINTER(i),
                                C.POINTER(i), i, i]),
        "orc_mg_create_semi": (p, [i, i, d, d, _D, _D, _D, _U8, i, i, i, i, i, i, i, i, d]),
        "orc_mg_level_strides": (None, [p, i, C.POINTER(i), C.POINTER(i)]),
        "orc_dense_solve": (i, [i, _D, _D]),
        "orc_levels": (i, [i, i, C.POINTER(i), C.POINTER(i), i]),
        "orc_levels_lim": (i, [i, i, C.POINTER(i), C.POINTER(i), i, i]),
        "orc_mg_create": (p, [i, i, d, d, _D, _D, _D, _U8, i, i, i, d]),
        "orc_mg_create_bc": (p, [i, i, d, d, _D, _D, _D, _U8, i, i, i, i, d]),
        "orc_mg_create_op": (p, [i, i, d, d, _D, _D, _D, _U8, i, i, i, i, i, d]),
        "orc_mg_create_full": (p, [i, i, d, d, _D, _D, _D, _U8, i, i, i, i, i, i, d]),
        "orc_mg_destroy": (None, [p]),
        "orc_mg_num_levels": (i, [p]),
        "orc_mg_level_shape": (None, [p, i, C.POINTER(i), C.POINTER(i)]),
        "orc_mg_stencil": (_D, [p, i]),
        "orc_mg_dir": (_U8, [p, i]),
        "orc_mg_level_rhs": (_D, [p, i]),
        "orc_mg_level_x": (_D, [p, i]),
        "orc_mg_vcycle": (None, [p, _D, _D]),
        "orc_mg_initial_residual": (d, [p, _D, _D]),
        "orc_mg_solve": (i, [p, _D, _D, d, i, C.POINTER(i), C.POINTER(d), _D, i]),
        "orc_error_norms": (None, [sz, _D, _D, _D]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _u8(a):
    if a is None:
        return None
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(_U8)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return _load().orc_num_threads()


def set_threads(n: int) -> None:
    """OpenMP threads of the calling host thread's later oracle calls."""
    _load().orc_set_threads(int(n))


# ---------------------------------------------------------------- setup ----

def jacobian_numeric(xp, yp, dx, dy):
    xp, yp = _f64(xp), _f64(yp)
    ny, nx = xp.shape
    J = np.empty((4, ny, nx))
    rc = _load().orc_jacobian_numeric(nx, ny, dx, dy, _d(xp), _d(yp), _d(J[0]), _d(J[1]),
                                      _d(J[2]), _d(J[3]))
    if rc != 0:
        raise ValueError("grid too small for the numeric Jacobian")
    return J


def field(phi, jac, dx, dy):
    """Physical electric field E' = (J^T)^-1 (-grad phi) at every node (eq. 2);
    grad phi by the differences of eq. 39-42 (one-sided on the edges).
    Returns (Ex', Ey')."""
    phi, jac = _f64(phi), _f64(jac)
    ny, nx = phi.shape
    ex, ey = np.empty_like(phi), np.empty_like(phi)
    _load().orc_field(nx, ny, dx, dy, _d(phi), _d(jac[0]), _d(jac[1]), _d(jac[2]), _d(jac[3]),
                      _d(ex), _d(ey))
    return ex, ey


def permittivity(jac, eps_phys=None):
    jac = _f64(jac)
    _, ny, nx = jac.shape
    out = np.empty((4, ny, nx))
    ep = None if eps_phys is None else _f64(eps_phys)
    _load().orc_permittivity(nx * ny, _d(jac[0]), _d(jac[1]), _d(jac[2]), _d(jac[3]), _d(ep),
                             _d(out[0]), _d(out[1]), _d(out[2]), _d(out[3]))
    return out[0], out[1], out[2], out[3]


def geometry_ok(det) -> bool:
    det = _f64(det)
    ny, nx = det.shape
    return bool(_load().orc_geometry_ok(nx, ny, _d(det)))


def rhs(rho, det):
    rho, det = _f64(rho), _f64(det)
    f = np.empty_like(rho)
    _load().orc_rhs(rho.size, _d(rho), _d(det), _d(f))
    return f


def dirichlet_set(nx, ny, mask=None, neumann=0):
    """Dirichlet flags: the outer ring except the edges in `neumann` (NEU_*
    bits, zero normal derivative), plus the mask."""
    d = np.empty((ny, nx), dtype=np.uint8)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    _load().orc_dirichlet_set_bc(nx, ny, _u8(m), int(neumann), _u8(d))
    return d


def fine_stencil(exx, exy, eyy, dx, dy, dirs):
    exx, exy, eyy = _f64(exx), _f64(exy), _f64(eyy)
    ny, nx = exx.shape
    st = np.empty((9, ny, nx))
    _load().orc_fine_stencil(nx, ny, dx, dy, _d(exx), _d(exy), _d(eyy), _u8(dirs), _d(st))
    return st


def flux_stencil(exx, exy, eyy, dx, dy, dirs):
    """The symmetric flux (energy) form of the operator as a 9-point stencil."""
    exx, exy, eyy = _f64(exx), _f64(exy), _f64(eyy)
    ny, nx = exx.shape
    st = np.empty((9, ny, nx))
    _load().orc_flux_stencil(nx, ny, dx, dy, _d(exx), _d(exy), _d(eyy), _u8(dirs), _d(st))
    return st


def setup(prob, eps_phys=None):
    """Setup of a ``workloads.GridProblem``: Jacobian (analytic partials when
    the problem carries them, else eq. 39-42 from the node coordinates),
    permittivity, det J, right-hand side and Dirichlet set."""
    if prob.jac is not None:
        J = _f64(prob.jac)
    else:
        J = jacobian_numeric(prob.xp, prob.yp, prob.dx, prob.dy)
    exx, exy, eyy, det = permittivity(J, eps_phys)
    f = rhs(prob.rho, det)
    neumann = getattr(prob, "neumann", 0)
    dirs = dirichlet_set(prob.nx, prob.ny, prob.mask, neumann)
    return {"jac": J, "exx": exx, "exy": exy, "eyy": eyy, "det": det, "f": f, "dir": dirs,
            "geometry_ok": geometry_ok(det), "neumann": neumann}


# ------------------------------------------------------------- operator ----

def apply(st, dirs, x):
    x = _f64(x)
    ny, nx = x.shape
    y = np.empty_like(x)
    _load().orc_apply(nx, ny, _d(_f64(st)), _u8(dirs), _d(x), _d(y))
    return y


def residual(st, dirs, x, b):
    x, b = _f64(x), _f64(b)
    ny, nx = x.shape
    r = np.empty_like(x)
    _load().orc_residual(nx, ny, _d(_f64(st)), _u8(dirs), _d(x), _d(b), _d(r))
    return r


def norm2_free(dirs, r):
    r = _f64(r)
    ny, nx = r.shape
    return _load().orc_norm2_free(nx, ny, _u8(dirs), _d(r))


def smooth(st, dirs, x, b, kind=GS4, sweeps=1, omega=0.8):
    """Returns a smoothed copy of x."""
    x = _f64(x).copy()
    b = _f64(b)
    ny, nx = x.shape
    _load().orc_smooth(nx, ny, _d(_f64(st)), _u8(dirs), _d(x), _d(b), kind, sweeps, omega)
    return x


def restrict_fw(rf, nxc, nyc):
    rf = _f64(rf)
    nyf, nxf = rf.shape
    fc = np.empty((nyc, nxc))
    _load().orc_restrict_fw(nxf, nyf, _d(rf), nxc, nyc, _d(fc))
    return fc


def restrict_fw_bc(rf, dirc):
    """Full weighting where the coarse ring may hold free (Neumann) nodes."""
    rf = _f64(rf)
    nyf, nxf = rf.shape
    nyc, nxc = dirc.shape
    fc = np.empty((nyc, nxc))
    _load().orc_restrict_fw_bc(nxf, nyf, _d(rf), nxc, nyc, _u8(np.ascontiguousarray(dirc)),
                               _d(fc))
    return fc


def prolong_add(ec, xf, dirf):
    ec = _f64(ec)
    xf = _f64(xf).copy()
    nyc, nxc = ec.shape
    nyf, nxf = xf.shape
    _load().orc_prolong_add(nxc, nyc, _d(ec), nxf, nyf, _u8(dirf), _d(xf))
    return xf


def galerkin(stf, dirf, nxc, nyc):
    stf = _f64(stf)
    _, nyf, nxf = stf.shape
    stc = np.empty((9, nyc, nxc))
    dirc = np.empty((nyc, nxc), dtype=np.uint8)
    _load().orc_galerkin(nxf, nyf, _d(stf), _u8(dirf), nxc, nyc, _d(stc), _u8(dirc))
    return stc, dirc


def coarse_shape(nxf, nyf, sx, sy):
    """Coarse grid of a transfer with strides (sx, sy): a halved axis (stride
    2) keeps every other node, a kept axis (stride 1) every node."""
    return ((nxf - 1) // 2 + 1 if sx == 2 else nxf, (nyf - 1) // 2 + 1 if sy == 2 else nyf)


def restrict_s(rf, sx, sy, dirc=None):
    """Restriction P^T / (sx sy) with per-axis strides (semi-coarsening when
    one of them is 1); dirc None gives zero on the whole coarse ring."""
    rf = _f64(rf)
    nyf, nxf = rf.shape
    nxc, nyc = coarse_shape(nxf, nyf, sx, sy)
    fc = np.empty((nyc, nxc))
    dc = None if dirc is None else np.ascontiguousarray(dirc, dtype=np.uint8)
    _load().orc_restrict_s(nxf, nyf, _d(rf), nxc, nyc, sx, sy, _u8(dc), _d(fc))
    return fc


def prolong_add_s(ec, xf, dirf, sx, sy):
    ec = _f64(ec)
    xf = _f64(xf).copy()
    nyc, nxc = ec.shape
    nyf, nxf = xf.shape
    _load().orc_prolong_add_s(nxc, nyc, _d(ec), nxf, nyf, sx, sy, _u8(dirf), _d(xf))
    return xf


def galerkin_s(stf, dirf, sx, sy):
    """(1 / (sx sy)) P^T A P with per-axis strides; returns (stencil, flags)."""
    stf = _f64(stf)
    _, nyf, nxf = stf.shape
    nxc, nyc = coarse_shape(nxf, nyf, sx, sy)
    stc = np.empty((9, nyc, nxc))
    dirc = np.empty((nyc, nxc), dtype=np.uint8)
    _load().orc_galerkin_s(nxf, nyf, _d(stf), _u8(dirf), nxc, nyc, sx, sy, _d(stc), _u8(dirc))
    return stc, dirc


def dense_solve(A, b):
    A = _f64(A).copy()
    b = _f64(b).copy()
    rc = _load().orc_dense_solve(b.size, _d(A), _d(b))
    if rc != 0:
        raise np.linalg.LinAlgError("zero pivot")
    return b


def levels(nx, ny, maxl=16, neumann=0, semi=0, semi_axis=0):
    """Level shapes; with Neumann edges the coarsest is at most 5 x 5 where
    halving reaches it, else at most 1024 nodes (the 201 x 201 family stops
    at 26 x 26).  semi: the first coarsenings halve axis semi_axis only."""
    a = (C.c_int * maxl)()
    b = (C.c_int * maxl)()
    if semi:
        L = _load().orc_levels_semi(nx, ny, semi, semi_axis, a, b, None, None, maxl,
                                    5 if neumann else 9)
    else:
        L = _load().orc_levels_lim(nx, ny, a, b, maxl, 5 if neumann else 9)
    return [(a[k], b[k]) for k in range(L)]


def error_norms(a, b):
    """(L_inf, L_2, L_1) of eq. 25-27 over all nodes."""
    a, b = _f64(a), _f64(b)
    out = np.empty(3)
    _load().orc_error_norms(a.size, _d(a), _d(b), _d(out))
    return tuple(float(v) for v in out)


# ------------------------------------------------------------ multigrid ----

class MG:
    """Oracle multigrid hierarchy (V(nu1, nu2), direct coarsest solve).
    smoother: GS4 (the GPU's ordering, "mirror mode"), GS_LEX (the paper's
    lexicographic ordering), JACOBI or ZEBRA_X (x-line Gauss-Seidel, even
    rows then odd rows).  coarse_op: GALERKIN (default) or REDISCRETIZE
    (eq. 18 on each coarse grid with the tensor sampled there; Dirichlet
    edges and the eq. 18 form only)."""

    def __init__(self, exx, exy, eyy, dx, dy, mask=None, nu1=2, nu2=2, smoother=GS4,
                 omega=0.8, neumann=0, flux=False, coarse_op=GALERKIN, semi=0, semi_axis=0):
        self._keep = [_f64(exx), _f64(exy), _f64(eyy)]
        ny, nx = self._keep[0].shape
        m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        self.nx, self.ny = nx, ny
        self._h = _load().orc_mg_create_semi(nx, ny, dx, dy, _d(self._keep[0]),
                                             _d(self._keep[1]), _d(self._keep[2]), _u8(m),
                                             int(neumann), 1 if flux else 0, int(coarse_op),
                                             int(semi), int(semi_axis), nu1, nu2, smoother,
                                             omega)
        if not self._h:
            raise ValueError(f"grid {nx}x{ny}: does not coarsen to <= 9x9 nodes, or the "
                             f"coarse operator does not apply to this problem")

    @classmethod
    def from_setup(cls, s, dx, dy, mask=None, **kw):
        kw.setdefault("neumann", s.get("neumann", 0))
        return cls(s["exx"], s["exy"], s["eyy"], dx, dy, mask=mask, **kw)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().orc_mg_destroy(h)
            self._h = None

    @property
    def num_levels(self):
        return _load().orc_mg_num_levels(self._h)

    def shape(self, l):
        a, b = C.c_int(), C.c_int()
        _load().orc_mg_level_shape(self._h, l, C.byref(a), C.byref(b))
        return a.value, b.value

    def strides(self, l):
        """Strides (sx, sy) of the transfer from level l to level l + 1."""
        a, b = C.c_int(), C.c_int()
        _load().orc_mg_level_strides(self._h, l, C.byref(a), C.byref(b))
        return a.value, b.value

    def _view(self, ptr, shape, dtype):
        n = int(np.prod(shape))
        if dtype == np.uint8:
            arr = np.ctypeslib.as_array(ptr, shape=(n,))
        else:
            arr = np.ctypeslib.as_array(ptr, shape=(n,))
        return arr.reshape(shape).copy()

    def stencil(self, l):
        nx, ny = self.shape(l)
        return self._view(_load().orc_mg_stencil(self._h, l), (9, ny, nx), np.float64)

    def dirs(self, l):
        nx, ny = self.shape(l)
        return self._view(_load().orc_mg_dir(self._h, l), (ny, nx), np.uint8)

    def level_rhs(self, l):
        nx, ny = self.shape(l)
        return self._view(_load().orc_mg_level_rhs(self._h, l), (ny, nx), np.float64)

    def level_x(self, l):
        nx, ny = self.shape(l)
        return self._view(_load().orc_mg_level_x(self._h, l), (ny, nx), np.float64)

    def vcycle(self, phi, f):
        phi = _f64(phi).copy()
        _load().orc_mg_vcycle(self._h, _d(phi), _d(_f64(f)))
        return phi

    def initial_residual(self, phi, f):
        phi = _f64(phi).copy()
        return _load().orc_mg_initial_residual(self._h, _d(phi), _d(_f64(f)))

    def solve(self, phi, f, rel_tol=1e-10, max_cycles=100, hist_len=0):
        """Returns (phi, status, cycles, rel, history).  status 0 converged,
        1 max_cycles reached, 2 non-finite residual."""
        phi = _f64(phi).copy()
        cyc, rel = C.c_int(), C.c_double()
        hist = np.zeros(max(hist_len, 1))
        st = _load().orc_mg_solve(self._h, _d(phi), _d(_f64(f)), rel_tol, max_cycles,
                                  C.byref(cyc), C.byref(rel), _d(hist), hist_len)
        return phi, st, cyc.value, rel.value, hist[:min(hist_len, cyc.value + 1)]


def generate_grid(xb, yb, dx, dy, rel_tol=1e-13, max_cycles=200, mask=None, px=None, py=None):
    """Numerical grid generation (Section 4.2, eq. 36-37): x'(xi, eta) and
    y'(xi, eta) solve Laplace's equation on the computational grid with the
    boundary map as Dirichlet data.  The operator is this oracle's eq. 18 with
    the identity tensor (the 5-point Laplacian), solved by its multigrid.
    xb, yb: node arrays carrying the boundary values on the outer ring and,
    where mask is 1, inside the grid (an embedded body's outline, Section
    5.2).  px, py: source terms (the adaptive grids of the conclusion: lap x' =
    px, lap y' = py on the computational grid); None means zero.  Returns
    (xp, yp)."""
    xb, yb = _f64(xb), _f64(yb)
    ny, nx = xb.shape
    one, zero = np.ones((ny, nx)), np.zeros((ny, nx))
    mg = MG(one, zero, one, dx, dy, mask=mask)
    fixed = np.zeros((ny, nx), dtype=bool)
    fixed[0, :] = fixed[-1, :] = fixed[:, 0] = fixed[:, -1] = True
    if mask is not None:
        fixed |= np.asarray(mask).astype(bool)
    out = []
    for b0, src in ((xb, px), (yb, py)):
        rhs_g = zero if src is None else _f64(src)
        start = np.where(fixed, b0, 0.0)
        phi, status, _, rel, _ = mg.solve(start, rhs_g, rel_tol, max_cycles)
        if status == 2:
            raise FloatingPointError("grid generation diverged")
        out.append(phi)
    return out[0], out[1]


def solve_problem(prob, rel_tol=1e-10, max_cycles=200, smoother=GS4, nu1=2, nu2=2,
                  eps_phys=None, hist_len=0, flux=False, coarse_op=GALERKIN, semi=0,
                  semi_axis=0):
    """Setup plus multigrid solve of a ``workloads.GridProblem`` from its
    ``phi0``.  Returns a dict with phi, cycles, rel, status and the setup."""
    s = setup(prob, eps_phys)
    mg = MG.from_setup(s, prob.dx, prob.dy, mask=prob.mask, nu1=nu1, nu2=nu2,
                       smoother=smoother, flux=flux, coarse_op=coarse_op, semi=semi,
                       semi_axis=semi_axis)
    phi, status, cycles, rel, hist = mg.solve(prob.phi0, s["f"], rel_tol, max_cycles, hist_len)
    return {"phi": phi, "status": status, "cycles": cycles, "rel": rel, "hist": hist,
            "setup": s, "mg": mg}


__all__ = [n for n in dir() if not n.startswith("_")]

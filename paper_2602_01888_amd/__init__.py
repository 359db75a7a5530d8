"""tomg: geometric multigrid for the coordinate-transformed Poisson equation
(arXiv 2602.01888) on AMD Instinct MI355X.

Python binding of ``libtomg.so`` (``include/tomg.h``).  Tensors are torch
tensors on the GPU; the workspace is a torch uint8 tensor, so PyTorch's
caching allocator owns all device memory.  Names follow the C-ABI:
``setup_coeffs``, ``vcycle``, ``solve``, ``residual_norm`` (methods of
``Problem`` and module functions taking a ``Problem``)."""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional, Sequence

import torch  # noqa: F401  (binds the HIP runtime before the library loads)

from . import _lib
from ._lib import (FIELD, STATUS_NAMES, TOMG_EGEOMETRY, TOMG_EINVAL, TOMG_ENOCONV,  # noqa: F401
                   TOMG_ENOMEM, TOMG_ENONFINITE, TOMG_ESTATE, TOMG_FP32_IR, TOMG_FP64,
                   TOMG_GS4, TOMG_JACOBI, TOMG_ZEBRA_X, TOMG_ZEBRA_XY, TOMG_NEU_E, TOMG_NEU_N,
                   TOMG_NEU_S, TOMG_NEU_W, TOMG_GALERKIN, TOMG_REDISCRETIZE, TOMG_OK, Config,
                   TOMG_MAP_PERTURBED_CIRCLE, TOMG_MAP_POLAR, TOMG_MAP_SINUSOIDAL,
                   TOMG_MAX_GAUSSIANS, MapDesc, SourceDesc)


class TomgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def make_config(nx, ny, dx, dy, xi0=0.0, eta0=0.0, precision="fp64", nu1=2, nu2=2,
                smoother="gs4", jacobi_omega=0.8, ir_inner_cycles=2, neumann=0,
                flux=False, coarse_op="galerkin", semi_levels=0, semi_axis="x") -> Config:
    lib = _lib.load()
    cfg = Config()
    lib.tomg_config_default(C.byref(cfg), nx, ny, dx, dy)
    cfg.xi0, cfg.eta0 = xi0, eta0
    cfg.precision = {"fp64": TOMG_FP64, "fp32_ir": TOMG_FP32_IR, "mixed": TOMG_FP32_IR}[precision]
    cfg.nu1, cfg.nu2 = nu1, nu2
    cfg.smoother = {"gs4": TOMG_GS4, "jacobi": TOMG_JACOBI, "zebra_x": TOMG_ZEBRA_X,
                    "zebra_xy": TOMG_ZEBRA_XY}[smoother]
    cfg.jacobi_omega = jacobi_omega
    cfg.ir_inner_cycles = ir_inner_cycles
    cfg.neumann = int(neumann)
    cfg.flux = 1 if flux else 0
    cfg.coarse_op = {"galerkin": TOMG_GALERKIN, "rediscretize": TOMG_REDISCRETIZE}[coarse_op]
    cfg.semi_levels = int(semi_levels)
    cfg.semi_axis = {"x": 0, "y": 1, 0: 0, 1: 1}[semi_axis]
    return cfg


def workspace_bytes(cfg: Config) -> int:
    return int(_lib.load().tomg_workspace_bytes(C.byref(cfg)))


def num_levels(cfg: Config) -> int:
    return int(_lib.load().tomg_num_levels(C.byref(cfg)))


def _ptr(t: Optional[torch.Tensor], dtype, shape=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


@dataclass
class SolveResult:
    status: int
    cycles: int
    rel: float

    @property
    def ok(self):
        return self.status == TOMG_OK


class Problem:
    """One grid problem: a caller-sized workspace on the current device and a
    library handle bound to a stream (default: the current torch stream)."""

    def __init__(self, nx, ny, dx, dy, xi0=0.0, eta0=0.0, precision="fp64", nu1=2, nu2=2,
                 smoother="gs4", jacobi_omega=0.8, ir_inner_cycles=2, device=None,
                 stream: Optional[torch.cuda.Stream] = None, neumann=0, flux=False,
                 coarse_op="galerkin", semi_levels=0, semi_axis="x"):
        self.lib = _lib.load()
        self.cfg = make_config(nx, ny, dx, dy, xi0, eta0, precision, nu1, nu2, smoother,
                               jacobi_omega, ir_inner_cycles, neumann, flux, coarse_op,
                               semi_levels, semi_axis)
        self.nx, self.ny = nx, ny
        nbytes = workspace_bytes(self.cfg)
        if nbytes == 0:
            raise TomgError(TOMG_EINVAL, f"invalid configuration {nx}x{ny}")
        self.device = torch.device("cuda") if device is None else torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._alloc_stream = torch.cuda.current_stream(self.device)
        self._mark_stream()
        self._h = C.c_void_p()
        self.from_map = False  # the last setup was setup_desc
        st = self.lib.tomg_create(C.byref(self.cfg), C.c_void_p(self.workspace.data_ptr()), nbytes,
                                  C.c_void_p(self.stream.cuda_stream), C.byref(self._h))
        if st != TOMG_OK:
            raise TomgError(st, "tomg_create failed")

    def _mark_stream(self):
        # the library's work on the problem's stream (from the argument store
        # of create on) uses the workspace: when that is not the stream the
        # workspace was allocated on, the allocator must not re-use the
        # memory before that stream's work has run
        if self.stream != self._alloc_stream:
            self.workspace.record_stream(self.stream)

    @classmethod
    def from_grid(cls, prob, **kw):
        """Problem sized for a ``workloads.GridProblem`` (its Neumann edges
        included)."""
        kw.setdefault("neumann", getattr(prob, "neumann", 0))
        return cls(prob.nx, prob.ny, prob.dx, prob.dy, prob.xi0, prob.eta0, **kw)

    # -- lifecycle ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self.lib.tomg_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_bytes(self) -> int:
        return self.workspace.numel()

    def last_error(self) -> str:
        return self.lib.tomg_last_error(self._h).decode()

    def _check(self, st, what):
        if st != TOMG_OK:
            raise TomgError(st, f"{what}: {self.last_error()}")

    def level_shape(self, level):
        a, b = C.c_int32(), C.c_int32()
        self._check(self.lib.tomg_level_shape(self._h, level, C.byref(a), C.byref(b)),
                    "level_shape")
        return a.value, b.value

    @property
    def num_levels(self):
        return num_levels(self.cfg)

    # -- the C-ABI calls ----------------------------------------------------
    def setup_coeffs(self, rho, xp=None, yp=None, jac=None, eps_phys=None, mask=None,
                     check=True):
        """Coefficient setup and hierarchy.  With check=False the work is
        queued without a host synchronisation and the geometry checks are
        reported later (``setup_check``, the next ``solve``, or a NaN
        residual from ``batch_step``); torch tensors passed here stay valid
        for the queued work as long as they were made on this problem's
        stream."""
        shp = (self.ny, self.nx)
        args = (_ptr(xp, torch.float64, shp, "xp"), _ptr(yp, torch.float64, shp, "yp"),
                _ptr(jac, torch.float64, (4,) + shp, "jac"),
                _ptr(eps_phys, torch.float64, shp, "eps_phys"),
                _ptr(rho, torch.float64, shp, "rho"), _ptr(mask, torch.uint8, shp, "mask"))
        fn = self.lib.setup_coeffs if check else self.lib.tomg_setup_coeffs_async
        self.from_map = False
        self._check(fn(self._h, *args), "setup_coeffs")

    def setup_desc(self, map_desc: MapDesc, source: SourceDesc, phi_init=None, check=True):
        """tomg_setup_coeffs_desc: setup from a map and a source descriptor
        (``map_desc()``, ``source_desc()``) evaluated on the device; phi_init
        (optional, float64 (ny, nx)) receives the Dirichlet data and zeros.
        check=False queues the work as ``setup_coeffs(check=False)``."""
        self.from_map = False
        st = self.lib.tomg_setup_coeffs_desc(
            self._h, C.byref(map_desc), C.byref(source),
            _ptr(phi_init, torch.float64, (self.ny, self.nx), "phi_init"),
            0 if check else _lib.TOMG_SETUP_ASYNC)
        self._check(st, "setup_coeffs_desc")
        self.from_map = True

    def update_rhs_desc(self, source: SourceDesc):
        """tomg_update_rhs_desc: a new source on the map of the last setup_desc."""
        self._check(self.lib.tomg_update_rhs_desc(self._h, C.byref(source)), "update_rhs_desc")

    def residual_history(self):
        """tomg_residual_history: relative residuals of the last solve, at its
        start and after each cycle (up to 256 entries)."""
        buf = (C.c_double * 256)()
        cnt = C.c_int32()
        self._check(self.lib.tomg_residual_history(self._h, buf, 256, C.byref(cnt)),
                    "residual_history")
        return list(buf[:cnt.value])

    def setup_check(self):
        """Raises TomgError if the last (asynchronous) setup failed its checks."""
        self._check(self.lib.tomg_setup_check(self._h), "setup_check")

    def update_rhs(self, rho):
        self._check(self.lib.tomg_update_rhs(self._h, _ptr(rho, torch.float64,
                                                           (self.ny, self.nx), "rho")),
                    "update_rhs")

    def vcycle(self, phi):
        self._check(self.lib.vcycle(self._h, _ptr(phi, torch.float64, (self.ny, self.nx), "phi")),
                    "vcycle")

    def solve(self, phi, rel_tol=1e-10, max_cycles=100, raise_on_error=True) -> SolveResult:
        cyc, rel = C.c_int32(), C.c_double()
        st = self.lib.solve(self._h, _ptr(phi, torch.float64, (self.ny, self.nx), "phi"),
                            rel_tol, max_cycles, C.byref(cyc), C.byref(rel))
        if raise_on_error and st not in (TOMG_OK, TOMG_ENOCONV):
            self._check(st, "solve")
        return SolveResult(st, cyc.value, rel.value)

    def residual_norm(self, phi):
        a, r = C.c_double(), C.c_double()
        self._check(self.lib.residual_norm(self._h, _ptr(phi, torch.float64, (self.ny, self.nx),
                                                         "phi"), C.byref(a), C.byref(r)),
                    "residual_norm")
        return a.value, r.value

    def laplace_grid(self, xp, yp, rel_tol=1e-12, max_cycles=200, mask=None, px=None,
                     py=None) -> int:
        """tomg_laplace_grid: fills xp, yp (map given on the ring and where
        mask is 1) with the solution of Laplace's equation elsewhere, or of
        Poisson's equation with the sources px, py; returns the cycles."""
        shp = (self.ny, self.nx)
        cyc = C.c_int32()
        self._check(self.lib.tomg_laplace_grid(self._h, _ptr(xp, torch.float64, shp, "xp"),
                                               _ptr(yp, torch.float64, shp, "yp"),
                                               _ptr(mask, torch.uint8, shp, "mask"),
                                               _ptr(px, torch.float64, shp, "px"),
                                               _ptr(py, torch.float64, shp, "py"), rel_tol,
                                               max_cycles, C.byref(cyc)), "laplace_grid")
        return cyc.value

    def field(self, phi, xp=None, yp=None, jac=None):
        """tomg_field: (Ex', Ey') of the potential phi under the map given by
        jac or by the node coordinates xp, yp."""
        shp = (self.ny, self.nx)
        ex = torch.empty(shp, dtype=torch.float64, device=self.device)
        ey = torch.empty_like(ex)
        self._check(self.lib.tomg_field(self._h, _ptr(phi, torch.float64, shp, "phi"),
                                        _ptr(xp, torch.float64, shp, "xp"),
                                        _ptr(yp, torch.float64, shp, "yp"),
                                        _ptr(jac, torch.float64, (4,) + shp, "jac"),
                                        C.c_void_p(ex.data_ptr()), C.c_void_p(ey.data_ptr())),
                    "field")
        return ex, ey

    # -- diagnostics ----------------------------------------------------------
    def export(self, what: str, level: int = 0) -> torch.Tensor:
        nx, ny = self.level_shape(level)
        if what == "dir":
            out = torch.empty((ny, nx), dtype=torch.uint8, device=self.device)
        elif what == "stencil":
            out = torch.empty((9, ny, nx), dtype=torch.float64, device=self.device)
        else:
            out = torch.empty((ny, nx), dtype=torch.float64, device=self.device)
        self._check(self.lib.tomg_export(self._h, FIELD[what], level, C.c_void_p(out.data_ptr())),
                    "export")
        return out

    def smooth(self, phi, sweeps=1):
        self._check(self.lib.tomg_smooth(self._h, _ptr(phi, torch.float64, (self.ny, self.nx),
                                                       "phi"), sweeps), "smooth")

    def set_stream(self, stream: torch.cuda.Stream):
        """tomg_set_stream: later calls run on `stream` (same device); the
        call first waits for the problem's old stream, so the work queued
        there is complete."""
        self._check(self.lib.tomg_set_stream(self._h, C.c_void_p(stream.cuda_stream)),
                    "set_stream")
        self.stream = stream
        self._mark_stream()

    def profile(self, enable: bool = True):
        self._check(self.lib.tomg_profile(self._h, 1 if enable else 0), "profile")

    def profile_read(self):
        """(down_ms_total, down_count, up_ms_total, up_count, chained_ms_total,
        chained_count) of level-0 passes (chained: the up pass of an FP32 inner
        cycle and the down pass of the next in one launch)."""
        out = (C.c_double * 6)()
        self._check(self.lib.tomg_profile_read(self._h, out), "profile_read")
        return tuple(out)

    def residual(self, phi) -> torch.Tensor:
        r = torch.empty_like(phi)
        self._check(self.lib.tomg_residual(self._h, _ptr(phi, torch.float64, (self.ny, self.nx),
                                                         "phi"), C.c_void_p(r.data_ptr())),
                    "residual")
        return r


def map_desc(kind: str, amp=0.0, centre=(0.5, 0.5), r_in=0.0, r_c=0.0, r_out=0.0, pert=0.0,
             coef=(0.0, 0.0, 0.0, 0.0), phase=0.0, value_in=0.0) -> MapDesc:
    """A tomg_map_desc: kind "sinusoidal" (amp), "circle" (perturbed circle:
    centre, r_in < r_c < r_out, pert, coef of cos 2..5 theta, phase,
    value_in on the conductor) or "polar" (value_in on the arc i = 0)."""
    m = MapDesc()
    m.kind = {"sinusoidal": TOMG_MAP_SINUSOIDAL, "circle": TOMG_MAP_PERTURBED_CIRCLE,
              "polar": TOMG_MAP_POLAR}[kind]
    m.amp = float(amp)
    m.cx, m.cy = float(centre[0]), float(centre[1])
    m.r_in, m.r_c, m.r_out, m.pert = float(r_in), float(r_c), float(r_out), float(pert)
    for k in range(4):
        m.coef[k] = float(coef[k])
    m.phase, m.value_in = float(phase), float(value_in)
    return m


def source_desc(amps, centres, sigma) -> SourceDesc:
    """A tomg_source_desc: rho' = sum_m amps[m] exp(-|x' - centres[m]|^2 / (2 sigma^2))."""
    if len(amps) > TOMG_MAX_GAUSSIANS or len(amps) != len(centres):
        raise TomgError(TOMG_EINVAL, f"{len(amps)} sources (at most {TOMG_MAX_GAUSSIANS})")
    s = SourceDesc()
    s.count, s.sigma = len(amps), float(sigma)
    for k, (a, c) in enumerate(zip(amps, centres)):
        s.amp[k], s.cx[k], s.cy[k] = float(a), float(c[0]), float(c[1])
    return s


# Module-level spellings of the C-ABI calls.
def setup_coeffs(p: Problem, rho, xp=None, yp=None, jac=None, eps_phys=None, mask=None):
    return p.setup_coeffs(rho, xp=xp, yp=yp, jac=jac, eps_phys=eps_phys, mask=mask)


def vcycle(p: Problem, phi):
    return p.vcycle(phi)


def solve(p: Problem, phi, rel_tol=1e-10, max_cycles=100):
    return p.solve(phi, rel_tol, max_cycles)


def residual_norm(p: Problem, phi):
    return p.residual_norm(phi)


def solve_batch(problems: Sequence[Problem], phis: Sequence[torch.Tensor], rel_tol=1e-10,
                max_cycles=100):
    """tomg_solve_batch: returns a list of SolveResult."""
    lib = _lib.load()
    n = len(problems)
    hs = (C.c_void_p * n)(*[p._h.value for p in problems])
    ps = (C.c_void_p * n)(*[_ptr(t, torch.float64, (p.ny, p.nx), "phi").value
                            for p, t in zip(problems, phis)])
    cyc = (C.c_int32 * n)()
    rel = (C.c_double * n)()
    sts = (C.c_int * n)()
    lib.tomg_solve_batch(hs, ps, n, rel_tol, max_cycles, cyc, rel, sts)
    return [SolveResult(sts[k], cyc[k], rel[k]) for k in range(n)]


def batch_step(problems: Sequence[Problem], phis: Sequence[torch.Tensor], fresh: Sequence[bool]):
    """tomg_batch_step: returns the relative residual of every problem after
    the step (initial norms for fresh ones, one cycle for the others)."""
    lib = _lib.load()
    n = len(problems)
    if n == 0:
        return []
    hs = (C.c_void_p * n)(*[p._h.value for p in problems])
    ps = (C.c_void_p * n)(*[_ptr(t, torch.float64, (p.ny, p.nx), "phi").value
                            for p, t in zip(problems, phis)])
    fr = (C.c_int32 * n)(*[1 if f else 0 for f in fresh])
    rel = (C.c_double * n)()
    st = lib.tomg_batch_step(hs, ps, n, fr, rel)
    if st != TOMG_OK:
        raise TomgError(st, "tomg_batch_step")
    return list(rel)


def batch_launch(problems: Sequence[Problem], phis: Sequence[torch.Tensor],
                 fresh: Sequence[bool], rel_out: torch.Tensor):
    """tomg_batch_launch: queues the step of ``batch_step`` on the stream of
    problems[0] and returns at once; rel_out (float64 device tensor of at
    least len(problems) elements) receives the relative residuals in stream
    order.  The caller keeps the problems, iterates and rel_out alive until
    the step has run."""
    lib = _lib.load()
    n = len(problems)
    if n == 0:
        return
    if not (rel_out.is_cuda and rel_out.dtype == torch.float64 and rel_out.is_contiguous()
            and rel_out.numel() >= n):
        raise TomgError(TOMG_EINVAL, "rel_out: contiguous float64 device tensor of >= n elements")
    hs = (C.c_void_p * n)(*[p._h.value for p in problems])
    ps = (C.c_void_p * n)(*[_ptr(t, torch.float64, (p.ny, p.nx), "phi").value
                            for p, t in zip(problems, phis)])
    fr = (C.c_int32 * n)(*[1 if f else 0 for f in fresh])
    st = lib.tomg_batch_launch(hs, ps, n, fr, C.c_void_p(rel_out.data_ptr()))
    if st != TOMG_OK:
        raise TomgError(st, "tomg_batch_launch")


NOALLOC_MAX_BYTES = 128 * 1024 * 1024  # TOMG_NOALLOC_MAX_BYTES


def solve_noalloc(cfg: Config, rho, phi, xp=None, yp=None, jac=None, eps_phys=None, mask=None,
                  rel_tol=1e-10, max_cycles=100, stream=None):
    """tomg_solve_noalloc: setup_coeffs + solve on the library's static
    workspace (no allocation by the library).  Returns (SolveResult,
    message)."""
    lib = _lib.load()
    shp = (cfg.ny, cfg.nx)
    s = stream if stream is not None else torch.cuda.current_stream(phi.device)
    cyc, rel = C.c_int32(), C.c_double()
    err = C.create_string_buffer(256)
    st = lib.tomg_solve_noalloc(C.byref(cfg), _ptr(xp, torch.float64, shp, "xp"),
                                _ptr(yp, torch.float64, shp, "yp"),
                                _ptr(jac, torch.float64, (4,) + shp, "jac"),
                                _ptr(eps_phys, torch.float64, shp, "eps_phys"),
                                _ptr(rho, torch.float64, shp, "rho"),
                                _ptr(mask, torch.uint8, shp, "mask"),
                                _ptr(phi, torch.float64, shp, "phi"), rel_tol, max_cycles,
                                C.c_void_p(s.cuda_stream), C.byref(cyc), C.byref(rel), err,
                                len(err))
    return SolveResult(st, cyc.value, rel.value), err.value.decode()


def copy_probe(src: torch.Tensor, dst: torch.Tensor, stream=None):
    """Device copy of src into dst with the library's STREAM-style kernel."""
    lib = _lib.load()
    nbytes = src.numel() * src.element_size()
    s = stream if stream is not None else torch.cuda.current_stream(src.device)
    st = lib.tomg_copy_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes,
                             C.c_void_p(s.cuda_stream))
    if st != TOMG_OK:
        raise TomgError(st, "copy_probe")


def upload(prob, device="cuda"):
    """Moves the arrays of a ``workloads.GridProblem`` to the GPU:
    returns dict(xp, yp, jac, rho, mask, phi0) of tensors (None where absent)."""
    def t(a, dtype=torch.float64):
        return None if a is None else torch.as_tensor(a, dtype=dtype).contiguous().to(device)
    return {"xp": t(prob.xp), "yp": t(prob.yp), "jac": t(prob.jac), "rho": t(prob.rho),
            "mask": t(prob.mask, torch.uint8), "phi0": t(prob.phi0)}


def setup_from_grid(prob, device="cuda", check=True, **kw):
    """Problem + upload + setup_coeffs for a ``workloads.GridProblem``.
    The analytic Jacobian is used when the problem carries one; check=False
    queues the setup with its checks deferred."""
    p = Problem.from_grid(prob, device=device, **kw)
    d = upload(prob, device)
    if d["jac"] is not None:
        p.setup_coeffs(d["rho"], jac=d["jac"], mask=d["mask"], check=check)
    else:
        p.setup_coeffs(d["rho"], xp=d["xp"], yp=d["yp"], mask=d["mask"], check=check)
    return p, d

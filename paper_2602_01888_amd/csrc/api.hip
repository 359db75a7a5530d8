// C-ABI of libtomg: argument checking, workspace layout, the cycle driver
// and the stopping test.  Kernels live in kernels.hip.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "tomg_internal.h"

namespace tomg {

// Halve while both node counts minus one are even and each side keeps at
// least 3 nodes; coarsen at least once, then while a side exceeds 9 nodes
// (5 with Neumann edges, whose ring nodes are unknowns on the coarsest
// level too: at most 25 coarsest unknowns instead of 49).  With
// semi-coarsening the first c.semi_levels coarsenings halve one axis only,
// each of them required.
int level_shapes(const tomg_config &c, int *nxs, int *nys, int *ck) {
  const int lim = c.neumann ? 5 : 9;
  if (c.nx < 5 || c.ny < 5) return 0;
  int L = 1;
  nxs[0] = c.nx;
  nys[0] = c.ny;
  while (L < kMaxLevels) {
    const int cx = nxs[L - 1], cy = nys[L - 1];
    int kind = 0;
    if (L - 1 < c.semi_levels) {
      const int side = c.semi_axis == 0 ? cx : cy;
      if ((side - 1) % 2 != 0 || side < 5) return 0;
      kind = c.semi_axis == 0 ? 1 : 2;
    } else {
      const bool halvable = ((cx - 1) % 2 == 0) && ((cy - 1) % 2 == 0) && cx >= 5 && cy >= 5;
      const bool wanted = (L == 1) || cx > lim || cy > lim;
      if (!halvable || !wanted) break;
    }
    nxs[L] = kind == 2 ? cx : (cx - 1) / 2 + 1;
    nys[L] = kind == 1 ? cy : (cy - 1) / 2 + 1;
    if (ck) ck[L - 1] = kind;
    ++L;
  }
  if (L < 2 || L - 1 < c.semi_levels) return 0;
  if (ck) ck[L - 1] = 0;
  // halving stopped above the bound: the coarsest level is kept when its
  // direct solve stays within kMaxCoarseNodes nodes
  if ((nxs[L - 1] > lim || nys[L - 1] > lim) &&
      (long)nxs[L - 1] * nys[L - 1] > kMaxCoarseNodes)
    return 0;
  return L;
}

static bool config_ok(const tomg_config &c) {
  if (c.nx < 5 || c.ny < 5) return false;
  if (!(c.dx > 0.0) || !(c.dy > 0.0) || !std::isfinite(c.dx) || !std::isfinite(c.dy)) return false;
  if (c.precision != TOMG_FP64 && c.precision != TOMG_FP32_IR) return false;
  if (c.nu1 < 1 || c.nu2 < 1 || c.nu1 > 4 || c.nu2 > 4) return false;
  if (c.smoother != TOMG_GS4 && c.smoother != TOMG_JACOBI && c.smoother != TOMG_ZEBRA_X &&
      c.smoother != TOMG_ZEBRA_XY)
    return false;
  if (c.smoother == TOMG_ZEBRA_XY &&
      (c.ny > kZebraMaxNx || c.nx > kZebraMaxNx || c.precision != TOMG_FP64))
    return false;
  if (c.smoother == TOMG_ZEBRA_X && c.nx > kZebraMaxNx) return false;  // the row in LDS
  if (c.smoother == TOMG_JACOBI && !(c.jacobi_omega > 0.0 && c.jacobi_omega <= 1.0)) return false;
  if (c.precision == TOMG_FP32_IR && (c.ir_inner_cycles < 1 || c.ir_inner_cycles > 16)) return false;
  if (c.neumann < 0 || c.neumann > 15) return false;
  if (c.flux != 0 && c.flux != 1) return false;
  if (c.coarse_op != TOMG_GALERKIN && c.coarse_op != TOMG_REDISCRETIZE) return false;
  // rediscretisation builds eq. 18 on every level: Dirichlet edges only
  if (c.coarse_op == TOMG_REDISCRETIZE && stored_level0(c)) return false;
  // semi-coarsened levels: fused four-colour passes and Galerkin operators
  if (c.semi_levels < 0 || c.semi_levels >= kMaxLevels || c.semi_axis < 0 || c.semi_axis > 1)
    return false;
  if (c.semi_levels > 0 && (c.smoother != TOMG_GS4 || c.coarse_op != TOMG_GALERKIN)) return false;
  int a[kMaxLevels], b[kMaxLevels];
  return level_shapes(c, a, b, nullptr) > 0;
}

bool make_layout(const tomg_config &cfg, Layout *lay) {
  if (!config_ok(cfg)) return false;
  Layout &o = *lay;
  o = Layout();
  o.L = level_shapes(cfg, o.nx, o.ny, o.ck);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) & ~(size_t)255;
    return at;
  };
  const size_t n0 = (size_t)cfg.nx * cfg.ny;
  o.scal = take((kNumSlots + kHistMax) * sizeof(double));
  const size_t nparts = std::max({(size_t)2 * kRedBlocks, fused_max_blocks(cfg.nx, cfg.ny),
                                  (size_t)2 * red_tiles(cfg.nx, cfg.ny)});
  o.partials = take(nparts * sizeof(double));
  // explicit inverse of the coarsest matrix, its node-to-unknown map and,
  // for a coarsest level that may hold more unknowns than the one-block
  // Gauss-Jordan takes (kMaxCoarseUnknowns: above kSmallCoarseNodes nodes,
  // or free ring nodes of Neumann edges on a semi-coarsened hierarchy, such
  // as 3 x 17 nodes without a Dirichlet edge), the band LU (half-width
  // nx + 1 in the row-major numbering of the unknowns)
  const int cxn = o.nx[o.L - 1], cyn = o.ny[o.L - 1];
  const size_t mc = (size_t)cxn * cyn;
  const int ring_x = !(cfg.neumann & TOMG_NEU_W) + !(cfg.neumann & TOMG_NEU_E);
  const int ring_y = !(cfg.neumann & TOMG_NEU_S) + !(cfg.neumann & TOMG_NEU_N);
  const long max_unknowns = (long)(cxn - ring_x) * (cyn - ring_y);
  const bool band = mc > (size_t)kSmallCoarseNodes || max_unknowns > kMaxCoarseUnknowns;
  const size_t mi = band ? mc : (size_t)kMaxCoarseUnknowns;
  o.cinv = take(mi * mi * sizeof(double));
  o.cidx = take((std::max(mc, (size_t)81) + 1) * sizeof(int));
  if (band) o.cband = take(mc * (2 * (size_t)(cxn + 1) + 1) * sizeof(double));
  o.args = take(sizeof(ArgsBlob));
  o.bout = take(kMaxBatch * sizeof(double));
  o.exx = take(n0 * 8);
  o.exy = take(n0 * 8);
  o.eyy = take(n0 * 8);
  o.det = take(n0 * 8);
  o.f = take(n0 * 8);
  o.tmp = take(n0 * 8);
  o.dir[0] = take(n0);
  // Neumann edges: the level-0 stencil with the ghost layer folded in
  if (stored_level0(cfg)) o.st[0] = take(9 * n0 * 8);
  for (int l = 1; l < o.L; ++l) {
    const size_t n = (size_t)o.nx[l] * o.ny[l];
    o.st[l] = take(9 * n * 8);
    o.x[l] = take(n * 8);
    o.x2[l] = take(n * 8);
    o.b[l] = take(n * 8);
    o.dir[l] = take(n);
  }
  if (cfg.smoother == TOMG_ZEBRA_XY)
    for (int l = 0; l < o.L; ++l) {
      const size_t n = (size_t)o.nx[l] * o.ny[l];
      o.stT[l] = take(9 * n * 8);
      o.xT[l] = take(n * 8);
      o.bT[l] = take(n * 8);
      o.dirT[l] = take(n);
    }
  if (cfg.precision == TOMG_FP32_IR) {
    o.exx32 = take(n0 * 4);
    o.exy32 = take(n0 * 4);
    o.eyy32 = take(n0 * 4);
    o.e32 = take(n0 * 4);
    o.e32b = take(n0 * 4);
    o.r32 = take(n0 * 4);
    o.phi2 = take(n0 * 8);
    if (stored_level0(cfg)) o.st32[0] = take(9 * n0 * 4);
    for (int l = 1; l < o.L; ++l) {
      const size_t n = (size_t)o.nx[l] * o.ny[l];
      o.st32[l] = take(9 * n * 4);
      o.x32[l] = take(n * 4);
      o.x2_32[l] = take(n * 4);
      o.b32[l] = take(n * 4);
    }
  }
  o.total = off;
  return true;
}

}  // namespace tomg

using namespace tomg;

static tomg_status fail(tomg_problem *p, tomg_status s, const char *fmt, ...) {
  if (p) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(p->err, sizeof(p->err), fmt, ap);
    va_end(ap);
  }
  return s;
}

#define HIP_TRY(p, expr)                                                                  \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(p, TOMG_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

// Copies the device scalar block (and, with n > kNumSlots, the first n -
// kNumSlots entries of the residual history after it) to the host and waits
// for the stream.
static tomg_status read_scalars(tomg_problem *p, double *h, int n = kNumSlots) {
  HIP_TRY(p, hipMemcpyAsync(h, p->scal, n * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(p, hipStreamSynchronize(p->stream));
  prof_harvest(p);
  return TOMG_OK;
}

static void destroy_events(tomg_problem *p) {
  for (int kind = 0; kind < tomg_problem::kProfKinds; ++kind)
    for (int e = 0; e < tomg_problem::kMaxEv; ++e)
      for (int q = 0; q < 2; ++q)
        if (p->ev[kind][e][q]) {
          (void)hipEventDestroy(p->ev[kind][e][q]);
          p->ev[kind][e][q] = nullptr;
        }
}

extern "C" {

void tomg_config_default(tomg_config *cfg, int32_t nx, int32_t ny, double dx, double dy) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->nx = nx;
  cfg->ny = ny;
  cfg->dx = dx;
  cfg->dy = dy;
  cfg->precision = TOMG_FP64;
  cfg->nu1 = 2;
  cfg->nu2 = 2;
  cfg->smoother = TOMG_GS4;
  cfg->jacobi_omega = 0.8;
  cfg->ir_inner_cycles = 2;
}

int32_t tomg_num_levels(const tomg_config *cfg) {
  if (!cfg || !config_ok(*cfg)) return 0;
  int a[kMaxLevels], b[kMaxLevels];
  return level_shapes(*cfg, a, b, nullptr);
}

size_t tomg_workspace_bytes(const tomg_config *cfg) {
  if (!cfg) return 0;
  Layout lay;
  return make_layout(*cfg, &lay) ? lay.total : 0;
}

}  // extern "C"

// Binds the problem state p to the workspace d_ws (laid out by lay) and
// queues the clearing of its scalar block and the store of its launch
// arguments on the stream.  Allocates nothing.
static hipError_t init_problem(tomg_problem *p, const tomg_config *cfg, const Layout &lay,
                               void *d_ws, size_t ws_bytes, void *stream) {
  p->err[0] = 0;
  p->cfg = *cfg;
  p->lay = lay;
  p->stream = (hipStream_t)stream;
  p->ws = (char *)d_ws;
  p->ws_bytes = ws_bytes;
  p->L = lay.L;
  char *w = p->ws;
  auto D = [&](size_t off) { return (double *)(w + off); };
  auto F = [&](size_t off) { return (float *)(w + off); };
  p->scal = D(lay.scal);
  p->partials = D(lay.partials);
  p->cinv = D(lay.cinv);
  p->cidx = (int *)(w + lay.cidx);
  p->cband = lay.cband ? D(lay.cband) : nullptr;
  p->exx = D(lay.exx);
  p->exy = D(lay.exy);
  p->eyy = D(lay.eyy);
  p->det = D(lay.det);
  p->f = D(lay.f);
  p->tmp = D(lay.tmp);
  for (int l = 0; l < p->L; ++l) {
    Level &v = p->lv[l];
    v.nx = lay.nx[l];
    v.ny = lay.ny[l];
    v.ck = lay.ck[l];
    v.n = (size_t)v.nx * v.ny;
    v.dir = (uint8_t *)(w + lay.dir[l]);
    if (l == 0 && stored_level0(*cfg)) v.st = D(lay.st[0]);
    if (cfg->smoother == TOMG_ZEBRA_XY) {
      v.stT = D(lay.stT[l]);
      v.xT = D(lay.xT[l]);
      v.bT = D(lay.bT[l]);
      v.dirT = (uint8_t *)(w + lay.dirT[l]);
    }
    if (l > 0) {
      v.st = D(lay.st[l]);
      v.x = D(lay.x[l]);
      v.x2 = D(lay.x2[l]);
      v.b = D(lay.b[l]);
    }
  }
  if (cfg->precision == TOMG_FP32_IR) {
    p->exx32 = F(lay.exx32);
    p->exy32 = F(lay.exy32);
    p->eyy32 = F(lay.eyy32);
    p->e32 = F(lay.e32);
    p->e32b = F(lay.e32b);
    p->phi2 = D(lay.phi2);
    p->r32 = F(lay.r32);
    if (stored_level0(*cfg)) p->lv[0].st32 = F(lay.st32[0]);
    for (int l = 1; l < p->L; ++l) {
      p->lv[l].st32 = F(lay.st32[l]);
      p->lv[l].x32 = F(lay.x32[l]);
      p->lv[l].x2_32 = F(lay.x2_32[l]);
      p->lv[l].b32 = F(lay.b32[l]);
    }
  }
  p->dargs = (ArgsBlob *)(w + lay.args);
  p->bout = D(lay.bout);
  // the single-workgroup tail assumes Dirichlet rings and halves both axes;
  // problems with a stored level-0 stencil (Neumann edges, flux form) or
  // semi-coarsened levels run the level passes down to the coarsest solve
  const bool no_tail = stored_level0(*cfg) || cfg->semi_levels > 0;
  p->lc = no_tail ? p->L - 1 : tail_level(p, false);
  p->lcb = no_tail ? p->L - 1 : tail_level(p, true);
  build_pass_args(p);
  build_tail_args(p);
  build_red_args(p);
  // queued on the stream, no host wait: a problem can be created while the
  // stream still runs other problems' work
  hipError_t e = launch_set_slots(p, (1u << kNumSlots) - 1u, 0.0);
  if (e == hipSuccess) e = upload_args(p);
  return e;
}

extern "C" {

tomg_status tomg_create(const tomg_config *cfg, void *d_ws, size_t ws_bytes, void *stream,
                        tomg_problem **out) {
  if (!out) return TOMG_EINVAL;
  *out = nullptr;
  if (!cfg || !d_ws) return TOMG_EINVAL;
  if (((uintptr_t)d_ws) % 256 != 0) return TOMG_EINVAL;
  Layout lay;
  if (!make_layout(*cfg, &lay)) return TOMG_EINVAL;
  if (ws_bytes < lay.total) return TOMG_ENOMEM;
  tomg_problem *p = new (std::nothrow) tomg_problem();
  if (!p) return TOMG_ENOMEM;
  if (init_problem(p, cfg, lay, d_ws, ws_bytes, stream) != hipSuccess) {
    delete p;
    return TOMG_EDEVICE;
  }
  *out = p;
  return TOMG_OK;
}

void tomg_destroy(tomg_problem *p) {
  if (!p) return;
  destroy_events(p);
  delete p;
}

const char *tomg_last_error(const tomg_problem *p) {
  if (!p) return "null problem";
  return p->err;
}

tomg_status tomg_set_stream(tomg_problem *p, void *stream) {
  if (!p) return TOMG_EINVAL;
  // work already queued for the problem (the argument store of its create,
  // an asynchronous setup) runs before anything on the new stream
  if (hipStreamSynchronize(p->stream) != hipSuccess)
    return fail(p, TOMG_EDEVICE, "set_stream: the previous stream failed");
  p->stream = (hipStream_t)stream;
  return TOMG_OK;
}

}  // extern "C"

// Status of the checks a setup leaves in the scalar block.
static tomg_status setup_status(tomg_problem *p, const double *h) {
  if (!(h[kSlotMinDet] > 0.0))
    return fail(p, TOMG_EGEOMETRY, "setup_coeffs: det J = %g <= 0 (folded or degenerate map)",
                h[kSlotMinDet]);
  if (h[kSlotBad] != 0.0)
    return fail(p, TOMG_ENONFINITE, "setup_coeffs: %g non-finite coefficients or sources",
                h[kSlotBad]);
  if (h[kSlotPivot] != 0.0)
    return fail(p, TOMG_EGEOMETRY,
                "setup_coeffs: singular coarsest-level matrix (a problem without Dirichlet "
                "nodes has no unique solution)");
  return TOMG_OK;
}

// After a read of the scalar block: reports the checks of an asynchronous
// setup that no call has reported yet.
static tomg_status pending_setup_status(tomg_problem *p, const double *h) {
  if (!p->unchecked) return TOMG_OK;
  tomg_status s = setup_status(p, h);
  if (s != TOMG_OK) {
    p->ready = false;
    return s;
  }
  p->unchecked = false;
  return TOMG_OK;
}

// Queues the setup kernels.  defer_inverse: the coarsest inverse waits for
// the problem's next cycle (batched with other problems' in a batch step).
static tomg_status setup_launch(tomg_problem *p, const double *d_xp, const double *d_yp,
                                const double *d_jac, const double *d_eps_phys,
                                const double *d_rho_phys, const uint8_t *d_mask,
                                bool defer_inverse) {
  p->ready = false;
  p->unchecked = false;
  if (!d_rho_phys) return fail(p, TOMG_EINVAL, "setup_coeffs: rho is NULL");
  if (!d_jac && (!d_xp || !d_yp))
    return fail(p, TOMG_EINVAL, "setup_coeffs: need the Jacobian or both coordinate arrays");
  // the setup's own source check replaces that of any earlier update_rhs
  // (the coarsest inverse gives its own singularity verdict)
  HIP_TRY(p, launch_set_slots(p, 1u << kSlotBadRhs, 0.0));
  p->has_map = false;
  HIP_TRY(p, launch_setup(p, d_xp, d_yp, d_jac, d_eps_phys, d_rho_phys, d_mask));
  HIP_TRY(p, launch_hierarchy(p, defer_inverse));
  return TOMG_OK;
}

static const char *source_desc_error(const tomg_source_desc *src) {
  if (!src) return "source descriptor is NULL";
  if (src->count < 0 || src->count > TOMG_MAX_GAUSSIANS)
    return "source count outside 0..TOMG_MAX_GAUSSIANS";
  if (src->count > 0 && !(src->sigma > 0.0)) return "source sigma <= 0";
  return nullptr;
}

static const char *map_desc_error(const tomg_map_desc *m) {
  if (!m) return "map descriptor is NULL";
  if (m->kind == TOMG_MAP_SINUSOIDAL || m->kind == TOMG_MAP_POLAR) return nullptr;
  if (m->kind != TOMG_MAP_PERTURBED_CIRCLE) return "unknown map kind";
  if (!(m->r_in < m->r_c && m->r_c < m->r_out))
    return "perturbed circle needs r_in < r_c < r_out";
  return nullptr;
}

// setup_launch for a map and a source given by descriptors.
static tomg_status setup_desc_launch(tomg_problem *p, const tomg_map_desc *map,
                                     const tomg_source_desc *src, double *d_phi_init,
                                     bool defer_inverse) {
  p->ready = false;
  p->unchecked = false;
  p->has_map = false;
  if (const char *e = map_desc_error(map)) return fail(p, TOMG_EINVAL, "setup_coeffs_desc: %s", e);
  if (const char *e = source_desc_error(src))
    return fail(p, TOMG_EINVAL, "setup_coeffs_desc: %s", e);
  HIP_TRY(p, launch_set_slots(p, 1u << kSlotBadRhs, 0.0));
  HIP_TRY(p, launch_setup_desc(p, *map, *src, d_phi_init));
  HIP_TRY(p, launch_hierarchy(p, defer_inverse));
  p->map = *map;
  p->has_map = true;
  return TOMG_OK;
}

extern "C" {

tomg_status setup_coeffs(tomg_problem *p, const double *d_xp, const double *d_yp,
                         const double *d_jac, const double *d_eps_phys,
                         const double *d_rho_phys, const uint8_t *d_mask) {
  if (!p) return TOMG_EINVAL;
  tomg_status s = setup_launch(p, d_xp, d_yp, d_jac, d_eps_phys, d_rho_phys, d_mask, false);
  if (s != TOMG_OK) return s;
  double h[kNumSlots];
  s = read_scalars(p, h);
  if (s != TOMG_OK) return s;
  s = setup_status(p, h);
  if (s != TOMG_OK) return s;
  p->ready = true;
  return TOMG_OK;
}

tomg_status tomg_setup_coeffs_async(tomg_problem *p, const double *d_xp, const double *d_yp,
                                    const double *d_jac, const double *d_eps_phys,
                                    const double *d_rho_phys, const uint8_t *d_mask) {
  if (!p) return TOMG_EINVAL;
  tomg_status s = setup_launch(p, d_xp, d_yp, d_jac, d_eps_phys, d_rho_phys, d_mask, true);
  if (s != TOMG_OK) return s;
  p->ready = true;
  p->unchecked = true;
  return TOMG_OK;
}

tomg_status tomg_setup_coeffs_desc(tomg_problem *p, const tomg_map_desc *map,
                                   const tomg_source_desc *src, double *d_phi_init,
                                   uint32_t flags) {
  if (!p) return TOMG_EINVAL;
  if (flags & ~(uint32_t)TOMG_SETUP_ASYNC)
    return fail(p, TOMG_EINVAL, "setup_coeffs_desc: unknown flags %#x", flags);
  const bool async = flags & TOMG_SETUP_ASYNC;
  tomg_status s = setup_desc_launch(p, map, src, d_phi_init, async);
  if (s != TOMG_OK) return s;
  if (async) {
    p->ready = true;
    p->unchecked = true;
    return TOMG_OK;
  }
  double h[kNumSlots];
  s = read_scalars(p, h);
  if (s != TOMG_OK) return s;
  s = setup_status(p, h);
  if (s != TOMG_OK) return s;
  p->ready = true;
  return TOMG_OK;
}

tomg_status tomg_update_rhs_desc(tomg_problem *p, const tomg_source_desc *src) {
  if (!p) return TOMG_EINVAL;
  if (!p->ready) return fail(p, TOMG_ESTATE, "update_rhs_desc before setup_coeffs");
  if (!p->has_map)
    return fail(p, TOMG_ESTATE, "update_rhs_desc: the problem was not set up from a map");
  if (const char *e = source_desc_error(src))
    return fail(p, TOMG_EINVAL, "update_rhs_desc: %s", e);
  HIP_TRY(p, launch_update_rhs_desc(p, p->map, *src));
  return TOMG_OK;
}

tomg_status tomg_residual_history(tomg_problem *p, double *out, int32_t cap, int32_t *count) {
  if (!p || (cap > 0 && !out) || cap < 0) return TOMG_EINVAL;
  double h[kNumSlots + kHistMax];
  HIP_TRY(p, hipMemcpyAsync(h, p->scal, sizeof h, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(p, hipStreamSynchronize(p->stream));
  const double c = h[kSlotCycles];
  const int n = std::isfinite(c) && c >= 0.0 ? (int)std::min(c + 1.0, (double)kHistMax) : 0;
  for (int k = 0; k < n && k < cap; ++k) out[k] = h[kNumSlots + k];
  if (count) *count = n;
  return TOMG_OK;
}

tomg_status tomg_setup_check(tomg_problem *p) {
  if (!p) return TOMG_EINVAL;
  if (!p->ready) return fail(p, TOMG_ESTATE, "setup_check before setup_coeffs");
  if (!p->unchecked) return TOMG_OK;
  HIP_TRY(p, launch_coarse_inverse(p));
  double h[kNumSlots];
  tomg_status s = read_scalars(p, h);
  if (s != TOMG_OK) return s;
  return pending_setup_status(p, h);
}

tomg_status tomg_update_rhs(tomg_problem *p, const double *d_rho_phys) {
  if (!p || !d_rho_phys) return TOMG_EINVAL;
  if (!p->ready) return fail(p, TOMG_ESTATE, "update_rhs before setup_coeffs");
  HIP_TRY(p, launch_update_rhs(p, d_rho_phys));
  return TOMG_OK;
}

tomg_status vcycle(tomg_problem *p, double *d_phi) {
  if (!p || !d_phi) return TOMG_EINVAL;
  if (!p->ready) return fail(p, TOMG_ESTATE, "vcycle before setup_coeffs");
  HIP_TRY(p, launch_coarse_inverse(p));
  if (p->cfg.precision == TOMG_FP32_IR) {
    HIP_TRY(p, launch_ir_residual(p, d_phi));
    HIP_TRY(p, launch_ir_correct(p, d_phi));
  } else {
    HIP_TRY(p, launch_vcycle64(p, d_phi, false));
  }
  return TOMG_OK;
}

tomg_status residual_norm(tomg_problem *p, const double *d_phi, double *abs_out,
                          double *rel_out) {
  if (!p || !d_phi) return TOMG_EINVAL;
  if (!p->ready) return fail(p, TOMG_ESTATE, "residual_norm before setup_coeffs");
  HIP_TRY(p, launch_coarse_inverse(p));  // its singularity verdict is reported here too
  HIP_TRY(p, launch_begin(p, d_phi, false));
  double h[kNumSlots];
  tomg_status s = read_scalars(p, h);
  if (s != TOMG_OK) return s;
  s = pending_setup_status(p, h);
  if (s != TOMG_OK) return s;
  if (abs_out) *abs_out = h[kSlotRes];
  if (rel_out) *rel_out = h[kSlotRel];
  return TOMG_OK;
}

tomg_status solve(tomg_problem *p, double *d_phi, double rel_tol, int32_t max_cycles,
                  int32_t *cycles_out, double *rel_res_out) {
  if (!p || !d_phi) return TOMG_EINVAL;
  if (!(rel_tol > 0.0) || max_cycles < 0) return fail(p, TOMG_EINVAL, "solve: bad tol/max_cycles");
  if (!p->ready) return fail(p, TOMG_ESTATE, "solve before setup_coeffs");
  HIP_TRY(p, launch_coarse_inverse(p));
  const bool ir = p->cfg.precision == TOMG_FP32_IR;
  // the device-side stopping test compares with this tolerance; the cycle
  // counter starts at zero
  p->up[0] = rel_tol;
  p->up[1] = 0.0;
  HIP_TRY(p, hipMemcpyAsync(p->scal + kSlotTol, p->up, 2 * sizeof(double),
                            hipMemcpyHostToDevice, p->stream));
  HIP_TRY(p, launch_begin(p, d_phi, ir));
  const bool queue = p->cfg.smoother == TOMG_GS4;
  // k cycles (refinement steps) queued behind the device convergence flag,
  // the first of them cycle number `first`
  auto launch_cycles = [&](int first, int k) {
    p->skip = queue ? p->scal + kSlotDone : nullptr;
    hipError_t e = hipSuccess;
    for (int q = 0; q < k && e == hipSuccess; ++q) {
      if (ir) {
        // the update and the next residual in one pass; the iterate of an
        // odd-numbered step lives in the problem's second array (steps
        // skipped past convergence are a suffix, so the executed count
        // tells where the last iterate is)
        e = launch_ir_inner(p);
        if (e == hipSuccess) e = launch_ir_step(p, d_phi, (first + q) & 1);
      } else {
        e = launch_vcycle64(p, d_phi, true);
      }
    }
    p->skip = nullptr;
    return e;
  };
  double h[kNumSlots + 1];
  int cycles = 0, queued = 0;
  double rel, rel0, prev = NAN;
  // A problem whose setup has been checked and that has converged before
  // queues its first cycles right behind the initial norms, with no host
  // check between: the initial norms set the device convergence flag (also
  // for a non-finite start), so cycles queued past it do nothing.  Their
  // number is what the last solve's contraction predicts from that solve's
  // initial relative residual (1 from a cold start, less for a sequence of
  // warm starts).  The initial relative residual is then read from the
  // first entry of the residual history.
  int k0 = 0;
  if (queue && !p->unchecked && max_cycles > 0 && p->last_rate > 0.0 && p->last_rate < 1.0) {
    const double from = std::min(1.0, std::max(p->last_rel0, rel_tol));
    k0 = std::max(1, std::min({(int)std::ceil(std::log(rel_tol / from) / std::log(p->last_rate)),
                               16, max_cycles}));
  }
  if (k0 > 0) {
    const hipError_t e = launch_cycles(0, k0);
    if (e != hipSuccess) return fail(p, TOMG_EDEVICE, "solve: cycle launch failed: %s",
                                     hipGetErrorString(e));
    tomg_status s = read_scalars(p, h, kNumSlots + 1);
    if (s != TOMG_OK) return s;
    rel0 = prev = h[kNumSlots];
    cycles = queued = (int)h[kSlotCycles];
    rel = h[kSlotRel];
  } else {
    tomg_status s = read_scalars(p, h);
    if (s != TOMG_OK) return s;
    s = pending_setup_status(p, h);
    if (s != TOMG_OK) return s;
    rel0 = rel = h[kSlotRel];
  }
  tomg_status s;
  tomg_status st = TOMG_ENOCONV;
  // Cycles are queued several at a time between host checks.  Each cycle's
  // norm sets the device convergence flag; the launches of cycles queued
  // past convergence see it and do nothing, so the iterate, the residual and
  // the cycle count are those of checking after every cycle.  The batch size
  // is the number of cycles the observed contraction predicts (at least 1).
  while (true) {
    if (!std::isfinite(rel)) {
      st = fail(p, TOMG_ENONFINITE, "solve: non-finite residual after %d cycles", cycles);
      break;
    }
    if (rel <= rel_tol) {
      st = TOMG_OK;
      break;
    }
    if (cycles >= max_cycles) {
      st = fail(p, TOMG_ENOCONV, "solve: rel. residual %.3e after %d cycles", rel, cycles);
      break;
    }
    int k = 1;
    // the unfused cycles (Jacobi, zebra) have no convergence check of their
    // own and are checked after every cycle
    if (queue) {
      const double rate = queued > 0 ? std::pow(rel / prev, 1.0 / queued) : NAN;
      if (std::isfinite(rate) && rate > 0.0 && rate < 1.0)
        k = (int)std::ceil(std::log(rel_tol / rel) / std::log(rate));
      else if (cycles == 0)
        k = 2;
      k = std::max(1, std::min(k, 16));
    }
    k = std::min(k, max_cycles - cycles);
    const hipError_t e = launch_cycles(cycles, k);
    if (e != hipSuccess) return fail(p, TOMG_EDEVICE, "solve: cycle launch failed: %s",
                                     hipGetErrorString(e));
    s = read_scalars(p, h);
    if (s != TOMG_OK) return s;
    prev = rel;
    queued = (int)h[kSlotCycles] - cycles;
    cycles = (int)h[kSlotCycles];
    rel = h[kSlotRel];
  }
  if (ir && (cycles & 1)) {  // the last iterate is in the second array
    HIP_TRY(p, hipMemcpyAsync(d_phi, p->phi2, p->lv[0].n * sizeof(double),
                              hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
  }
  if (st == TOMG_OK && cycles > 0 && rel0 > 0.0 && rel > 0.0) {
    p->last_rate = std::pow(rel / rel0, 1.0 / cycles);
    p->last_rel0 = rel0;
  }
  if (cycles_out) *cycles_out = cycles;
  if (rel_res_out) *rel_res_out = rel;
  return st;
}

// Batched solve.  Every stage of a cycle is one launch (per kBatchMax
// problems) across the problems still iterating; stages are aligned from
// the finest level, each problem taking part in the levels it has.  Every
// node sees the arithmetic of solve(), so each iterate is bitwise that of
// solve() after the same number of cycles (a batched pass uses taller row
// bands, so its residual norm is summed in another order).
}  // extern "C"

namespace {

// Batched execution needs one configuration of the cycle for all problems:
// one launch serves a stage of every problem, so the level-0 operator is
// either on-the-fly eq. 18 for all of them or a stored stencil for all, and
// the level transfers are the same (equal semi-coarsened levels).
bool batch_uniform(tomg_problem *const *probs, double *const *d_phis, int n) {
  const tomg_problem *lead = probs[0];
  if (!lead) return false;
  for (int k = 0; k < n; ++k) {
    const tomg_problem *p = probs[k];
    if (!p || !d_phis[k] || !p->ready) return false;
    if (p->cfg.precision != lead->cfg.precision || p->cfg.nu1 != lead->cfg.nu1 ||
        p->cfg.nu2 != lead->cfg.nu2 || p->cfg.smoother != TOMG_GS4 ||
        p->cfg.semi_levels != lead->cfg.semi_levels || p->cfg.semi_axis != lead->cfg.semi_axis ||
        stored_level0(p->cfg) != stored_level0(lead->cfg) ||
        p->cfg.ir_inner_cycles != lead->cfg.ir_inner_cycles)
      return false;
  }
  return true;
}

// Initial norms of the problems idx[0..cnt): |b| from the zero interior
// start and the residual of the given iterate; relative residuals to out[q]
// (to out[idx[q]] with by_index).
void batch_begin(tomg_problem *const *probs, const int *idx, int cnt, double *const *d_phis,
                 bool ir, double *out, hipStream_t s, bool by_index = false) {
  batch_begin_norms(probs, idx, cnt, ir, d_phis, s);
  batch_finalize(probs, idx, cnt, 2, kSlotB0, kRelNone, out, s, by_index);
  batch_finalize(probs, idx, cnt, 0, kSlotRes, kRelBegin, out, s, by_index);
}

// One V-cycle (FP64) or one refinement step (FP32 inner cycles) of the
// problems idx[0..cnt), then their residuals; relative residuals to out[q]
// (to out[idx[q]] with by_index).  Each stage is one launch over all
// problems that have that level above their single-workgroup tail.
// With roles (indexed like probs), the refinement update and residual run as
// one pass that moves problem k's iterate to its second array (roles[k] = 0)
// or back (1); without, the update is applied in place.
void batch_cycle(tomg_problem *const *probs, const int *idx, int cnt, double *const *d_phis,
                 bool ir, int inner, double *out, hipStream_t s, bool by_index = false,
                 const int *roles = nullptr) {
  int maxlc = 0;
  for (int q = 0; q < cnt; ++q) maxlc = std::max(maxlc, probs[idx[q]]->lcb);
  std::vector<int> lvl;
  auto participants = [&](int l) {
    lvl.clear();
    for (int q = 0; q < cnt; ++q)
      if (l < probs[idx[q]]->lcb) lvl.push_back(idx[q]);
    return (int)lvl.size();
  };
  for (int it = 0; it < (ir ? inner : 1); ++it) {
    for (int l = 0; l < maxlc; ++l)
      if (participants(l))
        batch_down(probs, lvl.data(), (int)lvl.size(), l, ir, ir && it == 0, d_phis, s);
    batch_tail(probs, idx, cnt, ir, s);
    for (int l = maxlc - 1; l >= 0; --l)
      if (participants(l)) batch_up(probs, lvl.data(), (int)lvl.size(), l, ir, !ir, d_phis, s);
  }
  if (ir) {
    if (roles) {
      batch_ir_step(probs, idx, cnt, d_phis, roles, s);
    } else {
      batch_ir_update(probs, idx, cnt, d_phis, s);
      batch_ir_residual(probs, idx, cnt, d_phis, s);
    }
    batch_finalize(probs, idx, cnt, 0, kSlotRes, kRelCycle, out, s, by_index);
  } else {
    batch_finalize(probs, idx, cnt, 1, kSlotRes, kRelCycle, out, s, by_index);
  }
}

bool read_back(double *host, const double *dev, int cnt, hipStream_t s) {
  if (cnt == 0) return true;
  if (hipGetLastError() != hipSuccess) return false;
  if (hipMemcpyAsync(host, dev, cnt * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
    return false;
  return hipStreamSynchronize(s) == hipSuccess;
}

}  // namespace

extern "C" {

tomg_status tomg_solve_batch(tomg_problem *const *probs, double *const *d_phis, int32_t n,
                             double rel_tol, int32_t max_cycles, int32_t *cycles_out,
                             double *rel_out, tomg_status *status_out) {
  if (!probs || !d_phis || n < 0 || n > kMaxBatch) return TOMG_EINVAL;
  if (n == 0) return TOMG_OK;
  if (!(rel_tol > 0.0) || max_cycles < 0) return TOMG_EINVAL;
  std::vector<tomg_status> st(n, TOMG_OK);
  std::vector<int> cyc(n, 0);
  std::vector<double> rel(n, 0.0);
  if (!batch_uniform(probs, d_phis, n)) {
    // mixed configurations: solve one after another
    tomg_status first = TOMG_OK;
    for (int k = 0; k < n; ++k) {
      int32_t c = 0;
      double r = 0.0;
      tomg_status s = probs[k] ? solve(probs[k], d_phis[k], rel_tol, max_cycles, &c, &r)
                               : TOMG_EINVAL;
      if (cycles_out) cycles_out[k] = c;
      if (rel_out) rel_out[k] = r;
      if (status_out) status_out[k] = s;
      if (s != TOMG_OK && first == TOMG_OK) first = s;
    }
    return first;
  }
  tomg_problem *lead = probs[0];
  hipStream_t s = lead->stream;
  const bool ir = lead->cfg.precision == TOMG_FP32_IR;
  std::vector<int> act(n);
  for (int k = 0; k < n; ++k) act[k] = k;
  std::vector<double> hrel(n);
  std::vector<int> role(n, 0);
  int na = n;
  batch_coarse_inverse(probs, act.data(), na, s);
  batch_begin(probs, act.data(), na, d_phis, ir, lead->bout, s);
  if (!read_back(hrel.data(), lead->bout, na, s)) return TOMG_EDEVICE;
  while (true) {
    // retire finished problems
    int w = 0;
    for (int q = 0; q < na; ++q) {
      const int k = act[q];
      const double r = hrel[q];
      rel[k] = r;
      if (!std::isfinite(r)) {
        st[k] = TOMG_ENONFINITE;
      } else if (r <= rel_tol) {
        st[k] = TOMG_OK;
      } else if (cyc[k] >= max_cycles) {
        st[k] = TOMG_ENOCONV;
      } else {
        act[w++] = k;
      }
    }
    na = w;
    if (na == 0) break;
    for (int q = 0; q < na; ++q) role[act[q]] = cyc[act[q]] & 1;
    batch_cycle(probs, act.data(), na, d_phis, ir, lead->cfg.ir_inner_cycles, lead->bout, s,
                false, ir ? role.data() : nullptr);
    for (int q = 0; q < na; ++q) ++cyc[act[q]];
    if (!read_back(hrel.data(), lead->bout, na, s)) return TOMG_EDEVICE;
  }
  if (ir) {  // iterates left in the second arrays after an odd step count
    std::vector<int> odd;
    for (int k = 0; k < n; ++k)
      if (cyc[k] & 1) odd.push_back(k);
    if (!odd.empty()) {
      batch_copy_back(probs, odd.data(), (int)odd.size(), d_phis, s);
      if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return TOMG_EDEVICE;
    }
  }
  tomg_status first = TOMG_OK;
  for (int k = 0; k < n; ++k) {
    if (cycles_out) cycles_out[k] = cyc[k];
    if (rel_out) rel_out[k] = rel[k];
    if (status_out) status_out[k] = st[k];
    if (st[k] == TOMG_ENOCONV)
      fail(probs[k], TOMG_ENOCONV, "solve_batch: rel. residual %.3e after %d cycles", rel[k], cyc[k]);
    if (st[k] != TOMG_OK && first == TOMG_OK) first = st[k];
  }
  return first;
}

// Queues one continuous-batching step; relative residuals to out[k] (device)
// for input position k.
static tomg_status batch_enqueue(tomg_problem *const *probs, double *const *d_phis, int32_t n,
                                 const int32_t *fresh, double *out) {
  if (!batch_uniform(probs, d_phis, n)) {
    for (int k = 0; k < n; ++k)
      if (probs[k] && !probs[k]->ready) return fail(probs[k], TOMG_ESTATE, "batch_step before setup_coeffs");
    return TOMG_EINVAL;
  }
  tomg_problem *lead = probs[0];
  hipStream_t s = lead->stream;
  const bool ir = lead->cfg.precision == TOMG_FP32_IR;
  std::vector<int> fr, cy, all(n);
  for (int k = 0; k < n; ++k) (fresh[k] ? fr : cy).push_back(k);
  // coarsest inverses of setups queued without one: one launch for all
  for (int k = 0; k < n; ++k) all[k] = k;
  batch_coarse_inverse(probs, all.data(), n, s);
  if (!fr.empty()) batch_begin(probs, fr.data(), (int)fr.size(), d_phis, ir, out, s, true);
  if (!cy.empty())
    batch_cycle(probs, cy.data(), (int)cy.size(), d_phis, ir, lead->cfg.ir_inner_cycles, out, s,
                true);
  return hipGetLastError() == hipSuccess ? TOMG_OK : TOMG_EDEVICE;
}

tomg_status tomg_batch_step(tomg_problem *const *probs, double *const *d_phis, int32_t n,
                            const int32_t *fresh, double *rel_out) {
  if (!probs || !d_phis || !fresh || !rel_out || n < 0 || n > kMaxBatch) return TOMG_EINVAL;
  if (n == 0) return TOMG_OK;
  tomg_status st = batch_enqueue(probs, d_phis, n, fresh, probs[0]->bout);
  if (st != TOMG_OK) return st;
  return read_back(rel_out, probs[0]->bout, n, probs[0]->stream) ? TOMG_OK : TOMG_EDEVICE;
}

tomg_status tomg_batch_launch(tomg_problem *const *probs, double *const *d_phis, int32_t n,
                              const int32_t *fresh, double *d_rel_out) {
  if (!probs || !d_phis || !fresh || !d_rel_out || n < 0 || n > kMaxBatch) return TOMG_EINVAL;
  if (n == 0) return TOMG_OK;
  return batch_enqueue(probs, d_phis, n, fresh, d_rel_out);
}

tomg_status tomg_laplace_grid(tomg_problem *p, double *d_xp, double *d_yp, const uint8_t *d_mask,
                              const double *d_px, const double *d_py, double rel_tol,
                              int32_t max_cycles, int32_t *cycles_out) {
  if (!p || !d_xp || !d_yp) return TOMG_EINVAL;
  if (!(rel_tol > 0.0) || max_cycles < 0)
    return fail(p, TOMG_EINVAL, "laplace_grid: bad tol/max_cycles");
  if (stored_level0(p->cfg))
    return fail(p, TOMG_EINVAL, "laplace_grid: needs Dirichlet edges and the eq. 18 form");
  p->ready = false;
  p->unchecked = false;
  HIP_TRY(p, launch_set_slots(p, 1u << kSlotBadRhs, 0.0));
  HIP_TRY(p, launch_setup_identity(p, d_mask));
  HIP_TRY(p, launch_hierarchy(p));
  double h[kNumSlots];
  tomg_status s = read_scalars(p, h);
  if (s != TOMG_OK) return s;
  if (h[kSlotPivot] != 0.0) return fail(p, TOMG_EGEOMETRY, "laplace_grid: singular coarsest matrix");
  p->ready = true;
  int32_t c1 = 0, c2 = 0;
  double r1 = 0.0, r2 = 0.0;
  // the right-hand side of each coordinate's equation: its source, or zero
  // (setup left f = 0)
  const size_t fb = p->lv[0].n * sizeof(double);
  if (d_px) HIP_TRY(p, hipMemcpyAsync(p->f, d_px, fb, hipMemcpyDeviceToDevice, p->stream));
  s = solve(p, d_xp, rel_tol, max_cycles, &c1, &r1);
  if (s == TOMG_OK) {
    if (d_py)
      HIP_TRY(p, hipMemcpyAsync(p->f, d_py, fb, hipMemcpyDeviceToDevice, p->stream));
    else if (d_px)
      HIP_TRY(p, launch_zero(p, p->f, p->lv[0].n));
    s = solve(p, d_yp, rel_tol, max_cycles, &c2, &r2);
  }
  if (cycles_out) *cycles_out = c1 > c2 ? c1 : c2;
  return s;
}

tomg_status tomg_field(tomg_problem *p, const double *d_phi, const double *d_xp,
                       const double *d_yp, const double *d_jac, double *d_ex, double *d_ey) {
  if (!p || !d_phi || !d_ex || !d_ey) return TOMG_EINVAL;
  if (!d_jac && (!d_xp || !d_yp))
    return fail(p, TOMG_EINVAL, "field: need the node coordinates or the Jacobian");
  if (!d_jac && (p->cfg.nx < 3 || p->cfg.ny < 3))
    return fail(p, TOMG_EINVAL, "field: numeric Jacobian needs 3 nodes per side");
  HIP_TRY(p, launch_field(p, d_phi, d_xp, d_yp, d_jac, d_ex, d_ey));
  return TOMG_OK;
}

tomg_status tomg_level_shape(const tomg_problem *p, int32_t level, int32_t *nx, int32_t *ny) {
  if (!p || level < 0 || level >= p->L) return TOMG_EINVAL;
  if (nx) *nx = p->lv[level].nx;
  if (ny) *ny = p->lv[level].ny;
  return TOMG_OK;
}

tomg_status tomg_export(tomg_problem *p, int32_t what, int32_t level, void *d_out) {
  if (!p || !d_out || level < 0 || level >= p->L) return TOMG_EINVAL;
  const Level &v = p->lv[level];
  const void *src = nullptr;
  size_t bytes = 0;
  switch (what) {
    case TOMG_FIELD_EXX: src = level == 0 ? p->exx : nullptr; bytes = v.n * 8; break;
    case TOMG_FIELD_EXY: src = level == 0 ? p->exy : nullptr; bytes = v.n * 8; break;
    case TOMG_FIELD_EYY: src = level == 0 ? p->eyy : nullptr; bytes = v.n * 8; break;
    case TOMG_FIELD_DET: src = level == 0 ? p->det : nullptr; bytes = v.n * 8; break;
    case TOMG_FIELD_RHS: src = level == 0 ? p->f : v.b; bytes = v.n * 8; break;
    case TOMG_FIELD_DIR: src = v.dir; bytes = v.n; break;
    case TOMG_FIELD_STENCIL: src = v.st; bytes = 9 * v.n * 8; break;  // level 0: Neumann only
    case TOMG_FIELD_X: src = level > 0 ? v.x : nullptr; bytes = v.n * 8; break;
    default: break;
  }
  if (!src) return fail(p, TOMG_EINVAL, "export: no array %d on level %d", what, level);
  HIP_TRY(p, hipMemcpyAsync(d_out, src, bytes, hipMemcpyDeviceToDevice, p->stream));
  return TOMG_OK;
}

tomg_status tomg_smooth(tomg_problem *p, double *d_phi, int32_t sweeps) {
  if (!p || !d_phi || sweeps < 0) return TOMG_EINVAL;
  if (!p->ready) return fail(p, TOMG_ESTATE, "smooth before setup_coeffs");
  HIP_TRY(p, launch_smooth0(p, d_phi, sweeps));
  return TOMG_OK;
}

tomg_status tomg_residual(tomg_problem *p, const double *d_phi, double *d_r) {
  if (!p || !d_phi || !d_r) return TOMG_EINVAL;
  if (!p->ready) return fail(p, TOMG_ESTATE, "residual before setup_coeffs");
  HIP_TRY(p, launch_residual0(p, d_phi, d_r));
  return TOMG_OK;
}

tomg_status tomg_profile(tomg_problem *p, int32_t enable) {
  if (!p) return TOMG_EINVAL;
  if (enable) {
    for (int kind = 0; kind < tomg_problem::kProfKinds; ++kind) {
      for (int e = 0; e < tomg_problem::kMaxEv; ++e)
        for (int q = 0; q < 2; ++q)
          if (!p->ev[kind][e][q]) HIP_TRY(p, hipEventCreate(&p->ev[kind][e][q]));
      p->nev[kind] = 0;
      p->prof_ms[kind] = 0.0;
      p->prof_cnt[kind] = 0.0;
    }
    p->prof = true;
  } else {
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    prof_harvest(p);
    p->prof = false;
  }
  return TOMG_OK;
}

tomg_status tomg_profile_read(tomg_problem *p, double *out) {
  if (!p || !out) return TOMG_EINVAL;
  HIP_TRY(p, hipStreamSynchronize(p->stream));
  prof_harvest(p);
  out[0] = p->prof_ms[0];
  out[1] = p->prof_cnt[0];
  out[2] = p->prof_ms[1];
  out[3] = p->prof_cnt[1];
  out[4] = p->prof_ms[2];
  out[5] = p->prof_cnt[2];
  return TOMG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Solve without any allocation (tomg_solve_noalloc)
// ---------------------------------------------------------------------------

namespace {

constexpr size_t kNoallocBytes = size_t(TOMG_NOALLOC_MAX_BYTES);

// The workspace of tomg_solve_noalloc.  Every GPU the library runs on holds
// its own copy of this array until the process ends.  In host code the name
// stands for a host-side shadow, not a device address: kernels and copies get
// the address hipGetSymbolAddress returned for the current device.
static __device__ __align__(256) char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array, looked up once per device
// (with that device current).
hipError_t scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr || ((uintptr_t)ptr) % 256 != 0) return hipErrorInvalidValue;
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

void set_err(char *err, size_t len, const char *msg) {
  if (err && len > 0) snprintf(err, len, "%s", msg);
}

}  // namespace

extern "C" {

tomg_status tomg_solve_noalloc(const tomg_config *cfg, const double *d_xp, const double *d_yp,
                               const double *d_jac, const double *d_eps_phys,
                               const double *d_rho_phys, const uint8_t *d_mask, double *d_phi,
                               double rel_tol, int32_t max_cycles, void *stream,
                               int32_t *cycles_out, double *rel_res_out, char *err,
                               size_t err_len) {
  set_err(err, err_len, "");
  if (!cfg || !d_phi) {
    set_err(err, err_len, "solve_noalloc: null configuration or phi");
    return TOMG_EINVAL;
  }
  Layout lay;
  if (!make_layout(*cfg, &lay)) {
    set_err(err, err_len, "solve_noalloc: invalid configuration");
    return TOMG_EINVAL;
  }
  if (lay.total > kNoallocBytes) {
    char msg[160];
    snprintf(msg, sizeof msg,
             "solve_noalloc: the problem needs %zu bytes of workspace, more than the "
             "static %zu",
             lay.total, kNoallocBytes);
    set_err(err, err_len, msg);
    return TOMG_ENOMEM;
  }
  void *ws = nullptr;
  if (scratch_address(&ws) != hipSuccess) {
    set_err(err, err_len, "solve_noalloc: the static workspace has no device address");
    return TOMG_EDEVICE;
  }
  // the problem state lives on this call's stack; the device work it queues
  // ends before the call returns (solve synchronises the stream)
  tomg_problem p;
  tomg_status s = TOMG_OK;
  if (init_problem(&p, cfg, lay, ws, kNoallocBytes, stream) != hipSuccess) {
    set_err(err, err_len, "solve_noalloc: launch failed");
    return TOMG_EDEVICE;
  }
  s = setup_coeffs(&p, d_xp, d_yp, d_jac, d_eps_phys, d_rho_phys, d_mask);
  if (s == TOMG_OK) s = solve(&p, d_phi, rel_tol, max_cycles, cycles_out, rel_res_out);
  if (s != TOMG_OK) {
    // setup_coeffs and solve leave their own message
    set_err(err, err_len, p.err);
    (void)hipStreamSynchronize(p.stream);  // no queued work outlives the stack state
  }
  destroy_events(&p);
  return s;
}

tomg_status tomg_copy_probe(const void *d_src, void *d_dst, size_t bytes, void *stream) {
  if (!d_src || !d_dst || bytes % 16 || ((uintptr_t)d_src % 16) || ((uintptr_t)d_dst % 16))
    return TOMG_EINVAL;
  return launch_copy_probe(d_src, d_dst, bytes, (hipStream_t)stream) == hipSuccess ? TOMG_OK
                                                                                 : TOMG_EDEVICE;
}

}  // extern "C"

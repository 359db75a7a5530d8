/*
 * tomg — geometric multigrid for the coordinate-transformed Poisson equation
 * on a uniform computational grid, for AMD Instinct MI355X (gfx950).
 *
 * Method: Gautam & Paradkar, "Multigrid Poisson Solver for Complex Geometries
 * Using Finite Difference Method", arXiv 2602.01888.  A map from the uniform
 * computational grid (xi, eta) to the physical domain (x', y') with Jacobian
 * J = dx'/dxi (eq. 1) turns the physical problem div'(eps' grad' phi) = -rho'
 * into div(eps grad phi) = -rho on the uniform grid, with
 *   eps = det J * J^-1 eps' J^-T            (eq. 10; components eq. 12-15)
 *   rho = rho' det J                        (eq. 11)
 * and phi unchanged (eq. 6).  The 9-point central-difference discretisation
 * of the expanded equation (eq. 17-18, coefficients k1..k6) is solved by a
 * multigrid V-cycle (Section 3, eq. 19-24).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - A node field is an array of nx*ny values, row-major with x fastest:
 *    node (i, j) is element j*nx + i; i runs along xi (spacing dx), j along
 *    eta (spacing dy).  Doubles unless stated.
 *  - Pointers named d_* are device pointers (HIP global memory on the GPU the
 *    problem was created on).  Host pointers are named without prefix.
 *  - The caller owns every buffer: the workspace, phi and all inputs.  The
 *    library never allocates or frees device memory.
 *  - Every call enqueues its work on the problem's stream, in stream order.
 *    Calls that return host values (solve, residual_norm, setup_coeffs)
 *    synchronise that stream; vcycle and tomg_update_rhs do not.
 *  - The outer ring of nodes and the nodes flagged in the mask are Dirichlet
 *    nodes; their values are taken from phi and are never written.  The
 *    problem solved is
 *        (A phi)_c = f_c  at free nodes c,      phi_d = given at Dirichlet d,
 *    where A is the operator of eq. 18 and f = -rho' det J.
 *  - Errors are returned as tomg_status; nothing aborts and no exception
 *    crosses this interface.  tomg_last_error() describes the last failure.
 *  - Different problems may be used concurrently from different host threads
 *    on different streams; one problem must not be used concurrently.
 */
#ifndef TOMG_H
#define TOMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tomg_problem tomg_problem;

typedef enum {
  TOMG_OK = 0,
  TOMG_EINVAL = -1,     /* bad argument: NULL, sizes not coarsenable, tol <= 0 ... */
  TOMG_ENOMEM = -2,     /* workspace smaller than tomg_workspace_bytes() */
  TOMG_EGEOMETRY = -3,  /* det J <= 0 at a node other than the four corners, or a
                           singular coarsest-level matrix (no Dirichlet node) */
  TOMG_ENOCONV = -4,    /* max_cycles reached; phi holds the last iterate */
  TOMG_ENONFINITE = -5, /* NaN/Inf in the coefficients, the source or the residual */
  TOMG_EDEVICE = -6,    /* a HIP runtime call failed */
  TOMG_ESTATE = -7      /* call out of order (e.g. vcycle before setup_coeffs) */
} tomg_status;

enum { TOMG_FP64 = 0, TOMG_FP32_IR = 1 };
enum { TOMG_GS4 = 0, TOMG_JACOBI = 1, TOMG_ZEBRA_X = 2, TOMG_ZEBRA_XY = 3 };

typedef struct {
  int32_t nx, ny;          /* nodes including the outer ring; (nx-1) and (ny-1)
                              must halve down to a coarsest grid of at most
                              9 x 9 nodes (e.g. 2^k + 1), nx, ny >= 5 */
  double xi0, eta0;        /* computational coordinates of node (0, 0) */
  double dx, dy;           /* computational spacings (dx != dy allowed) */
  int32_t precision;       /* TOMG_FP64, or TOMG_FP32_IR: FP32 V-cycles as the
                              inner solver of FP64 iterative refinement */
  int32_t nu1, nu2;        /* pre/post smoothing sweeps, 1..4 each (default 2, 2) */
  int32_t smoother;        /* TOMG_GS4 (four-colour Gauss-Seidel, default),
                              TOMG_JACOBI (damped Jacobi), or TOMG_ZEBRA_X
                              (zebra x-line Gauss-Seidel: even rows, then odd
                              rows, each solved exactly for its nodes with its
                              neighbours held -- for grids whose coupling along
                              i dominates; nx <= 4225), or TOMG_ZEBRA_XY (an
                              x-line sweep then a y-line sweep, for grids
                              anisotropic in both directions; the y-lines run as
                              x-lines of the transposed level, kept beside it;
                              nx, ny <= 4225, FP64, level-0 stencil stored).  The
                              latter three run the unfused cycle and cannot be
                              batched */
  double jacobi_omega;     /* damping of TOMG_JACOBI (default 0.8) */
  int32_t ir_inner_cycles; /* FP32 V-cycles per refinement step (default 2) */
  int32_t neumann;         /* edges with a homogeneous Neumann condition
                              (Section 4.1: zero normal derivative), a mask of
                              TOMG_NEU_W (i = 0), TOMG_NEU_E (i = nx-1),
                              TOMG_NEU_S (j = 0), TOMG_NEU_N (j = ny-1); default
                              0 (Dirichlet all round).  Nodes of these edges are
                              unknowns (a corner shared with a Dirichlet edge is
                              Dirichlet); eq. 18 is applied there with a mirror
                              ghost layer (phi and the tensor mirrored across
                              the edge, eps_xy with its sign changed) folded onto
                              the mirror nodes.  TOMG_FP64, or TOMG_FP32_IR (an
                              FP32 copy of the stored stencil feeds the inner
                              cycles; not with TOMG_ZEBRA_XY); the level-0
                              stencil is stored (9 planes more workspace), the
                              level passes run on it and the hierarchy ends in
                              a coarsest grid of at most 5 x 5 nodes; it is
                              batched only with other stored-stencil problems */
  int32_t flux;            /* operator form: 0 (default) the paper's expanded
                              eq. 18; 1 the symmetric flux (energy) form --
                              minus the gradient of a discrete energy with face
                              means of eps_xx, eps_yy and cell means of eps_xy
                              times cell-centred differences; symmetric, equal
                              to eq. 18 for constant eps, second order.  Like
                              Neumann edges it stores the level-0 stencil, takes
                              TOMG_FP64 or TOMG_FP32_IR, and is batched only
                              with other stored-stencil problems */
  int32_t coarse_op;       /* coarse-grid operator of eq. 23 (Section 3 does not
                              name one): TOMG_GALERKIN (default), the product
                              (1/4) P^T A P with the bilinear prolongation P
                              restricted to unknowns; or TOMG_REDISCRETIZE,
                              eq. 18 itself on each coarse grid (spacings 2^l
                              dx, 2^l dy) with the tensor of level 0 sampled at
                              the coarse nodes and the Dirichlet set sampled
                              likewise (plus the outer ring) -- Dirichlet edges
                              and the eq. 18 form only (neumann = 0, flux = 0,
                              not TOMG_ZEBRA_XY).  The discrete solution does
                              not depend on it; the convergence rate does */
  int32_t semi_levels;     /* semi-coarsening (an extension: Section 3 halves
                              both axes): the first semi_levels coarsenings of
                              the hierarchy halve axis semi_axis only and keep
                              every line of the other, the rest halve both.
                              The transfers are linear along the halved axis
                              and the identity along the kept one, with
                              restriction P^T / 2 and Galerkin coarse operators
                              (1/2) P^T A P.  For grids whose coupling along one
                              axis dominates (the semi-annulus of Section 4.1):
                              halving that axis alone keeps the four-colour
                              smoother's convergence independent of the
                              anisotropy.  Default 0; > 0 needs TOMG_GS4 and
                              TOMG_GALERKIN and runs the fused level passes down
                              to the coarsest solve; it is batched only with
                              problems of the same semi_levels and semi_axis */
  int32_t semi_axis;       /* axis halved by the semi-coarsened levels: 0 the
                              x axis (i, nx), 1 the y axis (j, ny) */
} tomg_config;

enum { TOMG_NEU_W = 1, TOMG_NEU_E = 2, TOMG_NEU_S = 4, TOMG_NEU_N = 8 };
enum { TOMG_GALERKIN = 0, TOMG_REDISCRETIZE = 1 };

/* Fills *cfg with the defaults above for an nx x ny grid of spacing dx, dy. */
void tomg_config_default(tomg_config *cfg, int32_t nx, int32_t ny, double dx, double dy);

/* Number of grid levels for cfg (>= 2), or 0 when the sizes do not coarsen
 * to a grid of at most 9 x 9 nodes. */
int32_t tomg_num_levels(const tomg_config *cfg);

/* Bytes of device workspace the problem needs (0 for an invalid config).
 * This is the problem's whole device footprint besides phi and the inputs,
 * so it is what a scheduler admits requests against. */
size_t tomg_workspace_bytes(const tomg_config *cfg);

/* Creates a problem on the current HIP device.  d_ws: caller-owned device
 * workspace of at least tomg_workspace_bytes(cfg) bytes, 256-byte aligned,
 * kept alive until tomg_destroy.  stream: a hipStream_t (NULL = the null
 * stream).  Host state only is allocated; the problem's launch arguments
 * are stored into the workspace by work queued on the stream (no host wait),
 * so a problem can be created while the stream is busy.  *out is NULL on
 * failure. */
tomg_status tomg_create(const tomg_config *cfg, void *d_ws, size_t ws_bytes, void *stream,
                        tomg_problem **out);

/* Frees the host state.  The caller frees the workspace afterwards. */
void tomg_destroy(tomg_problem *p);

/* Human-readable description of the last error on p (never NULL). */
const char *tomg_last_error(const tomg_problem *p);

/* Re-targets the problem to another stream (same device).  Waits on the
 * host for the problem's current stream first, so that the work already
 * queued there (the argument store of tomg_create, an asynchronous setup)
 * is complete before later calls run on the new stream. */
tomg_status tomg_set_stream(tomg_problem *p, void *stream);

/* Coefficient setup (eq. 1, 10-15, 11; numeric Jacobian eq. 39-42), then the
 * coarse-grid hierarchy.
 *   d_xp, d_yp : physical coordinates x'(xi_ij), y'(xi_ij); used for the
 *                numeric Jacobian (central differences inside, second-order
 *                one-sided differences on the edges).  Ignored when d_jac is
 *                given.
 *   d_jac      : nullable; 4 planes of nx*ny: dx'/dxi, dx'/deta, dy'/dxi,
 *                dy'/deta (J_xx, J_xy, J_yx, J_yy) for an analytic map.
 *   d_eps_phys : nullable; isotropic physical permittivity per node (NULL = 1).
 *   d_rho_phys : physical charge density rho' at the mapped nodes.
 *   d_mask     : nullable; uint8 per node, nonzero = interior Dirichlet node.
 * Inputs are read in stream order and may be freed once the call returns.
 * Returns TOMG_EGEOMETRY when det J <= 0 at any node but the four corners
 * (the operator never reads the corners), TOMG_ENONFINITE on NaN/Inf. */
tomg_status setup_coeffs(tomg_problem *p, const double *d_xp, const double *d_yp,
                         const double *d_jac, const double *d_eps_phys,
                         const double *d_rho_phys, const uint8_t *d_mask);

/* setup_coeffs (eq. 1, 10-15, 11; eq. 39-42) without its host
 * synchronisation: the same kernels are queued
 * on the problem's stream and the call returns at once, so that a caller
 * admitting new geometries while other solves run does not wait for the
 * device.  Argument errors are reported at once; the geometry checks
 * (det J, non-finite values, singular coarsest matrix) stay on the device and
 * are reported later: by the next solve or residual_norm (the status
 * setup_coeffs would have returned), by tomg_setup_check, and by
 * tomg_solve_batch / tomg_batch_step, which write a NaN relative residual for
 * a problem whose setup failed (tomg_solve_batch: status TOMG_ENONFINITE for
 * it; tomg_setup_check then names the cause).  The coarsest inverse is
 * launched with the problem's next cycle: a batched step launches those of
 * all the problems set up this way in one launch (one workgroup each).
 * Inputs must stay valid until the queued work has run (stream order). */
tomg_status tomg_setup_coeffs_async(tomg_problem *p, const double *d_xp, const double *d_yp,
                                    const double *d_jac, const double *d_eps_phys,
                                    const double *d_rho_phys, const uint8_t *d_mask);

/* ---- analytic maps and Gaussian sources evaluated on the device ---------- */
/* A request described by a few numbers instead of node arrays: the map from
 * the computational grid (xi_i = xi0 + i dx, eta_j = eta0 + j dy) to the
 * physical nodes, and a sum of Gaussian charge densities, evaluated by the
 * setup kernel itself (no input arrays, no host-to-device copy). */
enum {
  TOMG_MAP_SINUSOIDAL = 1,       /* x' = xi + amp s, y' = eta + amp s, s = sin(pi xi) sin(pi eta);
                                    analytic Jacobian; Dirichlet data 0 on the outer ring */
  TOMG_MAP_PERTURBED_CIRCLE = 2, /* radial stretch about (cx, cy): with r = |xi - c| and theta
                                    its polar angle, R(theta) = r_c + pert * sum_{k=2..5}
                                    coef[k-2] cos(k (theta - phase)); r' = r_in + (r - r_in)
                                    (R - r_in) / (r_c - r_in) on [r_in, r_c], r' = R + (r - r_c)
                                    (r_out - R) / (r_out - r_c) on (r_c, r_out], r' = r
                                    elsewhere, x' = c + r' (cos theta, sin theta); numeric
                                    Jacobian (eq. 39-42); nodes with r <= r_c are Dirichlet
                                    nodes of value value_in, the outer ring 0 */
  TOMG_MAP_POLAR = 3             /* x' = xi cos eta, y' = xi sin eta (eq. 29); analytic
                                    Jacobian; Dirichlet data value_in on the arc i = 0 and 0
                                    elsewhere on the ring */
};
#define TOMG_MAX_GAUSSIANS 16
typedef struct {
  int32_t kind;      /* TOMG_MAP_* */
  int32_t reserved;  /* set to zero */
  double amp;        /* TOMG_MAP_SINUSOIDAL */
  double cx, cy, r_in, r_c, r_out, pert, coef[4], phase;  /* TOMG_MAP_PERTURBED_CIRCLE */
  double value_in;   /* conductor (TOMG_MAP_PERTURBED_CIRCLE) or inner-arc (TOMG_MAP_POLAR) value */
} tomg_map_desc;
typedef struct {
  int32_t count;     /* Gaussians, 0 .. TOMG_MAX_GAUSSIANS */
  int32_t reserved;  /* set to zero */
  double sigma;      /* rho'(x') = sum_m amp[m] exp(-|x' - (cx[m], cy[m])|^2 / (2 sigma^2)) */
  double amp[TOMG_MAX_GAUSSIANS], cx[TOMG_MAX_GAUSSIANS], cy[TOMG_MAX_GAUSSIANS];
} tomg_source_desc;
enum { TOMG_SETUP_ASYNC = 1 };

/* setup_coeffs (eq. 1, 10-15, 11; eq. 39-42 for a numeric Jacobian) for a
 * map and source given by descriptors, evaluated node by node on the device
 * (physical permittivity 1).  d_phi_init (device, double[ny][nx], nullable)
 * receives the map's Dirichlet data and zeros elsewhere -- the initial guess
 * solve() takes.  flags: TOMG_SETUP_ASYNC queues the work without the host
 * check, as tomg_setup_coeffs_async; else as setup_coeffs.  The descriptors
 * are copied; tomg_update_rhs_desc re-uses the map.  TOMG_EINVAL for an
 * unknown map kind or flag, a perturbed circle without r_in < r_c < r_out,
 * count outside 0..TOMG_MAX_GAUSSIANS, or count > 0 with sigma <= 0. */
tomg_status tomg_setup_coeffs_desc(tomg_problem *p, const tomg_map_desc *map,
                                   const tomg_source_desc *src, double *d_phi_init,
                                   uint32_t flags);

/* tomg_update_rhs (eq. 11: f = -rho' det J) with the source given by a
 * descriptor, evaluated at the nodes of the map of the last
 * tomg_setup_coeffs_desc (TOMG_ESTATE if the problem was set up otherwise).
 * Asynchronous. */
tomg_status tomg_update_rhs_desc(tomg_problem *p, const tomg_source_desc *src);

/* The relative residual (the eq. 20 norm over the stopping test's
 * denominator, Section 3) of the problem's last solve, alone or batched:
 * out[0] at its start and out[c] after its cycle c.  *count (nullable)
 * receives the number of entries recorded (cycles + 1, at most 256); at
 * most cap are written to out (host memory, nullable when cap is 0).
 * Synchronises the problem's stream.  TOMG_EINVAL for a null problem or
 * cap < 0. */
tomg_status tomg_residual_history(tomg_problem *p, double *out, int32_t cap, int32_t *count);

/* Synchronises the problem's stream and returns the status of the checks of
 * the last setup (TOMG_OK, TOMG_EGEOMETRY or TOMG_ENONFINITE, as
 * setup_coeffs); a failed check makes the problem unusable until the next
 * setup, as for setup_coeffs.  TOMG_ESTATE before any setup. */
tomg_status tomg_setup_check(tomg_problem *p);

/* New source on the same geometry: f = -rho' det J from the stored det J
 * (eq. 11), without rebuilding the hierarchy.  Asynchronous. */
tomg_status tomg_update_rhs(tomg_problem *p, const double *d_rho_phys);

/* One V(nu1, nu2) cycle (Section 3, eq. 19-24) applied in place to d_phi.
 * Asynchronous.  For TOMG_FP32_IR problems this is one refinement step
 * (FP64 residual, ir_inner_cycles FP32 V-cycles, FP64 update). */
tomg_status vcycle(tomg_problem *p, double *d_phi);

/* Multigrid solve (Section 3): the V-cycle of eq. 19-24 repeated from the
 * initial guess in d_phi until the residual of eq. 20 has dropped by rel_tol.
 * The paper stops when the change of the iterate falls below a tolerance
 * (1e-10) in an unnamed norm; this library reads that test as the relative
 * residual of the discrete system,
 *     ||f - A phi||_2 / ||f - A phi0||_2 <= rel_tol   over free nodes,
 * where phi0 has the Dirichlet values of d_phi and zeros elsewhere (so the
 * measure does not depend on the initial guess).  When ||f - A phi0|| is 0
 * (phi0 already solves the problem) the denominator is the residual norm of
 * the initial guess instead.  Host outputs (nullable): *cycles_out cycles
 * (refinement steps for TOMG_FP32_IR) taken, *rel_res_out the final relative
 * residual.  Returns TOMG_ENOCONV with phi holding the last iterate if
 * max_cycles is reached, TOMG_ENONFINITE if the residual becomes NaN/Inf (a
 * non-finite initial residual leaves d_phi unchanged).  Cycles are queued in
 * groups behind a device-side convergence flag and the host reads the
 * residual between groups; cycles queued past convergence do nothing, so the
 * result, the cycle count and the residual history are those of a check
 * after every cycle.  Synchronises the problem's stream. */
tomg_status solve(tomg_problem *p, double *d_phi, double rel_tol, int32_t max_cycles,
                  int32_t *cycles_out, double *rel_res_out);

/* Residual norms of eq. 20 (r = f - A phi at free nodes, A the operator of
 * eq. 18): abs = ||r||_2; rel = abs / ||f - A phi0||_2 as in solve(), with
 * phi taken as the initial guess when that denominator is 0 (so rel is 1, or
 * 0 when abs is 0).  Host outputs, nullable; synchronises the problem's
 * stream. */
tomg_status residual_norm(tomg_problem *p, const double *d_phi, double *abs_out,
                          double *rel_out);

/* Solves n independent problems together, each by the multigrid solve of
 * Section 3 with solve()'s stopping test: each V-cycle stage is launched
 * once across all problems still iterating, on the first problem's stream,
 * and a problem leaves the batch as soon as it converges.  Per-problem host
 * outputs cycles_out[n], rel_out[n], status_out[n] (nullable).  Returns
 * TOMG_OK when every problem converged, else the first failing status.  The
 * per-node arithmetic is that of solve(), so after the same number of cycles
 * each iterate is bitwise the one solve() gives; a batched pass uses taller
 * row bands, so the level-0 residual norm is summed in another order and the
 * reported relative residual may differ from solve()'s in the last bits.
 * 1 <= n <= 4096.  Batched launches need
 * one cycle configuration (precision, nu1, nu2, four-colour smoother,
 * ir_inner_cycles, and one level-0 operator form: on-the-fly eq. 18 for all,
 * or a stored stencil -- Neumann edges, flux form -- for all); other mixes
 * are solved one after another.  Work the
 * caller queued for a problem on another stream must be ordered before the
 * call (the batch runs on the stream of probs[0]). */
tomg_status tomg_solve_batch(tomg_problem *const *probs, double *const *d_phis, int32_t n,
                             double rel_tol, int32_t max_cycles, int32_t *cycles_out,
                             double *rel_out, tomg_status *status_out);

/* One step of continuous batching (Section 3's V-cycle applied to a set of
 * problems that may change between steps).  For every k with fresh[k] != 0
 * the step only evaluates the initial norms: ||f - A phi0|| (phi0 = the
 * Dirichlet values of d_phis[k] and zero elsewhere) and the residual of the
 * iterate in d_phis[k].  Every other problem advances by one V-cycle
 * (TOMG_FP64) or one refinement step (TOMG_FP32_IR), in the same batched
 * launches as tomg_solve_batch.  rel_out[k] (host) receives each problem's
 * relative residual after the step; the caller decides when a problem
 * leaves.  A problem's sequence of steps gives bitwise the iterates of
 * solve() whatever other problems share the steps (and when they joined).  All problems need one
 * cycle configuration (else TOMG_EINVAL) and a completed setup_coeffs (else
 * TOMG_ESTATE); runs on the stream of probs[0] and synchronises it. */
tomg_status tomg_batch_step(tomg_problem *const *probs, double *const *d_phis, int32_t n,
                            const int32_t *fresh, double *rel_out);

/* tomg_batch_step (one V-cycle of Section 3, eq. 19-24, per problem) without
 * the host wait: the same step is queued on the
 * stream of probs[0] and the call returns; d_rel_out (double[n], device,
 * caller-owned) receives in stream order the relative residual of input k
 * at position k.  A server can then prepare the next step's problems on
 * the host (and queue their setup on the same stream) while this one runs,
 * and read d_rel_out after synchronising the stream or an event recorded
 * after this call.  The problems, their iterates and d_rel_out must stay
 * alive, and must not be freed or given to another call that reads them
 * from a different stream, until the step has run.  Arguments and errors
 * as tomg_batch_step (a null d_rel_out is TOMG_EINVAL); device faults of
 * the step surface at the next synchronising call. */
tomg_status tomg_batch_launch(tomg_problem *const *probs, double *const *d_phis, int32_t n,
                              const int32_t *fresh, double *d_rel_out);

/* Numerical grid generation (Section 4.2, eq. 36-37; Section 5.2 for an
 * embedded body): the node coordinates x'(xi, eta), y'(xi, eta) of the
 * physical grid solve Laplace's equation on the problem's computational
 * grid, with the boundary map as Dirichlet data.  On entry d_xp, d_yp
 * (double[ny][nx], device) hold the map on the outer ring and on the nodes
 * d_mask marks (uint8[ny][nx], device, nullable: 1 = the map is prescribed
 * there, such as the outline of an embedded square), and an initial guess
 * elsewhere (zeros will do); on return the other nodes solve the 5-point
 * Laplace equation to the relative residual rel_tol (as solve()),
 * *cycles_out (nullable) the larger of the two cycle counts.  d_px, d_py
 * (double[ny][nx], device, nullable) are source terms: the conclusion's
 * adaptive grids solve Poisson's equation lap x' = P, lap y' = Q on the
 * computational grid (the 5-point Laplacian, spacings dx, dy); along a grid
 * line x'' = P, so nodes cluster where P changes from negative to positive;
 * NULL means zero.  The
 * problem's operator is left as the identity tensor: call setup_coeffs
 * with the generated grid (d_xp, d_yp) before solving the physical
 * problem.  Errors as solve(); synchronises the problem's stream. */
tomg_status tomg_laplace_grid(tomg_problem *p, double *d_xp, double *d_yp, const uint8_t *d_mask,
                              const double *d_px, const double *d_py, double rel_tol,
                              int32_t max_cycles, int32_t *cycles_out);

/* Field recovery (eq. 2): the physical electric field E' = (J^T)^-1 E with
 * E = -grad phi on the uniform grid, at every node of the problem's grid.
 * grad phi uses the differences of eq. 39-42 (central inside, one-sided
 * second order on the edges).  The map is given as for setup_coeffs: d_jac
 * ([4][ny][nx] analytic partials, nullable) or the node coordinates d_xp,
 * d_yp (numeric Jacobian).  d_phi, d_ex, d_ey: double[ny][nx] on the device
 * (d_ex, d_ey written).  Does not need setup_coeffs.  Where det J = 0 (for
 * example the corner nodes of a square-to-disc map) the result is not
 * finite.  Asynchronous on the problem's stream. */
tomg_status tomg_field(tomg_problem *p, const double *d_phi, const double *d_xp,
                       const double *d_yp, const double *d_jac, double *d_ex, double *d_ey);

/* ---- allocation-free solve ---------------------------------------------- */
/* Largest workspace tomg_solve_noalloc offers (a 1025 x 1025 grid fits in
 * either precision). */
#define TOMG_NOALLOC_MAX_BYTES (128u * 1024u * 1024u)

/* For callers that cannot allocate memory -- code that must not call
 * hipMalloc or grow a heap, such as tight serving loops or harnesses that
 * forbid allocation: setup_coeffs followed by solve, on a problem whose
 * workspace is a static device array owned by the library
 * (TOMG_NOALLOC_MAX_BYTES bytes on each GPU it runs on, held until the
 * process ends) instead of a caller-owned one, with the problem's host state
 * on the call's stack.  The call allocates nothing, on the device or on the
 * host.  Arguments: cfg and stream as tomg_create (the current device's
 * array is used), the inputs as setup_coeffs, d_phi / rel_tol / max_cycles /
 * cycles_out / rel_res_out as solve; err (host, nullable) receives up to
 * err_len bytes of a message (empty on success).  A configuration whose
 * tomg_workspace_bytes exceeds TOMG_NOALLOC_MAX_BYTES is refused with
 * TOMG_ENOMEM before any device work.  Every call on a GPU uses that GPU's
 * one array, which keeps the last call's contents (each call initialises
 * what it reads): calls that overlap on one GPU -- from other host threads,
 * or a stream that has not finished an earlier call's work -- race.
 * Synchronises `stream`; results are those of tomg_create + setup_coeffs +
 * solve with the same arguments. */
tomg_status tomg_solve_noalloc(const tomg_config *cfg, const double *d_xp, const double *d_yp,
                               const double *d_jac, const double *d_eps_phys,
                               const double *d_rho_phys, const uint8_t *d_mask, double *d_phi,
                               double rel_tol, int32_t max_cycles, void *stream,
                               int32_t *cycles_out, double *rel_res_out, char *err,
                               size_t err_len);

/* ---- diagnostics: read back internal arrays (parity testing) ----------- */
enum {
  TOMG_FIELD_EXX = 0,    /* level 0, nx*ny doubles */
  TOMG_FIELD_EXY = 1,
  TOMG_FIELD_EYY = 2,
  TOMG_FIELD_DET = 3,
  TOMG_FIELD_RHS = 4,    /* level 0 f, or level l >= 1 coarse right-hand side */
  TOMG_FIELD_DIR = 5,    /* uint8 Dirichlet flags of level l */
  TOMG_FIELD_STENCIL = 6,/* level l >= 1, and level 0 with Neumann edges (the folded
                            operator): 9 planes, plane k = (dj+1)*3+(di+1) */
  TOMG_FIELD_X = 7       /* level l >= 1 correction from the last V-cycle */
};
/* Copies array `what` of level `level` into d_out (device); asynchronous. */
tomg_status tomg_export(tomg_problem *p, int32_t what, int32_t level, void *d_out);
/* Level (nx, ny) of a created problem (host outputs). */
tomg_status tomg_level_shape(const tomg_problem *p, int32_t level, int32_t *nx, int32_t *ny);
/* `sweeps` smoothing sweeps on level 0 in place (asynchronous). */
tomg_status tomg_smooth(tomg_problem *p, double *d_phi, int32_t sweeps);
/* d_r = f - A phi at free nodes, 0 at Dirichlet nodes (asynchronous). */
tomg_status tomg_residual(tomg_problem *p, const double *d_phi, double *d_r);

/* ---- measurement ----------------------------------------------------- */
/* enable != 0: bracket every level-0 down pass and up pass with HIP events
 * on the problem's stream; 0: stop.  Enabling resets the accumulators. */
tomg_status tomg_profile(tomg_problem *p, int32_t enable);
/* Synchronises the stream and returns out[6] = {total ms of level-0 down
 * passes, their count, total ms of level-0 up passes, their count, total ms
 * of the chained level-0 passes of FP32 inner cycles (the up pass of one
 * cycle and the down pass of the next in one launch), their count} since
 * tomg_profile(p, 1). */
tomg_status tomg_profile_read(tomg_problem *p, double *out);
/* STREAM-style device copy of `bytes` bytes (multiple of 16, 16-byte aligned
 * pointers) on `stream`: the practical HBM ceiling measured beside the
 * solver. */
tomg_status tomg_copy_probe(const void *d_src, void *d_dst, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* TOMG_H */

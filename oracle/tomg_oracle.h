/*
 * CPU FP64 oracle for the coordinate-transformed Poisson multigrid
 * (Gautam & Paradkar, "Multigrid Poisson Solver for Complex Geometries Using
 * Finite Difference Method", arXiv 2602.01888).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the independent checker of the
 * GPU solver: only the test suite, the smoke check and the benchmark's CPU
 * baseline load it.  It shares no source with the GPU library.
 *
 * Conventions: every node field is a double array of nx*ny values with node
 * (i, j) at index j*nx + i (i along the computational x axis, spacing dx;
 * j along y, spacing dy).  A 9-point stencil is 9 planes of nx*ny doubles;
 * plane k = (dj+1)*3 + (di+1) holds the coefficient of the neighbour at
 * (i+di, j+dj): 0 SW, 1 S, 2 SE, 3 W, 4 centre, 5 E, 6 NW, 7 N, 8 NE.
 * A "dir" array (uint8, nx*ny) marks Dirichlet nodes (the outer ring of the
 * grid plus any interior mask); every other node is free.
 */
#ifndef TOMG_ORACLE_H
#define TOMG_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_GS4 = 0, ORC_GS_LEX = 1, ORC_JACOBI = 2, ORC_ZEBRA_X = 3, ORC_ZEBRA_XY = 4 };
/* Edges with a homogeneous Neumann condition (bit mask). */
enum { ORC_NEU_W = 1, ORC_NEU_E = 2, ORC_NEU_S = 4, ORC_NEU_N = 8 };

int orc_num_threads(void);
void orc_set_threads(int n);

/* Jacobian by central differences (eq. 39-42) in the interior and
 * second-order one-sided differences on the grid edges.  Needs nx, ny >= 3. */
/* E' = (J^T)^-1 (-grad phi) at every node (eq. 2). */
void orc_field(int nx, int ny, double dx, double dy, const double *phi, const double *jxx,
               const double *jxy, const double *jyx, const double *jyy, double *ex,
               double *ey);
int orc_jacobian_numeric(int nx, int ny, double dx, double dy, const double *xp,
                         const double *yp, double *jxx, double *jxy, double *jyx,
                         double *jyy);

/* Permittivity tensor on the computational grid (eq. 10, components eq. 12-15)
 * and det J.  eps_phys (nullable) is an isotropic physical permittivity. */
void orc_permittivity(size_t n, const double *jxx, const double *jxy,
                      const double *jyx, const double *jyy,
                      const double *eps_phys, double *exx, double *exy,
                      double *eyy, double *det);

/* 1 when det J > 0 at every node except the four grid corners, else 0. */
int orc_geometry_ok(int nx, int ny, const double *det);

/* Right-hand side f = -rho' det J (eq. 11, with div(eps grad phi) = -rho). */
void orc_rhs(size_t n, const double *rho_phys, const double *det, double *f);

/* Dirichlet set: outer ring plus mask (nullable). */
void orc_dirichlet_set(int nx, int ny, const uint8_t *mask, uint8_t *dir);
/* The same with the edges in `neumann` left free (zero normal derivative). */
void orc_dirichlet_set_bc(int nx, int ny, const uint8_t *mask, int neumann, uint8_t *dir);

/* The paper's 9-point operator (eq. 18 and its coefficients k1..k6) written
 * as an explicit stencil at every free node; identity rows at Dirichlet
 * nodes.  A free node on the outer ring (Neumann edge) takes eq. 18 with a
 * mirror ghost layer, folded onto the mirror nodes. */
void orc_fine_stencil(int nx, int ny, double dx, double dy, const double *exx,
                      const double *exy, const double *eyy, const uint8_t *dir,
                      double *st);

/* Symmetric flux (energy) form of the same operator (face means of eps_xx,
 * eps_yy; cell means of eps_xy with cell-centred differences); equal to
 * eq. 18 for constant eps.  Neumann ring nodes as orc_fine_stencil. */
void orc_flux_stencil(int nx, int ny, double dx, double dy, const double *exx,
                      const double *exy, const double *eyy, const uint8_t *dir, double *st);

void orc_apply(int nx, int ny, const double *st, const uint8_t *dir,
               const double *x, double *y);
void orc_residual(int nx, int ny, const double *st, const uint8_t *dir,
                  const double *x, const double *b, double *r);
double orc_norm2_free(int nx, int ny, const uint8_t *dir, const double *r);

void orc_smooth(int nx, int ny, const double *st, const uint8_t *dir, double *x,
                const double *b, int kind, int sweeps, double omega);

void orc_restrict_fw(int nxf, int nyf, const double *rf, int nxc, int nyc,
                     double *fc);
void orc_restrict_fw_bc(int nxf, int nyf, const double *rf, int nxc, int nyc,
                        const uint8_t *dirc, double *fc);
void orc_prolong_add(int nxc, int nyc, const double *ec, int nxf, int nyf,
                     const uint8_t *dirf, double *xf);
void orc_galerkin(int nxf, int nyf, const double *stf, const uint8_t *dirf,
                  int nxc, int nyc, double *stc, uint8_t *dirc);
/* Semi-coarsening (an extension: the paper halves both axes): the same
 * transfers and Galerkin product with a stride per axis, 2 for an axis that
 * is halved and 1 for one that keeps every fine line; P is linear along a
 * halved axis and the identity along a kept one, the restriction is
 * P^T / (sx sy) and the coarse operator (1 / (sx sy)) P^T A P.  Strides
 * (2, 2) give exactly the functions above.  dirc of orc_restrict_s is
 * nullable (then every coarse ring node gets zero). */
void orc_restrict_s(int nxf, int nyf, const double *rf, int nxc, int nyc, int sx, int sy,
                    const uint8_t *dirc, double *fc);
void orc_prolong_add_s(int nxc, int nyc, const double *ec, int nxf, int nyf, int sx, int sy,
                       const uint8_t *dirf, double *xf);
void orc_galerkin_s(int nxf, int nyf, const double *stf, const uint8_t *dirf, int nxc,
                    int nyc, int sx, int sy, double *stc, uint8_t *dirc);

/* Dense Gaussian elimination with partial pivoting; A (m*m, row-major) and
 * b are overwritten; the solution is left in b.  Returns 0, or -1 when a
 * pivot is exactly zero. */
int orc_dense_solve(int m, double *A, double *b);

/* Multigrid hierarchy. */
typedef struct orc_mg orc_mg;
/* Largest coarsest level (nodes) kept when halving stops above the usual
 * 9 x 9 (5 x 5 with Neumann edges) bound. */
#define ORC_MAX_COARSE_NODES 1024
int orc_levels(int nx, int ny, int *nxs, int *nys, int maxl);
int orc_levels_lim(int nx, int ny, int *nxs, int *nys, int maxl, int lim);
/* The first `semi` coarsenings halve axis `semi_axis` only (0: x, 1: y);
 * sxs/sys (nullable) receive the strides of each level's transfer. */
int orc_levels_semi(int nx, int ny, int semi, int axis, int *nxs, int *nys, int *sxs, int *sys,
                    int maxl, int lim);
orc_mg *orc_mg_create(int nx, int ny, double dx, double dy, const double *exx,
                      const double *exy, const double *eyy, const uint8_t *mask,
                      int nu1, int nu2, int smoother, double omega);
orc_mg *orc_mg_create_bc(int nx, int ny, double dx, double dy, const double *exx,
                         const double *exy, const double *eyy, const uint8_t *mask,
                         int neumann, int nu1, int nu2, int smoother, double omega);
orc_mg *orc_mg_create_op(int nx, int ny, double dx, double dy, const double *exx,
                         const double *exy, const double *eyy, const uint8_t *mask,
                         int neumann, int flux, int nu1, int nu2, int smoother, double omega);
/* As orc_mg_create_op, with the coarse operator chosen: coarse_op 0 the
 * Galerkin product (1/4) P^T A P with the Dirichlet-aware prolongation, 1
 * rediscretisation -- eq. 18 on each coarse grid with the tensor and the
 * Dirichlet set sampled at the coarse nodes (Dirichlet edges and the eq. 18
 * form only; NULL otherwise). */
orc_mg *orc_mg_create_full(int nx, int ny, double dx, double dy, const double *exx,
                           const double *exy, const double *eyy, const uint8_t *mask,
                           int neumann, int flux, int coarse_op, int nu1, int nu2, int smoother,
                           double omega);
/* As orc_mg_create_full with the first `semi` coarsenings along axis
 * `semi_axis` only (Galerkin coarse operators; NULL with rediscretisation). */
orc_mg *orc_mg_create_semi(int nx, int ny, double dx, double dy, const double *exx,
                           const double *exy, const double *eyy, const uint8_t *mask,
                           int neumann, int flux, int coarse_op, int semi, int semi_axis,
                           int nu1, int nu2, int smoother, double omega);
void orc_mg_destroy(orc_mg *mg);
int orc_mg_num_levels(const orc_mg *mg);
void orc_mg_level_shape(const orc_mg *mg, int l, int *nx, int *ny);
/* Strides of the transfer from level l to level l + 1. */
void orc_mg_level_strides(const orc_mg *mg, int l, int *sx, int *sy);
const double *orc_mg_stencil(const orc_mg *mg, int l);
const uint8_t *orc_mg_dir(const orc_mg *mg, int l);
void orc_mg_vcycle(orc_mg *mg, double *phi, const double *f);
double orc_mg_initial_residual(orc_mg *mg, const double *phi, const double *f);
/* V-cycles from phi (its Dirichlet values held) until the relative
 * residual ||f - A phi||_2 / ||f - A phi0||_2 over free nodes is <= rel_tol
 * (phi0: the Dirichlet values with zeros elsewhere; when that norm is 0 the
 * denominator is the residual norm of the starting phi).  Returns 0 when
 * converged, 1 when max_cycles was reached, 2 on a non-finite residual. */
int orc_mg_solve(orc_mg *mg, double *phi, const double *f, double rel_tol,
                 int max_cycles, int *cycles_out, double *rel_out,
                 double *hist, int hist_len);
/* Coarse-level data written by the last V-cycle (right-hand side and
 * correction at level l >= 1). */
const double *orc_mg_level_rhs(const orc_mg *mg, int l);
const double *orc_mg_level_x(const orc_mg *mg, int l);

/* Error norms of eq. 25-27 over all nx*ny nodes: out = {Linf, L2, L1}. */
void orc_error_norms(size_t n, const double *a, const double *b, double *out);

#ifdef __cplusplus
}
#endif
#endif

/*
 * CPU FP64 oracle for the coordinate-transformed Poisson multigrid
 * (arXiv 2602.01888).  TEST INFRASTRUCTURE ONLY: the test suite, the smoke
 * check and the benchmark's CPU-baseline leg are its only users.
 *
 * It follows the paper's statement directly:
 *   Section 2   : J = dx'/dxi (eq. 1), eps = det J J^-1 eps' J^-T (eq. 10,
 *                 components eq. 12-15), rho = rho' det J (eq. 11);
 *   Section 2.1 : the expanded equation eq. 17 discretised by central
 *                 differences into the 9-point update eq. 18 with k1..k6;
 *                 Gauss-Seidel at omega = 1 is the multigrid smoother;
 *   Section 3   : residual correction eq. 19-24 on a hierarchy of grids;
 *   Section 4   : error norms eq. 25-27; numeric Jacobian eq. 39-42.
 * Where the paper leaves a choice open, the reading taken is stated at the
 * function that makes it.  Loops are plain and unblocked on purpose.
 */
#include "tomg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ID(i, j, nx) ((size_t)(j) * (size_t)(nx) + (size_t)(i))
#define PLANE(st, k, n) ((st) + (size_t)(k) * (n))
#define ORC_MAXL 16

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the calling host thread's later parallel loops (the results do
 * not depend on it: the loops run over independent nodes). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Section 2: Jacobian, permittivity, charge                                 */
/* ------------------------------------------------------------------------ */

/* d/dxi of a node field along i: eq. 39/41 in the interior; at i = 0 and
 * i = nx-1 the second-order one-sided formulas (the paper does not say what
 * it does on the edges). */
static double d_along_i(const double *a, int nx, int i, int j, double h) {
  if (i == 0)
    return (-3.0 * a[ID(0, j, nx)] + 4.0 * a[ID(1, j, nx)] - a[ID(2, j, nx)]) / (2.0 * h);
  if (i == nx - 1)
    return (3.0 * a[ID(nx - 1, j, nx)] - 4.0 * a[ID(nx - 2, j, nx)] + a[ID(nx - 3, j, nx)]) /
           (2.0 * h);
  return (a[ID(i + 1, j, nx)] - a[ID(i - 1, j, nx)]) / (2.0 * h);
}

/* d/deta along j: eq. 40/42, same edge treatment. */
static double d_along_j(const double *a, int nx, int ny, int i, int j, double h) {
  if (j == 0)
    return (-3.0 * a[ID(i, 0, nx)] + 4.0 * a[ID(i, 1, nx)] - a[ID(i, 2, nx)]) / (2.0 * h);
  if (j == ny - 1)
    return (3.0 * a[ID(i, ny - 1, nx)] - 4.0 * a[ID(i, ny - 2, nx)] + a[ID(i, ny - 3, nx)]) /
           (2.0 * h);
  return (a[ID(i, j + 1, nx)] - a[ID(i, j - 1, nx)]) / (2.0 * h);
}

/* Field recovery (eq. 2 with E = -grad phi on the computational grid):
 * E' = (J^T)^-1 E.  grad phi by the same differences as the Jacobian (eq.
 * 39-42 in the interior, one-sided second order on the edges).  J given as
 * four planes jxx = dx'/dxi, jxy = dx'/deta, jyx = dy'/dxi, jyy = dy'/deta.
 * (J^T)^-1 = [[jyy, -jyx], [-jxy, jxx]] / det J. */
void orc_field(int nx, int ny, double dx, double dy, const double *phi, const double *jxx,
               const double *jxy, const double *jyx, const double *jyy, double *ex,
               double *ey) {
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t c = ID(i, j, nx);
      const double e1 = -d_along_i(phi, nx, i, j, dx); /* E = -grad phi */
      const double e2 = -d_along_j(phi, nx, ny, i, j, dy);
      const double det = jxx[c] * jyy[c] - jxy[c] * jyx[c];
      ex[c] = (jyy[c] * e1 - jyx[c] * e2) / det;
      ey[c] = (-jxy[c] * e1 + jxx[c] * e2) / det;
    }
}

int orc_jacobian_numeric(int nx, int ny, double dx, double dy, const double *xp,
                         const double *yp, double *jxx, double *jxy, double *jyx,
                         double *jyy) {
  if (nx < 3 || ny < 3) return -1;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t c = ID(i, j, nx);
      jxx[c] = d_along_i(xp, nx, i, j, dx);     /* dx'/dxi  (eq. 39) */
      jxy[c] = d_along_j(xp, nx, ny, i, j, dy); /* dx'/deta (eq. 40) */
      jyx[c] = d_along_i(yp, nx, i, j, dx);     /* dy'/dxi  (eq. 41) */
      jyy[c] = d_along_j(yp, nx, ny, i, j, dy); /* dy'/deta (eq. 42) */
    }
  return 0;
}

void orc_permittivity(size_t n, const double *jxx, const double *jxy,
                      const double *jyx, const double *jyy,
                      const double *eps_phys, double *exx, double *exy,
                      double *eyy, double *det) {
  for (size_t c = 0; c < n; ++c) {
    double D = jxx[c] * jyy[c] - jxy[c] * jyx[c];
    double s = eps_phys ? eps_phys[c] : 1.0;
    /* eq. 12, 13 (= eq. 14), 15 */
    exx[c] = s * (jyy[c] * jyy[c] + jxy[c] * jxy[c]) / D;
    exy[c] = s * (-jyy[c] * jyx[c] - jxy[c] * jxx[c]) / D;
    eyy[c] = s * (jyx[c] * jyx[c] + jxx[c] * jxx[c]) / D;
    det[c] = D;
  }
}

int orc_geometry_ok(int nx, int ny, const double *det) {
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int corner = (i == 0 || i == nx - 1) && (j == 0 || j == ny - 1);
      if (corner) continue;
      double D = det[ID(i, j, nx)];
      if (!(D > 0.0)) return 0;
    }
  return 1;
}

void orc_rhs(size_t n, const double *rho_phys, const double *det, double *f) {
  /* eq. 11 gives rho = rho' det J; the equation solved is
   * div(eps grad phi) = -rho (eq. 7 and 17 with E = -grad phi). */
  for (size_t c = 0; c < n; ++c) f[c] = -rho_phys[c] * det[c];
}

void orc_dirichlet_set(int nx, int ny, const uint8_t *mask, uint8_t *dir) {
  orc_dirichlet_set_bc(nx, ny, mask, 0, dir);
}

/* Boundary conditions of Section 4.1: the paper's semi-annulus has a zero
 * normal derivative on its two straight sides.  An edge named in `neumann`
 * (ORC_NEU_W: i = 0, ORC_NEU_E: i = nx-1, ORC_NEU_S: j = 0, ORC_NEU_N:
 * j = ny-1) carries free nodes; a node is Dirichlet when it lies on an edge
 * that is not Neumann (so a corner shared with a Dirichlet edge is
 * Dirichlet) or under the mask. */
void orc_dirichlet_set_bc(int nx, int ny, const uint8_t *mask, int neumann, uint8_t *dir) {
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int ring = (i == 0 && !(neumann & ORC_NEU_W)) || (i == nx - 1 && !(neumann & ORC_NEU_E)) ||
                 (j == 0 && !(neumann & ORC_NEU_S)) || (j == ny - 1 && !(neumann & ORC_NEU_N));
      dir[ID(i, j, nx)] = (uint8_t)(ring || (mask && mask[ID(i, j, nx)]));
    }
}

/* ------------------------------------------------------------------------ */
/* Section 2.1: the 9-point operator                                         */
/* ------------------------------------------------------------------------ */

/* At a free node the discrete equation is
 *   k1 phi_E + k3 phi_W + k4 phi_N + k5 phi_S
 *     + k6 (phi_NE - phi_NW - phi_SE + phi_SW) - k2 phi_C = f,
 * i.e. eq. 18 before the division by k2 (the printed update omits that
 * division from the neighbour terms; expanding eq. 17 by central differences
 * puts it on every term).  eps_yx = eps_xy (eq. 13 = eq. 14). */
/* Index reflected about the grid edge: -k below 0, 2(n-1) - k above n-1. */
static int reflect(int k, int n) { return k < 0 ? -k : (k > n - 1 ? 2 * (n - 1) - k : k); }

/* Tensor component at a node that may lie one node outside the grid: the
 * mirror image across the edge.  Under a reflection of one axis eps_xx and
 * eps_yy are even and eps_xy changes sign (odd = 1 for eps_xy). */
static double mirrored(const double *a, int nx, int ny, int i, int j, int odd) {
  int ri = reflect(i, nx), rj = reflect(j, ny);
  double s = (odd && (ri != i) != (rj != j)) ? -1.0 : 1.0;
  return s * a[ID(ri, rj, nx)];
}

/* Free node on the outer ring (a Neumann edge).  A zero normal derivative
 * is imposed by a mirror ghost layer: the ghost values of phi and of the
 * tensor are those of the node's mirror image across the edge (eps_xy with
 * its sign changed), eq. 18 is written with them, and each ghost
 * coefficient is then added to the coefficient of the mirror node. */
static void edge_stencil(int nx, int ny, double idx2, double idy2, double idxy,
                         const double *exx, const double *exy, const double *eyy, int i, int j,
                         double a[9]) {
  double k2 = 2.0 * (mirrored(exx, nx, ny, i, j, 0) * idx2 + mirrored(eyy, nx, ny, i, j, 0) * idy2);
  double gx = (mirrored(exx, nx, ny, i + 1, j, 0) - mirrored(exx, nx, ny, i - 1, j, 0)) * idx2 / 4.0 +
              (mirrored(exy, nx, ny, i, j + 1, 1) - mirrored(exy, nx, ny, i, j - 1, 1)) * idxy / 4.0;
  double gy = (mirrored(eyy, nx, ny, i, j + 1, 0) - mirrored(eyy, nx, ny, i, j - 1, 0)) * idy2 / 4.0 +
              (mirrored(exy, nx, ny, i + 1, j, 1) - mirrored(exy, nx, ny, i - 1, j, 1)) * idxy / 4.0;
  double ax = mirrored(exx, nx, ny, i, j, 0) * idx2, ay = mirrored(eyy, nx, ny, i, j, 0) * idy2;
  double k6 = mirrored(exy, nx, ny, i, j, 1) * idxy / 2.0;
  double g[9] = {k6, ay - gy, -k6, ax - gx, -k2, ax + gx, -k6, ay + gy, k6};
  for (int k = 0; k < 9; ++k) a[k] = 0.0;
  for (int dj = -1; dj <= 1; ++dj)
    for (int di = -1; di <= 1; ++di) {
      int ti = reflect(i + di, nx) - i, tj = reflect(j + dj, ny) - j;
      a[(tj + 1) * 3 + (ti + 1)] += g[(dj + 1) * 3 + (di + 1)];
    }
}

void orc_fine_stencil(int nx, int ny, double dx, double dy, const double *exx,
                      const double *exy, const double *eyy, const uint8_t *dir,
                      double *st) {
  size_t n = (size_t)nx * ny;
  memset(st, 0, 9 * n * sizeof(double));
  double idx2 = 1.0 / (dx * dx), idy2 = 1.0 / (dy * dy), idxy = 1.0 / (dx * dy);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t c = ID(i, j, nx);
      if (dir[c]) {
        PLANE(st, 4, n)[c] = 1.0;
        continue;
      }
      if (i == 0 || j == 0 || i == nx - 1 || j == ny - 1) {
        double a[9];
        edge_stencil(nx, ny, idx2, idy2, idxy, exx, exy, eyy, i, j, a);
        for (int k = 0; k < 9; ++k) PLANE(st, k, n)[c] = a[k];
        continue;
      }
      size_t e = ID(i + 1, j, nx), w = ID(i - 1, j, nx);
      size_t no = ID(i, j + 1, nx), so = ID(i, j - 1, nx);
      double k2 = 2.0 * (exx[c] * idx2 + eyy[c] * idy2);
      double gx = (exx[e] - exx[w]) * idx2 / 4.0 + (exy[no] - exy[so]) * idxy / 4.0;
      double gy = (eyy[no] - eyy[so]) * idy2 / 4.0 + (exy[e] - exy[w]) * idxy / 4.0;
      double k1 = exx[c] * idx2 + gx;
      double k3 = exx[c] * idx2 - gx;
      double k4 = eyy[c] * idy2 + gy;
      double k5 = eyy[c] * idy2 - gy;
      double k6 = exy[c] * idxy / 2.0;
      PLANE(st, 0, n)[c] = k6;  /* SW */
      PLANE(st, 1, n)[c] = k5;  /* S  */
      PLANE(st, 2, n)[c] = -k6; /* SE */
      PLANE(st, 3, n)[c] = k3;  /* W  */
      PLANE(st, 4, n)[c] = -k2; /* C  */
      PLANE(st, 5, n)[c] = k1;  /* E  */
      PLANE(st, 6, n)[c] = -k6; /* NW */
      PLANE(st, 7, n)[c] = k4;  /* N  */
      PLANE(st, 8, n)[c] = k6;  /* NE */
    }
}

/* Symmetric flux (energy) form of div(eps grad phi), an alternative to the
 * expanded eq. 18.  The operator is minus the gradient of the discrete
 * energy
 *   1/2 sum_xfaces exx_f (dphi)^2 / dx^2 + 1/2 sum_yfaces eyy_f (dphi)^2 / dy^2
 *     + sum_cells exy_c gx_c gy_c,
 * with face values the mean of the two nodes, cell values the mean of the
 * four corners and gx_c, gy_c the cell-centred differences of phi; its
 * matrix is therefore symmetric, and for constant eps it is eq. 18.  Free
 * ring nodes (Neumann edges) use the mirror ghost layer of edge_stencil. */
static void flux_stencil_at(int nx, int ny, double dx, double dy, const double *exx,
                            const double *exy, const double *eyy, int i, int j, double a[9]) {
  double g[9] = {0};
  double ixx = 1.0 / (dx * dx), iyy = 1.0 / (dy * dy), ixy = 1.0 / (dx * dy);
  double c0 = mirrored(exx, nx, ny, i, j, 0), d0 = mirrored(eyy, nx, ny, i, j, 0);
  double aw = 0.5 * (c0 + mirrored(exx, nx, ny, i - 1, j, 0)) * ixx;
  double ae = 0.5 * (c0 + mirrored(exx, nx, ny, i + 1, j, 0)) * ixx;
  double as = 0.5 * (d0 + mirrored(eyy, nx, ny, i, j - 1, 0)) * iyy;
  double an = 0.5 * (d0 + mirrored(eyy, nx, ny, i, j + 1, 0)) * iyy;
  g[3] += aw;
  g[5] += ae;
  g[1] += as;
  g[7] += an;
  g[4] -= aw + ae + as + an;
  /* the four cells with a corner at (i, j): x in [i+ci, i+ci+1], y in [j+cj, j+cj+1] */
  for (int cj = -1; cj <= 0; ++cj)
    for (int ci = -1; ci <= 0; ++ci) {
      double bxy = 0.25 * (mirrored(exy, nx, ny, i + ci, j + cj, 1) +
                           mirrored(exy, nx, ny, i + ci + 1, j + cj, 1) +
                           mirrored(exy, nx, ny, i + ci, j + cj + 1, 1) +
                           mirrored(exy, nx, ny, i + ci + 1, j + cj + 1, 1));
      int pn = -ci, qn = -cj; /* corner of (i, j) in the cell */
      for (int qm = 0; qm <= 1; ++qm)
        for (int pm = 0; pm <= 1; ++pm) {
          /* d^2 (gx gy) / d phi_n d phi_m, with d gx / d phi_(p,q) = (2p-1)/(2 dx) */
          double h = ((2 * pn - 1) * (2 * qm - 1) + (2 * pm - 1) * (2 * qn - 1)) * 0.25 * ixy;
          g[(cj + qm + 1) * 3 + (ci + pm + 1)] -= bxy * h;
        }
    }
  for (int k = 0; k < 9; ++k) a[k] = 0.0;
  for (int dj = -1; dj <= 1; ++dj)
    for (int di = -1; di <= 1; ++di) {
      int ti = reflect(i + di, nx) - i, tj = reflect(j + dj, ny) - j;
      a[(tj + 1) * 3 + (ti + 1)] += g[(dj + 1) * 3 + (di + 1)];
    }
}

void orc_flux_stencil(int nx, int ny, double dx, double dy, const double *exx,
                      const double *exy, const double *eyy, const uint8_t *dir, double *st) {
  size_t n = (size_t)nx * ny;
  memset(st, 0, 9 * n * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t c = ID(i, j, nx);
      if (dir[c]) {
        PLANE(st, 4, n)[c] = 1.0;
        continue;
      }
      double a[9];
      flux_stencil_at(nx, ny, dx, dy, exx, exy, eyy, i, j, a);
      for (int k = 0; k < 9; ++k) PLANE(st, k, n)[c] = a[k];
    }
}

/* Sum of the off-centre stencil terms at (i, j). */
static double offcentre(int nx, size_t n, const double *st, const double *x, int i, int j) {
  double s = 0.0;
  int ny = (int)(n / (size_t)nx);
  for (int dj = -1; dj <= 1; ++dj)
    for (int di = -1; di <= 1; ++di) {
      if (di == 0 && dj == 0) continue;
      /* a free node on a Neumann edge has no coefficient outside the grid */
      if (i + di < 0 || i + di >= nx || j + dj < 0 || j + dj >= ny) continue;
      int k = (dj + 1) * 3 + (di + 1);
      s += PLANE(st, k, n)[ID(i, j, nx)] * x[ID(i + di, j + dj, nx)];
    }
  return s;
}

void orc_apply(int nx, int ny, const double *st, const uint8_t *dir,
               const double *x, double *y) {
  size_t n = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t c = ID(i, j, nx);
      y[c] = dir[c] ? 0.0 : offcentre(nx, n, st, x, i, j) + PLANE(st, 4, n)[c] * x[c];
    }
}

/* Residual of eq. 20, r = b - A x, on free nodes; zero on Dirichlet nodes. */
void orc_residual(int nx, int ny, const double *st, const uint8_t *dir,
                  const double *x, const double *b, double *r) {
  size_t n = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t c = ID(i, j, nx);
      r[c] = dir[c] ? 0.0 : b[c] - (offcentre(nx, n, st, x, i, j) + PLANE(st, 4, n)[c] * x[c]);
    }
}

double orc_norm2_free(int nx, int ny, const uint8_t *dir, const double *r) {
  double s = 0.0;
  for (size_t c = 0; c < (size_t)nx * ny; ++c)
    if (!dir[c]) s += r[c] * r[c];
  return sqrt(s);
}

/* ------------------------------------------------------------------------ */
/* Smoothers (Section 2.1: Gauss-Seidel, i.e. omega = 1, smooths)            */
/* ------------------------------------------------------------------------ */

static void relax(int nx, size_t n, const double *st, double *x, const double *b, int i, int j) {
  size_t c = ID(i, j, nx);
  x[c] = (b[c] - offcentre(nx, n, st, x, i, j)) / PLANE(st, 4, n)[c];
}

/* Paper-faithful ordering: eq. 18 reads new values at i-1 (every j) and at
 * (i, j-1), i.e. an outer loop over i and an inner loop over j. */
static void sweep_lex(int nx, int ny, const double *st, const uint8_t *dir, double *x,
                      const double *b) {
  size_t n = (size_t)nx * ny;
  for (int i = 0; i < nx; ++i)
    for (int j = 0; j < ny; ++j)
      if (!dir[ID(i, j, nx)]) relax(nx, n, st, x, b, i, j);
}

/* Four-colour ordering: colour (i mod 2) + 2 (j mod 2), colours 0,1,2,3 in
 * turn.  No two nodes of one colour are 9-point neighbours, so each colour
 * is an independent set and the result does not depend on the order inside
 * a colour. */
static void sweep_gs4(int nx, int ny, const double *st, const uint8_t *dir, double *x,
                      const double *b) {
  size_t n = (size_t)nx * ny;
  for (int colour = 0; colour < 4; ++colour) {
    int pi = colour & 1, pj = colour >> 1;
#pragma omp parallel for schedule(static)
    for (int j = pj; j < ny; j += 2)
      for (int i = pi; i < nx; i += 2)
        if (!dir[ID(i, j, nx)]) relax(nx, n, st, x, b, i, j);
  }
}

/* Damped Jacobi: x <- x + omega (b - A x) / A_CC. */
static void sweep_jacobi(int nx, int ny, const double *st, const uint8_t *dir, double *x,
                         const double *b, double omega) {
  size_t n = (size_t)nx * ny;
  double *r = (double *)malloc(n * sizeof(double));
  orc_residual(nx, ny, st, dir, x, b, r);
  for (size_t c = 0; c < n; ++c)
    if (!dir[c]) x[c] += omega * r[c] / PLANE(st, 4, n)[c];
  free(r);
}

/* Zebra line Gauss-Seidel along x (an extension for anisotropic grids,
 * where the coupling along i dominates): the even rows j are relaxed first,
 * each solved exactly for its own nodes with the rows above and below held,
 * then the odd rows.  A row is a tridiagonal system over all its nodes: a
 * free node keeps its W, C, E coefficients and moves the six off-row terms
 * to the right-hand side; a Dirichlet node is the identity row holding its
 * value.  Solved by Thomas elimination (the rows are diagonally dominant). */
static void sweep_zebra_x(int nx, int ny, const double *st, const uint8_t *dir, double *x,
                          const double *b) {
  size_t n = (size_t)nx * ny;
  for (int parity = 0; parity < 2; ++parity) {
#pragma omp parallel
    {
      double *a = (double *)malloc(4 * (size_t)nx * sizeof(double));
      double *c = a + nx, *e = c + nx, *d = e + nx;
#pragma omp for schedule(static)
      for (int j = parity; j < ny; j += 2) {
        for (int i = 0; i < nx; ++i) {
          size_t q = ID(i, j, nx);
          if (dir[q]) {
            a[i] = 0.0;
            c[i] = 1.0;
            e[i] = 0.0;
            d[i] = x[q];
            continue;
          }
          a[i] = i > 0 ? PLANE(st, 3, n)[q] : 0.0;
          c[i] = PLANE(st, 4, n)[q];
          e[i] = i < nx - 1 ? PLANE(st, 5, n)[q] : 0.0;
          double s = b[q];
          for (int dj = -1; dj <= 1; dj += 2) {
            if (j + dj < 0 || j + dj >= ny) continue;
            for (int di = -1; di <= 1; ++di) {
              if (i + di < 0 || i + di >= nx) continue;
              s -= PLANE(st, (dj + 1) * 3 + (di + 1), n)[q] * x[ID(i + di, j + dj, nx)];
            }
          }
          d[i] = s;
        }
        /* Thomas: forward elimination, back substitution */
        for (int i = 1; i < nx; ++i) {
          double m = a[i] / c[i - 1];
          c[i] -= m * e[i - 1];
          d[i] -= m * d[i - 1];
        }
        x[ID(nx - 1, j, nx)] = d[nx - 1] / c[nx - 1];
        for (int i = nx - 2; i >= 0; --i)
          x[ID(i, j, nx)] = (d[i] - e[i] * x[ID(i + 1, j, nx)]) / c[i];
      }
      free(a);
    }
  }
}

/* The same along y: the even columns i, then the odd columns, each solved
 * exactly along j (S, C, N coefficients; the six off-column terms and b on
 * the right). */
static void sweep_zebra_y(int nx, int ny, const double *st, const uint8_t *dir, double *x,
                          const double *b) {
  size_t n = (size_t)nx * ny;
  for (int parity = 0; parity < 2; ++parity) {
#pragma omp parallel
    {
      double *a = (double *)malloc(4 * (size_t)ny * sizeof(double));
      double *c = a + ny, *e = c + ny, *d = e + ny;
#pragma omp for schedule(static)
      for (int i = parity; i < nx; i += 2) {
        for (int j = 0; j < ny; ++j) {
          size_t q = ID(i, j, nx);
          if (dir[q]) {
            a[j] = 0.0;
            c[j] = 1.0;
            e[j] = 0.0;
            d[j] = x[q];
            continue;
          }
          a[j] = j > 0 ? PLANE(st, 1, n)[q] : 0.0;
          c[j] = PLANE(st, 4, n)[q];
          e[j] = j < ny - 1 ? PLANE(st, 7, n)[q] : 0.0;
          double s = b[q];
          for (int di = -1; di <= 1; di += 2) {
            if (i + di < 0 || i + di >= nx) continue;
            for (int dj = -1; dj <= 1; ++dj) {
              if (j + dj < 0 || j + dj >= ny) continue;
              s -= PLANE(st, (dj + 1) * 3 + (di + 1), n)[q] * x[ID(i + di, j + dj, nx)];
            }
          }
          d[j] = s;
        }
        for (int j = 1; j < ny; ++j) {
          double m = a[j] / c[j - 1];
          c[j] -= m * e[j - 1];
          d[j] -= m * d[j - 1];
        }
        x[ID(i, ny - 1, nx)] = d[ny - 1] / c[ny - 1];
        for (int j = ny - 2; j >= 0; --j)
          x[ID(i, j, nx)] = (d[j] - e[j] * x[ID(i, j + 1, nx)]) / c[j];
      }
      free(a);
    }
  }
}

void orc_smooth(int nx, int ny, const double *st, const uint8_t *dir, double *x,
                const double *b, int kind, int sweeps, double omega) {
  for (int s = 0; s < sweeps; ++s) {
    if (kind == ORC_GS_LEX)
      sweep_lex(nx, ny, st, dir, x, b);
    else if (kind == ORC_ZEBRA_X)
      sweep_zebra_x(nx, ny, st, dir, x, b);
    else if (kind == ORC_ZEBRA_XY) {
      sweep_zebra_x(nx, ny, st, dir, x, b);
      sweep_zebra_y(nx, ny, st, dir, x, b);
    }
    else if (kind == ORC_JACOBI)
      sweep_jacobi(nx, ny, st, dir, x, b, omega);
    else
      sweep_gs4(nx, ny, st, dir, x, b);
  }
}

/* ------------------------------------------------------------------------ */
/* Section 3: grid transfers and the coarse operator                         */
/* ------------------------------------------------------------------------ */

/* Bilinear interpolation weight of a coarse node for a fine node at offset
 * d = fine index - 2 * coarse index along one axis. */
static double pw(int d) { return d == 0 ? 1.0 : (d == 1 || d == -1) ? 0.5 : 0.0; }

/* Semi-coarsening (not in the paper, which halves both axes): a coarse grid
 * may also be halved along one axis only, the other axis keeping every fine
 * line.  Each transfer below takes a stride per axis -- 2 for an axis that is
 * halved, 1 for one that is kept -- and the interpolation weight along an
 * axis is the linear weight pw for stride 2 and the identity for stride 1.
 * P is the tensor product of the two axis weights; the restriction is
 * P^T / (sx sy) (full weighting along the halved axes) and the coarse
 * operator (1 / (sx sy)) P^T A_h P, so that with both strides 2 every
 * formula below is the one of the full coarsening. */
static double tw(int s, int d) { return s == 2 ? pw(d) : (d == 0 ? 1.0 : 0.0); }
/* Coarse indices K of an axis of stride s with a non-zero weight at fine
 * index g: K = g/2 .. (g+1)/2 for stride 2, K = g for stride 1. */
static int klo(int s, int g) { return s == 2 ? g / 2 : g; }
static int khi(int s, int g) { return s == 2 ? (g + 1) / 2 : g; }

/* Restriction I_h^H = P^T / (sx sy) (the paper does not name one).  With
 * both strides 2 it is full weighting,
 * r_H(I,J) = (1/16) [4 r(2I,2J) + 2 (edge neighbours) + (corner neighbours)];
 * with one stride 1 it is full weighting along the halved axis alone,
 * (1/4) [r(2I-1) + 2 r(2I) + r(2I+1)] on the coarse node's fine line.
 * Interior coarse nodes take the sum; on the coarse outer ring a free node
 * (a Neumann edge, when dirc is given) sums over the fine nodes of its
 * support that lie inside the grid (the transpose of the prolongation,
 * which has no fine nodes outside), and every other ring node gets zero. */
void orc_restrict_s(int nxf, int nyf, const double *rf, int nxc, int nyc, int sx, int sy,
                    const uint8_t *dirc, double *fc) {
  const double scale = (double)(sx * sy);
  for (int J = 0; J < nyc; ++J)
    for (int I = 0; I < nxc; ++I) {
      double s = 0.0;
      int ring = (I == 0 || J == 0 || I == nxc - 1 || J == nyc - 1);
      if (!ring || (dirc && !dirc[ID(I, J, nxc)]))
        for (int dj = -1; dj <= 1; ++dj)
          for (int di = -1; di <= 1; ++di) {
            double w = tw(sx, di) * tw(sy, dj);
            if (w == 0.0) continue;
            int fi = sx * I + di, fj = sy * J + dj;
            if (fi < 0 || fj < 0 || fi >= nxf || fj >= nyf) continue;
            s += w / scale * rf[ID(fi, fj, nxf)];
          }
      fc[ID(I, J, nxc)] = s;
    }
}

/* Full weighting at coarse interior nodes, zero on the coarse outer ring. */
void orc_restrict_fw(int nxf, int nyf, const double *rf, int nxc, int nyc, double *fc) {
  orc_restrict_s(nxf, nyf, rf, nxc, nyc, 2, 2, NULL, fc);
}

/* Full weighting where the coarse outer ring may hold free nodes (a
 * Neumann edge). */
void orc_restrict_fw_bc(int nxf, int nyf, const double *rf, int nxc, int nyc,
                        const uint8_t *dirc, double *fc) {
  orc_restrict_s(nxf, nyf, rf, nxc, nyc, 2, 2, dirc, fc);
}

/* Prolongation I_H^h (bilinear for strides 2, 2; linear along the halved
 * axis for a semi-coarsened level) and the correction of eq. 24, applied at
 * free fine nodes only (Dirichlet values are never changed). */
void orc_prolong_add_s(int nxc, int nyc, const double *ec, int nxf, int nyf, int sx, int sy,
                       const uint8_t *dirf, double *xf) {
  (void)nyc;
  for (int j = 0; j < nyf; ++j)
    for (int i = 0; i < nxf; ++i) {
      if (dirf[ID(i, j, nxf)]) continue;
      double s = 0.0;
      for (int J = klo(sy, j); J <= khi(sy, j); ++J)
        for (int I = klo(sx, i); I <= khi(sx, i); ++I)
          s += tw(sx, i - sx * I) * tw(sy, j - sy * J) * ec[ID(I, J, nxc)];
      xf[ID(i, j, nxf)] += s;
    }
}

void orc_prolong_add(int nxc, int nyc, const double *ec, int nxf, int nyf,
                     const uint8_t *dirf, double *xf) {
  orc_prolong_add_s(nxc, nyc, ec, nxf, nyf, 2, 2, dirf, xf);
}

/* Coarse operator of eq. 23.  The paper does not say how A_H is formed; the
 * reading taken is the Galerkin product A_H = (1/(sx sy)) P^T A_h P with P
 * the prolongation of the level (bilinear for the full coarsening, so the
 * factor is 1/4) restricted to the unknowns: rows of P at fine Dirichlet
 * nodes are zero, and only coarse nodes that are not Dirichlet carry a
 * column.  A coarse node is Dirichlet when it lies on the coarse outer ring
 * or when every fine node it interpolates to is Dirichlet (its column of P
 * would be empty); such nodes get an identity row. */
void orc_galerkin_s(int nxf, int nyf, const double *stf, const uint8_t *dirf, int nxc,
                    int nyc, int sx, int sy, double *stc, uint8_t *dirc) {
  size_t nf = (size_t)nxf * nyf, nc = (size_t)nxc * nyc;
  const double scale = (double)(sx * sy);
  for (int J = 0; J < nyc; ++J)
    for (int I = 0; I < nxc; ++I) {
      /* on the ring the coarse node keeps the kind of the fine node it sits
       * on (Dirichlet, or free on a Neumann edge) */
      int d = (I == 0 || J == 0 || I == nxc - 1 || J == nyc - 1) &&
              dirf[ID(sx * I, sy * J, nxf)];
      if (!d) {
        int any_free = 0;
        for (int dj = -1; dj <= 1; ++dj)
          for (int di = -1; di <= 1; ++di) {
            if (tw(sx, di) * tw(sy, dj) == 0.0) continue;
            int fi = sx * I + di, fj = sy * J + dj;
            if (fi < 0 || fj < 0 || fi >= nxf || fj >= nyf) continue;
            if (!dirf[ID(fi, fj, nxf)]) any_free = 1;
          }
        d = !any_free;
      }
      dirc[ID(I, J, nxc)] = (uint8_t)d;
    }
  memset(stc, 0, 9 * nc * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int J = 0; J < nyc; ++J)
    for (int I = 0; I < nxc; ++I) {
      size_t C = ID(I, J, nxc);
      if (dirc[C]) {
        PLANE(stc, 4, nc)[C] = 1.0;
        continue;
      }
      double acc[9] = {0};
      /* row C of P^T: fine nodes f = (sx I + a, sy J + b) with weight
       * tw(sx, a) tw(sy, b) */
      for (int b = -1; b <= 1; ++b)
        for (int a = -1; a <= 1; ++a) {
          double wf = tw(sx, a) * tw(sy, b);
          if (wf == 0.0) continue;
          int fi = sx * I + a, fj = sy * J + b;
          if (fi < 0 || fj < 0 || fi >= nxf || fj >= nyf) continue;
          size_t f = ID(fi, fj, nxf);
          if (dirf[f]) continue;
          /* row f of A_h: neighbours g = f + (p, q) */
          for (int q = -1; q <= 1; ++q)
            for (int p = -1; p <= 1; ++p) {
              int gi = fi + p, gj = fj + q;
              if (gi < 0 || gj < 0 || gi >= nxf || gj >= nyf) continue;
              size_t g = ID(gi, gj, nxf);
              if (dirf[g]) continue;
              double a_fg = PLANE(stf, (q + 1) * 3 + (p + 1), nf)[f];
              /* column K of P: coarse nodes K with a weight at g */
              for (int KJ = klo(sy, gj); KJ <= khi(sy, gj); ++KJ)
                for (int KI = klo(sx, gi); KI <= khi(sx, gi); ++KI) {
                  int oi = KI - I, oj = KJ - J;
                  if (oi < -1 || oi > 1 || oj < -1 || oj > 1) continue;
                  if (dirc[ID(KI, KJ, nxc)]) continue;
                  double wg = tw(sx, gi - sx * KI) * tw(sy, gj - sy * KJ);
                  acc[(oj + 1) * 3 + (oi + 1)] += wf * a_fg * wg;
                }
            }
        }
      for (int k = 0; k < 9; ++k) PLANE(stc, k, nc)[C] = acc[k] / scale;
    }
}

void orc_galerkin(int nxf, int nyf, const double *stf, const uint8_t *dirf,
                  int nxc, int nyc, double *stc, uint8_t *dirc) {
  orc_galerkin_s(nxf, nyf, stf, dirf, nxc, nyc, 2, 2, stc, dirc);
}

int orc_dense_solve(int m, double *A, double *b) {
  for (int k = 0; k < m; ++k) {
    int p = k;
    for (int r = k + 1; r < m; ++r)
      if (fabs(A[(size_t)r * m + k]) > fabs(A[(size_t)p * m + k])) p = r;
    if (A[(size_t)p * m + k] == 0.0) return -1;
    if (p != k) {
      for (int c = 0; c < m; ++c) {
        double t = A[(size_t)k * m + c];
        A[(size_t)k * m + c] = A[(size_t)p * m + c];
        A[(size_t)p * m + c] = t;
      }
      double t = b[k];
      b[k] = b[p];
      b[p] = t;
    }
    for (int r = k + 1; r < m; ++r) {
      double l = A[(size_t)r * m + k] / A[(size_t)k * m + k];
      for (int c = k; c < m; ++c) A[(size_t)r * m + c] -= l * A[(size_t)k * m + c];
      b[r] -= l * b[k];
    }
  }
  for (int k = m - 1; k >= 0; --k) {
    double s = b[k];
    for (int c = k + 1; c < m; ++c) s -= A[(size_t)k * m + c] * b[c];
    b[k] = s / A[(size_t)k * m + k];
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Section 3: the V-cycle                                                    */
/* ------------------------------------------------------------------------ */

/* Grid hierarchy: halve while both node counts minus one are even and each
 * side keeps at least 3 nodes; always coarsen at least once, then keep
 * coarsening while either side exceeds 9 nodes.  A grid whose halving stops
 * above that (an odd number of intervals, as the 201 x 201 grid of Section
 * 4.1 reaches at 26 x 26) keeps that coarsest level when it has at most
 * ORC_MAX_COARSE_NODES nodes; its direct solve is then larger.  Returns the
 * number of levels, or 0 when neither holds. */
int orc_levels(int nx, int ny, int *nxs, int *nys, int maxl) {
  return orc_levels_lim(nx, ny, nxs, nys, maxl, 9);
}

/* The same with the coarsest side bounded by `lim` nodes.  With Neumann
 * edges the coarsest ring holds unknowns too, so the hierarchy is taken one
 * halving further, to at most 5 x 5 nodes, which keeps the direct coarsest
 * system as small as the all-Dirichlet 9 x 9 one (at most 49 unknowns
 * there, at most 25 here). */
int orc_levels_lim(int nx, int ny, int *nxs, int *nys, int maxl, int lim) {
  return orc_levels_semi(nx, ny, 0, 0, nxs, nys, NULL, NULL, maxl, lim);
}

/* The same with the first `semi` coarsenings halving one axis only (axis 0:
 * x, the node count nx; axis 1: y), each of them required (the grid is
 * refused when that axis cannot be halved); the rule above then goes on
 * from the last semi-coarsened grid.  sxs[l], sys[l] (nullable) receive
 * the strides of the transfer from level l to level l + 1. */
int orc_levels_semi(int nx, int ny, int semi, int axis, int *nxs, int *nys, int *sxs, int *sys,
                    int maxl, int lim) {
  int L = 1;
  nxs[0] = nx;
  nys[0] = ny;
  if (nx < 5 || ny < 5 || semi < 0 || axis < 0 || axis > 1) return 0;
  while (L < maxl) {
    int cx = nxs[L - 1], cy = nys[L - 1];
    int sx, sy;
    if (L - 1 < semi) {
      int c = axis == 0 ? cx : cy;
      if ((c - 1) % 2 != 0 || c < 5) return 0;
      sx = axis == 0 ? 2 : 1;
      sy = axis == 0 ? 1 : 2;
    } else {
      int can = ((cx - 1) % 2 == 0) && ((cy - 1) % 2 == 0) && cx >= 5 && cy >= 5;
      int want = (L == 1) || cx > lim || cy > lim;
      if (!(can && want)) break;
      sx = sy = 2;
    }
    nxs[L] = sx == 2 ? (cx - 1) / 2 + 1 : cx;
    nys[L] = sy == 2 ? (cy - 1) / 2 + 1 : cy;
    if (sxs) sxs[L - 1] = sx;
    if (sys) sys[L - 1] = sy;
    ++L;
  }
  if (L < 2 || L - 1 < semi) return 0;
  if ((nxs[L - 1] > lim || nys[L - 1] > lim) &&
      (long)nxs[L - 1] * nys[L - 1] > ORC_MAX_COARSE_NODES)
    return 0;
  return L;
}

struct orc_mg {
  int L, nu1, nu2, smoother;
  double omega;
  int nx[ORC_MAXL], ny[ORC_MAXL];
  int sx[ORC_MAXL], sy[ORC_MAXL]; /* strides of the transfer from level l to l + 1 */
  double *st[ORC_MAXL];
  uint8_t *dir[ORC_MAXL];
  double *x[ORC_MAXL], *b[ORC_MAXL], *r[ORC_MAXL];
  int m;        /* unknowns on the coarsest level */
  int *cidx;    /* coarsest node -> unknown index, or -1 */
  double *Ac;   /* coarsest matrix, m*m */
  double *work; /* m*m + m scratch */
};

orc_mg *orc_mg_create(int nx, int ny, double dx, double dy, const double *exx,
                      const double *exy, const double *eyy, const uint8_t *mask,
                      int nu1, int nu2, int smoother, double omega) {
  return orc_mg_create_bc(nx, ny, dx, dy, exx, exy, eyy, mask, 0, nu1, nu2, smoother, omega);
}

orc_mg *orc_mg_create_bc(int nx, int ny, double dx, double dy, const double *exx,
                         const double *exy, const double *eyy, const uint8_t *mask,
                         int neumann, int nu1, int nu2, int smoother, double omega) {
  return orc_mg_create_op(nx, ny, dx, dy, exx, exy, eyy, mask, neumann, 0, nu1, nu2, smoother,
                          omega);
}

orc_mg *orc_mg_create_op(int nx, int ny, double dx, double dy, const double *exx,
                         const double *exy, const double *eyy, const uint8_t *mask,
                         int neumann, int flux, int nu1, int nu2, int smoother, double omega) {
  return orc_mg_create_full(nx, ny, dx, dy, exx, exy, eyy, mask, neumann, flux, 0, nu1, nu2,
                            smoother, omega);
}

/* Rediscretised coarse level l (Section 3 gives eq. 23's coarse problem but
 * not its operator; the tensor is computed once on the fine grid and
 * sampled on the coarser ones): the coarse tensor is the fine tensor at the
 * coarse node's position -- node (I, J) of level l takes level l-1's value at
 * (2I, 2J) -- and so is the Dirichlet set (plus the outer ring); the
 * operator is then eq. 18 itself with the coarse spacings (twice the fine
 * ones). */
static void rediscretise_level(int nxf, int nyf, const double *exf, const double *eyf,
                               const double *ezf, const uint8_t *dirf, int nxc, int nyc,
                               double dxc, double dyc, double *exc, double *eyc, double *ezc,
                               uint8_t *dirc, double *stc) {
  (void)nyf;
  for (int J = 0; J < nyc; ++J)
    for (int I = 0; I < nxc; ++I) {
      size_t c = ID(I, J, nxc), f = ID(2 * I, 2 * J, nxf);
      exc[c] = exf[f];
      eyc[c] = eyf[f];
      ezc[c] = ezf[f];
      int ring = I == 0 || J == 0 || I == nxc - 1 || J == nyc - 1;
      dirc[c] = (uint8_t)(ring || dirf[f]);
    }
  orc_fine_stencil(nxc, nyc, dxc, dyc, exc, eyc, ezc, dirc, stc);
}

orc_mg *orc_mg_create_full(int nx, int ny, double dx, double dy, const double *exx,
                           const double *exy, const double *eyy, const uint8_t *mask,
                           int neumann, int flux, int coarse_op, int nu1, int nu2, int smoother,
                           double omega) {
  return orc_mg_create_semi(nx, ny, dx, dy, exx, exy, eyy, mask, neumann, flux, coarse_op, 0, 0,
                            nu1, nu2, smoother, omega);
}

orc_mg *orc_mg_create_semi(int nx, int ny, double dx, double dy, const double *exx,
                           const double *exy, const double *eyy, const uint8_t *mask,
                           int neumann, int flux, int coarse_op, int semi, int semi_axis,
                           int nu1, int nu2, int smoother, double omega) {
  /* rediscretisation applies eq. 18 on every level: Dirichlet edges and the
   * full coarsening only */
  if (coarse_op != 0 && (coarse_op != 1 || neumann != 0 || flux != 0 || semi != 0)) return NULL;
  orc_mg *mg = (orc_mg *)calloc(1, sizeof(orc_mg));
  mg->L = orc_levels_semi(nx, ny, semi, semi_axis, mg->nx, mg->ny, mg->sx, mg->sy, ORC_MAXL,
                          neumann ? 5 : 9);
  if (mg->L == 0) {
    free(mg);
    return NULL;
  }
  mg->nu1 = nu1;
  mg->nu2 = nu2;
  mg->smoother = smoother;
  mg->omega = omega;
  for (int l = 0; l < mg->L; ++l) {
    size_t n = (size_t)mg->nx[l] * mg->ny[l];
    mg->st[l] = (double *)calloc(9 * n, sizeof(double));
    mg->dir[l] = (uint8_t *)calloc(n, 1);
    mg->x[l] = (double *)calloc(n, sizeof(double));
    mg->b[l] = (double *)calloc(n, sizeof(double));
    mg->r[l] = (double *)calloc(n, sizeof(double));
  }
  orc_dirichlet_set_bc(nx, ny, mask, neumann, mg->dir[0]);
  if (flux)
    orc_flux_stencil(nx, ny, dx, dy, exx, exy, eyy, mg->dir[0], mg->st[0]);
  else
    orc_fine_stencil(nx, ny, dx, dy, exx, exy, eyy, mg->dir[0], mg->st[0]);
  if (coarse_op == 1) {
    /* the tensor of the level above, starting from the fine grid's */
    size_t n0 = (size_t)nx * ny;
    double *t[2][3];
    for (int q = 0; q < 2; ++q)
      for (int k = 0; k < 3; ++k) t[q][k] = (double *)malloc(n0 * sizeof(double));
    memcpy(t[0][0], exx, n0 * sizeof(double));
    memcpy(t[0][1], exy, n0 * sizeof(double));
    memcpy(t[0][2], eyy, n0 * sizeof(double));
    double hx = dx, hy = dy;
    for (int l = 1; l < mg->L; ++l) {
      int a = (l - 1) & 1, b = l & 1;
      hx *= 2.0;
      hy *= 2.0;
      rediscretise_level(mg->nx[l - 1], mg->ny[l - 1], t[a][0], t[a][1], t[a][2], mg->dir[l - 1],
                         mg->nx[l], mg->ny[l], hx, hy, t[b][0], t[b][1], t[b][2], mg->dir[l],
                         mg->st[l]);
    }
    for (int q = 0; q < 2; ++q)
      for (int k = 0; k < 3; ++k) free(t[q][k]);
  } else {
    for (int l = 1; l < mg->L; ++l)
      orc_galerkin_s(mg->nx[l - 1], mg->ny[l - 1], mg->st[l - 1], mg->dir[l - 1], mg->nx[l],
                     mg->ny[l], mg->sx[l - 1], mg->sy[l - 1], mg->st[l], mg->dir[l]);
  }
  /* coarsest dense system over its free nodes */
  int l = mg->L - 1, cx = mg->nx[l], cy = mg->ny[l];
  size_t nc = (size_t)cx * cy;
  mg->cidx = (int *)malloc(nc * sizeof(int));
  mg->m = 0;
  for (size_t c = 0; c < nc; ++c) mg->cidx[c] = mg->dir[l][c] ? -1 : mg->m++;
  mg->Ac = (double *)calloc((size_t)mg->m * mg->m + 1, sizeof(double));
  mg->work = (double *)calloc((size_t)mg->m * mg->m + mg->m + 1, sizeof(double));
  for (int J = 0; J < cy; ++J)
    for (int I = 0; I < cx; ++I) {
      int row = mg->cidx[ID(I, J, cx)];
      if (row < 0) continue;
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
          if (I + di < 0 || J + dj < 0 || I + di >= cx || J + dj >= cy) continue;
          int col = mg->cidx[ID(I + di, J + dj, cx)];
          if (col < 0) continue;
          mg->Ac[(size_t)row * mg->m + col] =
              PLANE(mg->st[l], (dj + 1) * 3 + (di + 1), nc)[ID(I, J, cx)];
        }
    }
  return mg;
}

void orc_mg_destroy(orc_mg *mg) {
  if (!mg) return;
  for (int l = 0; l < mg->L; ++l) {
    free(mg->st[l]);
    free(mg->dir[l]);
    free(mg->x[l]);
    free(mg->b[l]);
    free(mg->r[l]);
  }
  free(mg->cidx);
  free(mg->Ac);
  free(mg->work);
  free(mg);
}

int orc_mg_num_levels(const orc_mg *mg) { return mg->L; }
void orc_mg_level_shape(const orc_mg *mg, int l, int *nx, int *ny) {
  *nx = mg->nx[l];
  *ny = mg->ny[l];
}
void orc_mg_level_strides(const orc_mg *mg, int l, int *sx, int *sy) {
  *sx = mg->sx[l];
  *sy = mg->sy[l];
}
const double *orc_mg_stencil(const orc_mg *mg, int l) { return mg->st[l]; }
const uint8_t *orc_mg_dir(const orc_mg *mg, int l) { return mg->dir[l]; }
const double *orc_mg_level_rhs(const orc_mg *mg, int l) { return mg->b[l]; }
const double *orc_mg_level_x(const orc_mg *mg, int l) { return mg->x[l]; }

/* Coarsest level: solve A_H x = b exactly (the paper leaves the coarse
 * solver open; a direct solve is taken). */
static void coarsest_solve(orc_mg *mg, double *x, const double *b) {
  int l = mg->L - 1, cx = mg->nx[l], cy = mg->ny[l], m = mg->m;
  size_t nc = (size_t)cx * cy;
  double *A = mg->work, *rhs = mg->work + (size_t)m * m;
  memcpy(A, mg->Ac, (size_t)m * m * sizeof(double));
  for (size_t c = 0; c < nc; ++c)
    if (mg->cidx[c] >= 0) rhs[mg->cidx[c]] = b[c];
  orc_dense_solve(m, A, rhs);
  for (size_t c = 0; c < nc; ++c) x[c] = mg->cidx[c] >= 0 ? rhs[mg->cidx[c]] : 0.0;
}

/* One V(nu1, nu2) cycle at level l on (x, b): pre-smoothing, residual
 * (eq. 20), restriction to the coarse right-hand side (eq. 23), recursive
 * coarse solve from a zero guess, prolongation and correction (eq. 24),
 * post-smoothing. */
static void vcycle_level(orc_mg *mg, int l, double *x, const double *b) {
  int nx = mg->nx[l], ny = mg->ny[l];
  if (l == mg->L - 1) {
    coarsest_solve(mg, x, b);
    return;
  }
  orc_smooth(nx, ny, mg->st[l], mg->dir[l], x, b, mg->smoother, mg->nu1, mg->omega);
  orc_residual(nx, ny, mg->st[l], mg->dir[l], x, b, mg->r[l]);
  orc_restrict_s(nx, ny, mg->r[l], mg->nx[l + 1], mg->ny[l + 1], mg->sx[l], mg->sy[l],
                 mg->dir[l + 1], mg->b[l + 1]);
  memset(mg->x[l + 1], 0, (size_t)mg->nx[l + 1] * mg->ny[l + 1] * sizeof(double));
  vcycle_level(mg, l + 1, mg->x[l + 1], mg->b[l + 1]);
  orc_prolong_add_s(mg->nx[l + 1], mg->ny[l + 1], mg->x[l + 1], nx, ny, mg->sx[l], mg->sy[l],
                    mg->dir[l], x);
  orc_smooth(nx, ny, mg->st[l], mg->dir[l], x, b, mg->smoother, mg->nu2, mg->omega);
}

void orc_mg_vcycle(orc_mg *mg, double *phi, const double *f) { vcycle_level(mg, 0, phi, f); }

/* ||f - A phi0||_2 over free nodes with phi0 = phi on Dirichlet nodes and 0
 * on free nodes: the norm the stopping test divides by. */
double orc_mg_initial_residual(orc_mg *mg, const double *phi, const double *f) {
  int nx = mg->nx[0], ny = mg->ny[0];
  size_t n = (size_t)nx * ny;
  double *z = mg->x[0];
  for (size_t c = 0; c < n; ++c) z[c] = mg->dir[0][c] ? phi[c] : 0.0;
  orc_residual(nx, ny, mg->st[0], mg->dir[0], z, f, mg->r[0]);
  return orc_norm2_free(nx, ny, mg->dir[0], mg->r[0]);
}

/* Relative residual of the stopping test: ||r|| / ||f - A phi0||, phi0 the
 * Dirichlet data with zeros elsewhere.  When that norm is 0 (phi0 already
 * solves the problem) the denominator is r0, the residual norm of the
 * starting iterate, so a warm start is iterated until its own residual has
 * dropped by the tolerance; a zero residual is 0, a non-finite one stays
 * non-finite. */
static double rel_residual(double rn, double b0, double r0) {
  if (rn == 0.0) return 0.0;
  return rn / (b0 > 0.0 ? b0 : r0);
}

int orc_mg_solve(orc_mg *mg, double *phi, const double *f, double rel_tol,
                 int max_cycles, int *cycles_out, double *rel_out, double *hist,
                 int hist_len) {
  int nx = mg->nx[0], ny = mg->ny[0];
  double b0 = orc_mg_initial_residual(mg, phi, f);
  int cycles = 0;
  double rel;
  orc_residual(nx, ny, mg->st[0], mg->dir[0], phi, f, mg->r[0]);
  double rn = orc_norm2_free(nx, ny, mg->dir[0], mg->r[0]);
  const double r0 = rn;
  rel = rel_residual(rn, b0, r0);
  if (hist && hist_len > 0) hist[0] = rel;
  int status = 1;
  while (1) {
    if (!isfinite(rel)) {
      status = 2;
      break;
    }
    if (rel <= rel_tol) {
      status = 0;
      break;
    }
    if (cycles >= max_cycles) break;
    orc_mg_vcycle(mg, phi, f);
    ++cycles;
    orc_residual(nx, ny, mg->st[0], mg->dir[0], phi, f, mg->r[0]);
    rn = orc_norm2_free(nx, ny, mg->dir[0], mg->r[0]);
    rel = rel_residual(rn, b0, r0);
    if (hist && cycles < hist_len) hist[cycles] = rel;
  }
  *cycles_out = cycles;
  *rel_out = rel;
  return status;
}

void orc_error_norms(size_t n, const double *a, const double *b, double *out) {
  double linf = 0.0, s2 = 0.0, s1 = 0.0;
  for (size_t c = 0; c < n; ++c) {
    double e = fabs(a[c] - b[c]);
    if (e > linf) linf = e;
    s2 += e * e;
    s1 += e;
  }
  out[0] = linf;                    /* eq. 25 */
  out[1] = sqrt(s2 / (double)n);    /* eq. 26, N^2 = number of nodes */
  out[2] = s1 / (double)n;          /* eq. 27 */
}

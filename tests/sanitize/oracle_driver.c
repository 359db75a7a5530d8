/* Drives the oracle's C code over small problems so that a build with
 * -fsanitize=address,undefined checks its memory accesses and arithmetic:
 * setup (numeric Jacobian, permittivity, right-hand side), the operator,
 * smoothers, transfers, Galerkin products, the dense solve and full
 * multigrid solves with every smoother, Neumann edges, the flux form,
 * rediscretisation and a large (26 x 26) coarsest level.  Exits nonzero if
 * a solve fails to converge. */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "tomg_oracle.h"

static int failures = 0;

static void check(int ok, const char *what) {
  if (!ok) {
    fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

/* Sinusoidal map on [0,1]^2 with amplitude a, source rho, Dirichlet data g. */
static void problem(int n, double a, double *xp, double *yp, double *rho, double *phi0) {
  const double d = 1.0 / (n - 1);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      const double xi = i * d, eta = j * d, s = sin(M_PI * xi) * sin(M_PI * eta);
      const size_t c = (size_t)j * n + i;
      xp[c] = xi + a * s;
      yp[c] = eta + a * s;
      rho[c] = exp(-((xp[c] - 0.4) * (xp[c] - 0.4) + (yp[c] - 0.6) * (yp[c] - 0.6)) / 0.02);
      phi0[c] = (i == 0 || j == 0 || i == n - 1 || j == n - 1) ? xp[c] * yp[c] : 0.0;
    }
}

static void solve_case(int n, int neumann, int flux, int coarse_op, int smoother, double omega,
                       const char *name) {
  const size_t N = (size_t)n * n;
  const double d = 1.0 / (n - 1);
  double *xp = malloc(N * sizeof(double)), *yp = malloc(N * sizeof(double));
  double *rho = malloc(N * sizeof(double)), *phi = malloc(N * sizeof(double));
  double *J[4], *exx = malloc(N * sizeof(double)), *exy = malloc(N * sizeof(double));
  double *eyy = malloc(N * sizeof(double)), *det = malloc(N * sizeof(double));
  double *f = malloc(N * sizeof(double)), *ex = malloc(N * sizeof(double));
  double *ey = malloc(N * sizeof(double));
  for (int k = 0; k < 4; ++k) J[k] = malloc(N * sizeof(double));
  problem(n, 0.1, xp, yp, rho, phi);
  check(orc_jacobian_numeric(n, n, d, d, xp, yp, J[0], J[1], J[2], J[3]) == 0, "jacobian");
  orc_permittivity(N, J[0], J[1], J[2], J[3], NULL, exx, exy, eyy, det);
  check(orc_geometry_ok(n, n, det), "geometry");
  orc_rhs(N, rho, det, f);
  orc_mg *mg = orc_mg_create_full(n, n, d, d, exx, exy, eyy, NULL, neumann, flux, coarse_op, 2,
                                  2, smoother, omega);
  check(mg != NULL, name);
  if (mg) {
    int cycles = 0;
    double rel = 0.0, hist[8];
    const int st = orc_mg_solve(mg, phi, f, 1e-10, 400, &cycles, &rel, hist, 8);
    check(st == 0, name);
    orc_mg_vcycle(mg, phi, f);
    (void)orc_mg_initial_residual(mg, phi, f);
    for (int l = 1; l < orc_mg_num_levels(mg); ++l) {
      (void)orc_mg_level_rhs(mg, l);
      (void)orc_mg_level_x(mg, l);
    }
    orc_field(n, n, d, d, phi, J[0], J[1], J[2], J[3], ex, ey);
    double e[3];
    orc_error_norms(N, ex, ey, e);
    check(isfinite(e[0]), "field");
    orc_mg_destroy(mg);
  }
  for (int k = 0; k < 4; ++k) free(J[k]);
  free(xp); free(yp); free(rho); free(phi); free(exx); free(exy); free(eyy); free(det);
  free(f); free(ex); free(ey);
}

int main(void) {
  orc_set_threads(2);
  /* level rules, including a large coarsest level and refused grids */
  int a[16], b[16];
  check(orc_levels(201, 201, a, b, 16) == 4 && a[3] == 26, "levels 201");
  check(orc_levels(1001, 1001, a, b, 16) == 0, "levels 1001");
  check(orc_levels_lim(33, 17, a, b, 16, 5) > 0, "levels 33x17");
  /* dense solve with pivoting, and a singular matrix */
  double A[9] = {0, 2, 1, 1, 1, 0, 3, 0, 1}, r[3] = {3, 2, 4};
  check(orc_dense_solve(3, A, r) == 0, "dense");
  double Z[4] = {0, 0, 0, 0}, z[2] = {1, 1};
  check(orc_dense_solve(2, Z, z) == -1, "dense singular");
  /* every smoother, the flux form, Neumann edges, rediscretisation */
  solve_case(33, 0, 0, 0, 0, 0.8, "gs4");
  solve_case(33, 0, 0, 0, 1, 0.8, "jacobi");
  solve_case(33, 0, 0, 0, 2, 0.8, "zebra_x");
  solve_case(33, 0, 0, 0, 3, 0.8, "zebra_xy");
  solve_case(33, ORC_NEU_S | ORC_NEU_E, 0, 0, 0, 0.8, "neumann");
  solve_case(33, 0, 1, 0, 0, 0.8, "flux");
  solve_case(33, 0, 0, 1, 0, 0.8, "rediscretize");
  solve_case(51, 0, 0, 0, 0, 0.8, "coarsest 26x26");
  solve_case(17, ORC_NEU_W | ORC_NEU_E | ORC_NEU_S, 1, 0, 0, 0.8, "neumann flux");
  if (failures) return 1;
  printf("oracle driver: all cases ran\n");
  return 0;
}

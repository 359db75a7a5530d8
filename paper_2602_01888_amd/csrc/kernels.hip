// HIP kernels of the multigrid V-cycle for the coordinate-transformed
// Poisson equation (arXiv 2602.01888, Sections 2-3), for gfx950.
//
// Node (i, j) of an nx x ny level is element j*nx + i.  Level 0 applies the
// operator of eq. 18 directly from the permittivity tensor (eq. 12-15), so
// the six coefficients k1..k6 are formed in registers and never stored;
// coarse levels store a 9-point stencil (9 planes, plane k = (dj+1)*3+(di+1)).
//
// Every reduction runs on a fixed grid of kRedBlocks blocks and a fixed
// tree, so a residual norm is bitwise reproducible from run to run.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "tomg_internal.h"

namespace tomg {
namespace {

// ---------------------------------------------------------------------------
// Operators.  row(c, x, off, diag): (A x)_c = off + diag * x_c.
// ---------------------------------------------------------------------------

// Level 0: eq. 18 from the stored tensor.  k2 multiplies phi_C with a minus
// sign; k1, k3, k4, k5 the E, W, N, S neighbours; k6 the diagonal difference
// phi_NE - phi_NW - phi_SE + phi_SW (the cross derivative).
template <typename T>
struct EpsOp {
  const T *exx, *exy, *eyy;
  int nx;
  T cx, cy;    // 1/dx^2, 1/dy^2
  T qx, qy;    // 1/(4 dx^2), 1/(4 dy^2)
  T qxy, hxy;  // 1/(4 dx dy), 1/(2 dx dy)

  __device__ __forceinline__ void coefs(size_t c, T &k1, T &k3, T &k4, T &k5, T &k6,
                                        T &k2) const {
    const size_t s = (size_t)nx;
    const T ax = exx[c] * cx, ay = eyy[c] * cy;
    // first-derivative terms of eq. 17: (d eps_xx/dx + d eps_yx/dy) d phi/dx and
    // (d eps_yy/dy + d eps_xy/dx) d phi/dy, by central differences
    const T gx = (exx[c + 1] - exx[c - 1]) * qx + (exy[c + s] - exy[c - s]) * qxy;
    const T gy = (eyy[c + s] - eyy[c - s]) * qy + (exy[c + 1] - exy[c - 1]) * qxy;
    k1 = ax + gx;
    k3 = ax - gx;
    k4 = ay + gy;
    k5 = ay - gy;
    k6 = exy[c] * hxy;
    k2 = T(2) * (ax + ay);
  }
  __device__ __forceinline__ void row(size_t c, const T *x, T &off, T &diag) const {
    T k1, k3, k4, k5, k6, k2;
    coefs(c, k1, k3, k4, k5, k6, k2);
    const size_t s = (size_t)nx;
    off = k1 * x[c + 1] + k3 * x[c - 1] + k4 * x[c + s] + k5 * x[c - s] +
          k6 * ((x[c + s + 1] - x[c + s - 1]) - (x[c - s + 1] - x[c - s - 1]));
    diag = -k2;
  }
  __device__ __forceinline__ T diag(size_t c) const { return -T(2) * (exx[c] * cx + eyy[c] * cy); }
  __device__ __forceinline__ void full(size_t c, T a[9]) const {
    T k1, k3, k4, k5, k6, k2;
    coefs(c, k1, k3, k4, k5, k6, k2);
    a[0] = k6;  a[1] = k5; a[2] = -k6;
    a[3] = k3;  a[4] = -k2; a[5] = k1;
    a[6] = -k6; a[7] = k4; a[8] = k6;
  }
};

// Coarse levels: stored 9-point stencil.
template <typename T>
struct StOp {
  const T *st;
  size_t n;
  int nx;
  __device__ __forceinline__ void row(size_t c, const T *x, T &off, T &diag) const {
    const size_t s = (size_t)nx;
    off = st[c] * x[c - s - 1] + st[n + c] * x[c - s] + st[2 * n + c] * x[c - s + 1] +
          st[3 * n + c] * x[c - 1] + st[5 * n + c] * x[c + 1] + st[6 * n + c] * x[c + s - 1] +
          st[7 * n + c] * x[c + s] + st[8 * n + c] * x[c + s + 1];
    diag = st[4 * n + c];
  }
  __device__ __forceinline__ T diag(size_t c) const { return st[4 * n + c]; }
  __device__ __forceinline__ void full(size_t c, T a[9]) const {
    for (int k = 0; k < 9; ++k) a[k] = st[k * n + c];
  }
};

// Stored stencil on a level whose outer ring may hold free nodes (Neumann
// edges).  A free ring node has no coefficient outside the grid, so the
// neighbours it would read there are replaced by in-range nodes (the
// products with the zero coefficients vanish); loads never leave the array.
template <typename T>
struct StOpB {
  const T *st;
  size_t n;
  int nx, ny;
  __device__ __forceinline__ void row(size_t c, const T *x, T &off, T &diag) const {
    const int j = (int)(c / (size_t)nx), i = (int)(c - (size_t)j * nx);
    const size_t s = (size_t)nx;
    const size_t w = i > 0 ? c - 1 : c, e = i < nx - 1 ? c + 1 : c;
    const size_t ds = j > 0 ? s : 0, us = j < ny - 1 ? s : 0;
    off = st[c] * x[w - ds] + st[n + c] * x[c - ds] + st[2 * n + c] * x[e - ds] +
          st[3 * n + c] * x[w] + st[5 * n + c] * x[e] + st[6 * n + c] * x[w + us] +
          st[7 * n + c] * x[c + us] + st[8 * n + c] * x[e + us];
    diag = st[4 * n + c];
  }
  __device__ __forceinline__ T diag(size_t c) const { return st[4 * n + c]; }
  __device__ __forceinline__ void full(size_t c, T a[9]) const {
    for (int k = 0; k < 9; ++k) a[k] = st[k * n + c];
  }
};

template <typename T>
StOpB<T> st_op_b(const T *st, int nx, int ny) {
  StOpB<T> o;
  o.st = st;
  o.n = (size_t)nx * ny;
  o.nx = nx;
  o.ny = ny;
  return o;
}

template <typename T>
EpsOp<T> eps_op(const T *exx, const T *exy, const T *eyy, int nx, double dx, double dy) {
  EpsOp<T> o;
  o.exx = exx;
  o.exy = exy;
  o.eyy = eyy;
  o.nx = nx;
  o.cx = T(1.0 / (dx * dx));
  o.cy = T(1.0 / (dy * dy));
  o.qx = T(0.25 / (dx * dx));
  o.qy = T(0.25 / (dy * dy));
  o.qxy = T(0.25 / (dx * dy));
  o.hxy = T(0.5 / (dx * dy));
  return o;
}

template <typename T>
StOp<T> st_op(const T *st, int nx, int ny) {
  StOp<T> o;
  o.st = st;
  o.n = (size_t)nx * ny;
  o.nx = nx;
  return o;
}

// ---------------------------------------------------------------------------
// Block reductions (wave64 shuffles, then LDS across the block's waves).
// ---------------------------------------------------------------------------

template <int OP>
__device__ __forceinline__ double combine(double a, double b) {
  return OP == 0 ? a + b : (OP == 1 ? fmin(a, b) : fmax(a, b));
}

template <int OP>
__device__ double block_reduce(double v) {
  __shared__ double red[kRedThreads / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = combine<OP>(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    v = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v = combine<OP>(v, red[w]);
  }
  __syncthreads();
  return v;  // valid in thread 0
}

// Relative residual of the stopping test: v / ||f - A phi0|| (phi0: the
// Dirichlet values and zero elsewhere).  When that norm is 0 -- the zero
// interior start is already the solution -- the denominator is the residual
// norm r0 of the solve's starting iterate, so a warm start still iterates
// until its residual has dropped by the tolerance.  v = 0 gives 0; a
// non-finite v stays non-finite.
__device__ __forceinline__ double rel_residual(double v, double b0, double r0) {
  if (v == 0.0) return 0.0;
  return v / (b0 > 0.0 ? b0 : r0);
}

// The residual history after the scalar slots: entry 0 at the start of a
// solve, entry c after its cycle c (cycles counted in kSlotCycles, which
// the start of a batched solve resets; a single solve resets it itself).
__device__ __forceinline__ void record_history(double *scal, int rel, double r) {
  const int c = rel == kRelBegin ? 0 : (int)scal[kSlotCycles];
  if (c >= 0 && c < kHistMax) scal[kNumSlots + c] = r;
}

// One block: fixed-order reduction of n partials into out[0].
// OP 0 sum, 1 min, 2 max; do_sqrt takes the square root of the result.
// rel == kRelBegin (the initial norms of a solve): out[0] is also recorded as
// the starting iterate's residual scal[kSlotR0]; rel != kRelNone: the
// relative residual (rel_residual) into scal[kSlotRel] and its comparison
// with scal[kSlotTol] into scal[kSlotDone]; kRelCycle also counts a cycle.
// A nonzero *skip makes the launch a no-op.
template <int OP>
__global__ void k_finalize(const double *partials, int n, int stride, double *out, int do_sqrt,
                           double *scal, int rel, const double *skip) {
  if (skip && *skip != 0.0) return;
  double v = OP == 0 ? 0.0 : (OP == 1 ? INFINITY : -INFINITY);
  for (int k = threadIdx.x; k < n; k += blockDim.x) v = combine<OP>(v, partials[(size_t)k * stride]);
  v = block_reduce<OP>(v);
  if (threadIdx.x == 0) {
    if (do_sqrt) v = sqrt(v);
    out[0] = v;
    if (rel != kRelNone) {
      if (rel == kRelBegin) scal[kSlotR0] = v;
      const double r = rel_residual(v, scal[kSlotB0], scal[kSlotR0]);
      scal[kSlotRel] = r;
      // a non-finite start also stops cycles queued behind it
      scal[kSlotDone] = (r <= scal[kSlotTol] || (rel == kRelBegin && !isfinite(r))) ? 1.0 : 0.0;
      if (rel == kRelCycle) scal[kSlotCycles] += 1.0;
      record_history(scal, rel, r);
    }
  }
}

// scal[slot] = v for the slots named in a bit mask (a fill kernel rather
// than a memset, so that a captured stream records no memset node).
__global__ void k_set_slots(double *scal, unsigned mask, double v) {
  const int k = threadIdx.x;
  if (k < kNumSlots && ((mask >> k) & 1u)) scal[k] = v;
}

// ---------------------------------------------------------------------------
// Setup (eq. 1, 10-15, 11; numeric Jacobian eq. 39-42)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double d_i(const double *a, int nx, int i, size_t c, double inv2h) {
  if (i == 0) return (-3.0 * a[c] + 4.0 * a[c + 1] - a[c + 2]) * inv2h;
  if (i == nx - 1) return (3.0 * a[c] - 4.0 * a[c - 1] + a[c - 2]) * inv2h;
  return (a[c + 1] - a[c - 1]) * inv2h;
}
__device__ __forceinline__ double d_j(const double *a, int nx, int ny, int j, size_t c,
                                      double inv2h) {
  const size_t s = (size_t)nx;
  if (j == 0) return (-3.0 * a[c] + 4.0 * a[c + s] - a[c + 2 * s]) * inv2h;
  if (j == ny - 1) return (3.0 * a[c] - 4.0 * a[c - s] + a[c - 2 * s]) * inv2h;
  return (a[c + s] - a[c - s]) * inv2h;
}

// Grid-stride over the nodes in memory order, so that the whole grid of
// threads sweeps one contiguous window of the arrays.  When exx32 is given
// the FP32 copies of the tensor used by the inner solver of iterative
// refinement are written beside the FP64 fields.
__global__ void k_setup(int nx, int ny, double dx, double dy, const double *__restrict__ xp,
                        const double *__restrict__ yp, const double *__restrict__ jac,
                        const double *__restrict__ epsp, const double *__restrict__ rho,
                        const uint8_t *__restrict__ mask, double *__restrict__ exx,
                        double *__restrict__ exy, double *__restrict__ eyy,
                        double *__restrict__ det, double *__restrict__ f,
                        uint8_t *__restrict__ dir, float *__restrict__ exx32,
                        float *__restrict__ exy32, float *__restrict__ eyy32,
                        double *__restrict__ partials, int neumann) {
  const size_t n = (size_t)nx * ny;
  const double i2dx = 0.5 / dx, i2dy = 0.5 / dy;
  double mind = INFINITY, bad = 0.0;
  const bool small = n < (size_t(1) << 32);
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x) {
    {
      int i, j;
      if (small) {
        j = (int)((unsigned)c / (unsigned)nx);
        i = (int)((unsigned)c - (unsigned)j * (unsigned)nx);
      } else {
        j = (int)(c / nx);
        i = (int)(c - (size_t)j * nx);
      }
      double jxx, jxy, jyx, jyy;
      if (jac) {
        jxx = jac[c];
        jxy = jac[n + c];
        jyx = jac[2 * n + c];
        jyy = jac[3 * n + c];
      } else {
        jxx = d_i(xp, nx, i, c, i2dx);
        jxy = d_j(xp, nx, ny, j, c, i2dy);
        jyx = d_i(yp, nx, i, c, i2dx);
        jyy = d_j(yp, nx, ny, j, c, i2dy);
      }
      const double D = jxx * jyy - jxy * jyx;
      const double s = epsp ? epsp[c] : 1.0;
      const double vxx = s * (jyy * jyy + jxy * jxy) / D;
      const double vxy = s * (-jyy * jyx - jxy * jxx) / D;
      const double vyy = s * (jyx * jyx + jxx * jxx) / D;
      const double fv = -rho[c] * D;
      __builtin_nontemporal_store(vxx, exx + c);
      __builtin_nontemporal_store(vxy, exy + c);
      __builtin_nontemporal_store(vyy, eyy + c);
      __builtin_nontemporal_store(D, det + c);
      __builtin_nontemporal_store(fv, f + c);
      if (exx32) {
        exx32[c] = (float)vxx;
        exy32[c] = (float)vxy;
        eyy32[c] = (float)vyy;
      }
      // the ring is Dirichlet except on Neumann edges (a corner shared with
      // a Dirichlet edge stays Dirichlet)
      const bool ring = (i == 0 && !(neumann & TOMG_NEU_W)) ||
                        (i == nx - 1 && !(neumann & TOMG_NEU_E)) ||
                        (j == 0 && !(neumann & TOMG_NEU_S)) ||
                        (j == ny - 1 && !(neumann & TOMG_NEU_N));
      dir[c] = (uint8_t)(ring || (mask && mask[c]));
      // the operator never reads a Dirichlet corner; a corner between two
      // Neumann edges is an unknown and is checked like any other node
      const bool corner = ring && (i == 0 || i == nx - 1) && (j == 0 || j == ny - 1);
      if (!corner) {
        mind = fmin(mind, D);
        if (!isfinite(vxx) || !isfinite(vxy) || !isfinite(vyy) || !isfinite(fv)) bad += 1.0;
      }
    }
  }
  const double m = block_reduce<1>(mind);
  const double b = block_reduce<0>(bad);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = m;
    partials[2 * blockIdx.x + 1] = b;
  }
}

// Neumann edges: the level-0 operator written out as a 9-point stencil at
// every node (identity rows at Dirichlet nodes).  At a free node the
// coefficients are those of eq. 18 (k1..k6); at a free node of the outer
// ring the values outside the grid are ghosts, the mirror images across the
// edge (eps_xx, eps_yy mirrored, eps_xy mirrored with its sign changed, phi
// mirrored), so the coefficient of each ghost is added to that of the node
// it mirrors.  Memory-order grid stride.
__device__ __forceinline__ int mirror_index(int k, int n) {
  return k < 0 ? -k : (k > n - 1 ? 2 * (n - 1) - k : k);
}

__global__ void k_fold_stencil(EpsOp<double> op, int ny, const uint8_t *__restrict__ dir,
                               double *__restrict__ st, int flux) {
  const int nx = op.nx;
  const size_t n = (size_t)nx * ny;
  const bool small = n < (size_t(1) << 32);
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x) {
    int i, j;
    if (small) {  // 32-bit division where the index fits
      j = (int)((unsigned)c / (unsigned)nx);
      i = (int)((unsigned)c - (unsigned)j * (unsigned)nx);
    } else {
      j = (int)(c / (size_t)nx);
      i = (int)(c - (size_t)j * nx);
    }
    double a[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) a[k] = 0.0;
    if (dir[c]) {
      a[4] = 1.0;
    } else {
      // tensor component at (ii, jj), one node outside the grid at most
      auto ev = [&](const double *v, int ii, int jj, bool odd) {
        const int ri = mirror_index(ii, nx), rj = mirror_index(jj, ny);
        const double s = (odd && ((ri != ii) != (rj != jj))) ? -1.0 : 1.0;
        return s * v[(size_t)rj * nx + ri];
      };
      double g[9];
      if (flux) {
        // minus the gradient of the discrete energy: face means of eps_xx and
        // eps_yy on squared face differences, cell means of eps_xy on the
        // product of cell-centred differences (d gx / d phi at cell corner
        // (p, q) is (2p - 1) / (2 dx), d gy is (2q - 1) / (2 dy))
        const double c0 = op.exx[c], d0 = op.eyy[c];
        const double aw = 0.5 * (c0 + ev(op.exx, i - 1, j, false)) * op.cx;
        const double ae = 0.5 * (c0 + ev(op.exx, i + 1, j, false)) * op.cx;
        const double as = 0.5 * (d0 + ev(op.eyy, i, j - 1, false)) * op.cy;
        const double an = 0.5 * (d0 + ev(op.eyy, i, j + 1, false)) * op.cy;
#pragma unroll
        for (int k = 0; k < 9; ++k) g[k] = 0.0;
        g[3] = aw;
        g[5] = ae;
        g[1] = as;
        g[7] = an;
        g[4] = -(aw + ae + as + an);
#pragma unroll
        for (int cj = -1; cj <= 0; ++cj)
#pragma unroll
          for (int ci = -1; ci <= 0; ++ci) {
            const double bxy =
                0.25 * (ev(op.exy, i + ci, j + cj, true) + ev(op.exy, i + ci + 1, j + cj, true) +
                        ev(op.exy, i + ci, j + cj + 1, true) +
                        ev(op.exy, i + ci + 1, j + cj + 1, true));
            const int pn = -ci, qn = -cj;
#pragma unroll
            for (int qm = 0; qm <= 1; ++qm)
#pragma unroll
              for (int pm = 0; pm <= 1; ++pm) {
                const double h =
                    ((2 * pn - 1) * (2 * qm - 1) + (2 * pm - 1) * (2 * qn - 1)) * op.qxy;
                g[(cj + qm + 1) * 3 + ci + pm + 1] -= bxy * h;
              }
          }
      } else {
        const double ax = op.exx[c] * op.cx, ay = op.eyy[c] * op.cy;
        const double gx = (ev(op.exx, i + 1, j, false) - ev(op.exx, i - 1, j, false)) * op.qx +
                          (ev(op.exy, i, j + 1, true) - ev(op.exy, i, j - 1, true)) * op.qxy;
        const double gy = (ev(op.eyy, i, j + 1, false) - ev(op.eyy, i, j - 1, false)) * op.qy +
                          (ev(op.exy, i + 1, j, true) - ev(op.exy, i - 1, j, true)) * op.qxy;
        const double k6 = op.exy[c] * op.hxy;
        g[0] = k6;
        g[1] = ay - gy;
        g[2] = -k6;
        g[3] = ax - gx;
        g[4] = -2.0 * (ax + ay);
        g[5] = ax + gx;
        g[6] = -k6;
        g[7] = ay + gy;
        g[8] = k6;
      }
      // each ghost coefficient onto its mirror node; the target slot is
      // selected arithmetically so that a[] stays in registers (adding 0.0
      // leaves the other slots unchanged)
#pragma unroll
      for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
        for (int di = -1; di <= 1; ++di) {
          const int ti = mirror_index(i + di, nx) - i, tj = mirror_index(j + dj, ny) - j;
          const int tk = (tj + 1) * 3 + ti + 1;
          const double v = g[(dj + 1) * 3 + di + 1];
#pragma unroll
          for (int k = 0; k < 9; ++k) a[k] += k == tk ? v : 0.0;
        }
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) st[k * n + c] = a[k];
  }
}

// Field recovery (eq. 2): E' = (J^T)^-1 E with E = -grad phi on the uniform
// grid, at every node.  grad phi and the numeric Jacobian use the same
// differences (eq. 39-42, one-sided second order on the edges); an analytic
// Jacobian is taken from jac when given.  Memory-order grid stride.
__global__ void k_field(int nx, int ny, double dx, double dy, const double *__restrict__ phi,
                        const double *__restrict__ xp, const double *__restrict__ yp,
                        const double *__restrict__ jac, double *__restrict__ ex,
                        double *__restrict__ ey) {
  const size_t n = (size_t)nx * ny;
  const double i2dx = 0.5 / dx, i2dy = 0.5 / dy;
  const bool small = n < (size_t(1) << 32);
  // four nodes per trip, so that their loads are in flight together
#pragma unroll 4
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x) {
    int i, j;
    if (small) {
      j = (int)((unsigned)c / (unsigned)nx);
      i = (int)((unsigned)c - (unsigned)j * (unsigned)nx);
    } else {
      j = (int)(c / nx);
      i = (int)(c - (size_t)j * nx);
    }
    double jxx, jxy, jyx, jyy;
    if (jac) {
      jxx = jac[c];
      jxy = jac[n + c];
      jyx = jac[2 * n + c];
      jyy = jac[3 * n + c];
    } else {
      jxx = d_i(xp, nx, i, c, i2dx);
      jxy = d_j(xp, nx, ny, j, c, i2dy);
      jyx = d_i(yp, nx, i, c, i2dx);
      jyy = d_j(yp, nx, ny, j, c, i2dy);
    }
    const double e1 = -d_i(phi, nx, i, c, i2dx), e2 = -d_j(phi, nx, ny, j, c, i2dy);
    const double D = jxx * jyy - jxy * jyx;
    __builtin_nontemporal_store((jyy * e1 - jyx * e2) / D, ex + c);
    __builtin_nontemporal_store((-jxy * e1 + jxx * e2) / D, ey + c);
  }
}

// The identity tensor (eps = I, det J = 1, f = 0; outer ring Dirichlet): the
// operator of eq. 18 becomes the 5-point Laplacian, which the numerical grid
// generation of Section 4.2 (eq. 36-37) solves for x' and y'.  Writes the
// setup partials (min det 1, no non-finite values) like k_setup.
__global__ void k_setup_identity(int nx, int ny, double *__restrict__ exx,
                                 double *__restrict__ exy, double *__restrict__ eyy,
                                 double *__restrict__ det, double *__restrict__ f,
                                 uint8_t *__restrict__ dir, const uint8_t *__restrict__ mask,
                                 float *__restrict__ exx32, float *__restrict__ exy32,
                                 float *__restrict__ eyy32, double *__restrict__ partials) {
  const size_t n = (size_t)nx * ny;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x) {
    const size_t j = c / nx, i = c - j * nx;
    exx[c] = 1.0;
    exy[c] = 0.0;
    eyy[c] = 1.0;
    det[c] = 1.0;
    f[c] = 0.0;
    if (exx32) {
      exx32[c] = 1.0f;
      exy32[c] = 0.0f;
      eyy32[c] = 1.0f;
    }
    dir[c] = (uint8_t)(i == 0 || j == 0 || i == (size_t)nx - 1 || j == (size_t)ny - 1 ||
                       (mask && mask[c]));
  }
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = 1.0;
    partials[2 * blockIdx.x + 1] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Setup from descriptors: the map and the sources evaluated at each node
// ---------------------------------------------------------------------------

// Physical coordinates of computational point (xi, eta) under map m;
// (cph, sph) = (cos, sin) of the perturbation phase.
template <int KIND>
__device__ __forceinline__ void map_point(const tomg_map_desc &m, double cph, double sph,
                                          double xi, double eta, double &x, double &y) {
  if constexpr (KIND == TOMG_MAP_SINUSOIDAL) {
    const double s = sin(M_PI * xi) * sin(M_PI * eta);
    x = xi + m.amp * s;
    y = eta + m.amp * s;
  } else if constexpr (KIND == TOMG_MAP_POLAR) {
    x = xi * cos(eta);
    y = xi * sin(eta);
  } else {
    const double ux = xi - m.cx, uy = eta - m.cy;
    const double r = hypot(ux, uy);
    if (r >= m.r_in && r <= m.r_out) {
      const double ct = ux / r, st = uy / r;
      // cos(k (theta - phase)) for k = 2..5 from cos(theta - phase) by the
      // recurrence cos((k+1) p) = 2 cos p cos(k p) - cos((k-1) p)
      const double c1 = ct * cph + st * sph;
      double ckm1 = c1, ck = 2.0 * c1 * c1 - 1.0;
      double R = m.coef[0] * ck;
#pragma unroll
      for (int k = 3; k <= 5; ++k) {
        const double cn = 2.0 * c1 * ck - ckm1;
        ckm1 = ck;
        ck = cn;
        R += m.coef[k - 2] * ck;
      }
      R = m.r_c + m.pert * R;
      const double rp = r <= m.r_c ? m.r_in + (r - m.r_in) * (R - m.r_in) / (m.r_c - m.r_in)
                                   : R + (r - m.r_c) * (m.r_out - R) / (m.r_out - m.r_c);
      x = m.cx + rp * ct;
      y = m.cy + rp * st;
    } else {  // outside the stretched annulus the map is the identity
      x = xi;
      y = eta;
    }
  }
}

__device__ __forceinline__ double gaussians(const tomg_source_desc &g, double x, double y) {
  const double inv = 1.0 / (2.0 * g.sigma * g.sigma);
  double v = 0.0;
  for (int k = 0; k < g.count; ++k) {
    const double ax = x - g.cx[k], ay = y - g.cy[k];
    v += g.amp[k] * exp(-(ax * ax + ay * ay) * inv);
  }
  return v;
}

// Second-order differences of both map coordinates along one axis at index
// q of n points (central inside, one-sided on the edges, as for node
// coordinates given as arrays); at(k, x, y) gives the point of index k.
template <class F>
__device__ __forceinline__ void diff_axis(F at, int q, int n, double inv2h, double x0,
                                          double y0, double &gx, double &gy) {
  double xa, ya, xb, yb;
  if (q == 0 || q == n - 1) {
    const int s = q == 0 ? 1 : -1;
    at(q + s, xa, ya);
    at(q + 2 * s, xb, yb);
    gx = s * (-3.0 * x0 + 4.0 * xa - xb) * inv2h;
    gy = s * (-3.0 * y0 + 4.0 * ya - yb) * inv2h;
  } else {
    at(q + 1, xa, ya);
    at(q - 1, xb, yb);
    gx = (xa - xb) * inv2h;
    gy = (ya - yb) * inv2h;
  }
}

// k_setup with the map, the sources and the Dirichlet set evaluated from
// descriptors (physical permittivity 1); phi_init (nullable) receives the
// map's Dirichlet data and zeros elsewhere.
template <int KIND>
__global__ void k_setup_desc(int nx, int ny, double xi0, double eta0, double dx, double dy,
                             tomg_map_desc m, tomg_source_desc src, double *__restrict__ exx,
                             double *__restrict__ exy, double *__restrict__ eyy,
                             double *__restrict__ det, double *__restrict__ f,
                             uint8_t *__restrict__ dir, float *__restrict__ exx32,
                             float *__restrict__ exy32, float *__restrict__ eyy32,
                             double *__restrict__ phi_init, double *__restrict__ partials,
                             int neumann) {
  const size_t n = (size_t)nx * ny;
  const double i2dx = 0.5 / dx, i2dy = 0.5 / dy;
  const double cph = cos(m.phase), sph = sin(m.phase);
  double mind = INFINITY, bad = 0.0;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(c / (size_t)nx), i = (int)(c - (size_t)j * nx);
    const double xi = xi0 + i * dx, eta = eta0 + j * dy;
    double x, y, jxx, jxy, jyx, jyy;
    map_point<KIND>(m, cph, sph, xi, eta, x, y);
    if constexpr (KIND == TOMG_MAP_SINUSOIDAL) {
      const double a = m.amp * M_PI * cos(M_PI * xi) * sin(M_PI * eta);
      const double b = m.amp * M_PI * sin(M_PI * xi) * cos(M_PI * eta);
      jxx = 1.0 + a;
      jxy = b;
      jyx = a;
      jyy = 1.0 + b;
    } else if constexpr (KIND == TOMG_MAP_POLAR) {
      jxx = cos(eta);
      jxy = -xi * sin(eta);
      jyx = sin(eta);
      jyy = xi * cos(eta);
    } else {  // numeric Jacobian from the map at the neighbouring nodes
      diff_axis([&](int k, double &px, double &py) {
        map_point<KIND>(m, cph, sph, xi0 + k * dx, eta, px, py);
      }, i, nx, i2dx, x, y, jxx, jyx);
      diff_axis([&](int k, double &px, double &py) {
        map_point<KIND>(m, cph, sph, xi, eta0 + k * dy, px, py);
      }, j, ny, i2dy, x, y, jxy, jyy);
    }
    const double D = jxx * jyy - jxy * jyx;
    const double vxx = (jyy * jyy + jxy * jxy) / D;
    const double vxy = (-jyy * jyx - jxy * jxx) / D;
    const double vyy = (jyx * jyx + jxx * jxx) / D;
    const double fv = -gaussians(src, x, y) * D;
    __builtin_nontemporal_store(vxx, exx + c);
    __builtin_nontemporal_store(vxy, exy + c);
    __builtin_nontemporal_store(vyy, eyy + c);
    __builtin_nontemporal_store(D, det + c);
    __builtin_nontemporal_store(fv, f + c);
    if (exx32) {
      exx32[c] = (float)vxx;
      exy32[c] = (float)vxy;
      eyy32[c] = (float)vyy;
    }
    const bool ring = (i == 0 && !(neumann & TOMG_NEU_W)) ||
                      (i == nx - 1 && !(neumann & TOMG_NEU_E)) ||
                      (j == 0 && !(neumann & TOMG_NEU_S)) ||
                      (j == ny - 1 && !(neumann & TOMG_NEU_N));
    bool held = false;  // interior Dirichlet node of the map (the conductor)
    double g = 0.0;     // Dirichlet value
    if constexpr (KIND == TOMG_MAP_PERTURBED_CIRCLE) {
      held = hypot(xi - m.cx, eta - m.cy) <= m.r_c;
      if (held) g = m.value_in;
    } else if constexpr (KIND == TOMG_MAP_POLAR) {
      if (i == 0 && ring) g = m.value_in;
    }
    dir[c] = (uint8_t)(ring || held);
    if (phi_init) phi_init[c] = (ring || held) ? g : 0.0;
    const bool corner = ring && (i == 0 || i == nx - 1) && (j == 0 || j == ny - 1);
    if (!corner) {
      mind = fmin(mind, D);
      if (!isfinite(vxx) || !isfinite(vxy) || !isfinite(vyy) || !isfinite(fv)) bad += 1.0;
    }
  }
  const double mn = block_reduce<1>(mind);
  const double b = block_reduce<0>(bad);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = mn;
    partials[2 * blockIdx.x + 1] = b;
  }
}

// f = -rho' det J with rho' from a source descriptor at the nodes of map m.
template <int KIND>
__global__ void k_update_rhs_desc(int nx, int ny, double xi0, double eta0, double dx, double dy,
                                  tomg_map_desc m, tomg_source_desc src, const double *det,
                                  double *f, double *partials) {
  const size_t n = (size_t)nx * ny;
  const double cph = cos(m.phase), sph = sin(m.phase);
  double bad = 0.0;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(c / (size_t)nx), i = (int)(c - (size_t)j * nx);
    double x, y;
    map_point<KIND>(m, cph, sph, xi0 + i * dx, eta0 + j * dy, x, y);
    const double rho = gaussians(src, x, y);
    f[c] = -rho * det[c];
    if (!isfinite(rho)) bad += 1.0;
  }
  const double b = block_reduce<0>(bad);
  if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

__global__ void k_update_rhs(const double *rho, const double *det, double *f, size_t n,
                             double *partials) {
  double bad = 0.0;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x) {
    const double v = -rho[c] * det[c];
    f[c] = v;
    if (!isfinite(rho[c])) bad += 1.0;
  }
  const double b = block_reduce<0>(bad);
  if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

__host__ __device__ constexpr double pw(int d) { return d == 0 ? 1.0 : ((d == 1 || d == -1) ? 0.5 : 0.0); }

// Galerkin coarsening of one level (eq. 23; the paper leaves the coarse
// operator open): A_H = (1/4) P^T A_h P with P bilinear, zero rows at fine
// Dirichlet nodes and no columns at coarse Dirichlet nodes, identity rows
// there.  A coarse node is Dirichlet on the ring and where all nine fine
// nodes of its support are Dirichlet (its column of P is empty).
//
// A workgroup owns kGX x kGY coarse nodes.  It stages the fine Dirichlet
// flags of its window, derives the coarse flags of the tile and its one-node
// halo, and computes each fine stencil of the window once into LDS with the
// couplings to Dirichlet fine nodes already zeroed; each thread then sums
// the 81 (fine node, neighbour) products of its coarse node with
// compile-time weights.  The summation order is that of the triple sum
// (fine row b, a; neighbour q, p; coarse column).
constexpr int kGX = 32, kGY = 8;  // 32 x 8 measured fastest of 16x8, 32x4, 32x8, 64x2, 64x4
constexpr int kGFX = 2 * kGX + 1, kGFY = 2 * kGY + 1;  // fine stencil window
constexpr int kGDX = 2 * kGX + 5, kGDY = 2 * kGY + 5;  // fine flag window
constexpr int kGCX = kGX + 2, kGCY = kGY + 2;          // coarse flag window

template <class Op>
__global__ __launch_bounds__(kGX *kGY) void k_coarsen(Op opf, const uint8_t *dirf, int nxf,
                                                      int nyf, int nxc, int nyc, uint8_t *dirc,
                                                      double *stc, float *stc32) {
  __shared__ double S[9][kGFY][kGFX];
  __shared__ uint8_t DF[kGDY][kGDX];
  __shared__ uint8_t DC[kGCY][kGCX];
  constexpr int NT = kGX * kGY;
  const int t = threadIdx.x;
  const int I0 = blockIdx.x * kGX, J0 = blockIdx.y * kGY;
  // fine flags at (2 I0 - 3 + x, 2 J0 - 3 + y); outside the grid counts as Dirichlet
  for (int k = t; k < kGDX * kGDY; k += NT) {
    const int x = k % kGDX, y = k / kGDX;
    const int fi = 2 * I0 - 3 + x, fj = 2 * J0 - 3 + y;
    DF[y][x] = (fi < 0 || fj < 0 || fi >= nxf || fj >= nyf) ? 1 : dirf[(size_t)fj * nxf + fi];
  }
  __syncthreads();
  // coarse flags at (I0 - 1 + x, J0 - 1 + y); support of coarse x at fine 2x + 1 + a
  for (int k = t; k < kGCX * kGCY; k += NT) {
    const int x = k % kGCX, y = k / kGCX;
    const int I = I0 - 1 + x, J = J0 - 1 + y;
    uint8_t d = 1;
    if (I >= 0 && J >= 0 && I < nxc && J < nyc) {
      // on the ring the coarse node keeps the kind of the fine node under it
      // (Dirichlet, or free on a Neumann edge)
      d = (I == 0 || J == 0 || I == nxc - 1 || J == nyc - 1) && DF[2 * y + 1][2 * x + 1];
      if (!d) {
        bool all = true;
#pragma unroll
        for (int b = -1; b <= 1; ++b)
#pragma unroll
          for (int a = -1; a <= 1; ++a) all = all && DF[2 * y + 1 + b][2 * x + 1 + a];
        d = all;
      }
      if (x >= 1 && y >= 1 && x <= kGX && y <= kGY) dirc[(size_t)J * nxc + I] = d;
    }
    DC[y][x] = d;
  }
  // fine stencils at (2 I0 - 1 + x, 2 J0 - 1 + y) = flag window (x + 2, y + 2);
  // a non-Dirichlet fine node is interior or on a Neumann edge, where the
  // stored stencil has no coefficient outside the grid
  for (int k = t; k < kGFX * kGFY; k += NT) {
    const int x = k % kGFX, y = k / kGFX;
    double s[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) s[q] = 0.0;
    if (!DF[y + 2][x + 2]) {
      const int fi = 2 * I0 - 1 + x, fj = 2 * J0 - 1 + y;
      opf.full((size_t)fj * nxf + fi, s);
#pragma unroll
      for (int q = -1; q <= 1; ++q)
#pragma unroll
        for (int pp = -1; pp <= 1; ++pp)
          if (DF[y + 2 + q][x + 2 + pp]) s[(q + 1) * 3 + pp + 1] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) S[q][y][x] = s[q];
  }
  __syncthreads();
  const int tx = t % kGX, ty = t / kGX;
  const int I = I0 + tx, J = J0 + ty;
  if (I >= nxc || J >= nyc) return;
  const size_t nc = (size_t)nxc * nyc, C = (size_t)J * nxc + I;
  double acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  if (DC[ty + 1][tx + 1]) {
    acc[4] = 1.0;
  } else {
#pragma unroll
    for (int b = -1; b <= 1; ++b)
#pragma unroll
      for (int a = -1; a <= 1; ++a) {
        const int wx = 2 * tx + 1 + a, wy = 2 * ty + 1 + b;  // fine node 2C + (a, b)
#pragma unroll
        for (int q = -1; q <= 1; ++q)
#pragma unroll
          for (int pp = -1; pp <= 1; ++pp) {
            const double s = S[(q + 1) * 3 + pp + 1][wy][wx];
            const int u = a + pp, v = b + q;  // neighbour 2C + (u, v)
#pragma unroll
            for (int oj = -1; oj <= 1; ++oj)
#pragma unroll
              for (int oi = -1; oi <= 1; ++oi) {
                const int du = u - 2 * oi, dv = v - 2 * oj;
                if (du >= -1 && du <= 1 && dv >= -1 && dv <= 1)
                  acc[(oj + 1) * 3 + oi + 1] += (pw(a) * pw(b) * pw(du) * pw(dv)) * s;
              }
          }
      }
#pragma unroll
    for (int oj = -1; oj <= 1; ++oj)
#pragma unroll
      for (int oi = -1; oi <= 1; ++oi) {
        double &v = acc[(oj + 1) * 3 + oi + 1];
        v = DC[ty + 1 + oj][tx + 1 + oi] ? 0.0 : v * 0.25;
      }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) stc[k * nc + C] = acc[k];
  if (stc32) {
#pragma unroll
    for (int k = 0; k < 9; ++k) stc32[k * nc + C] = (float)acc[k];
  }
}

// Level-1 coarsening straight from the tensor: the workgroup stages ε_xx,
// ε_xy, ε_yy of its fine window in LDS (one coalesced load per value instead
// of nine per fine stencil), and each thread forms the nine fine stencils of
// its coarse node from LDS with the level-0 formula (the same expressions as
// EpsOp::coefs, so the products and their order are those of k_coarsen).
constexpr int kGEX = 2 * kGX + 3, kGEY = 2 * kGY + 3;  // tensor window, origin 2 I0 - 2

// Three waves per SIMD (at most 168 VGPRs instead of 172): 371 -> 286 us at
// 4097^2; four (128 VGPRs, spilling) took 520 us.
__global__ __launch_bounds__(kGX *kGY, 3) void k_coarsen_eps(EpsOp<double> op, const uint8_t *dirf,
                                                          int nxf, int nyf, int nxc, int nyc,
                                                          uint8_t *dirc, double *stc,
                                                          float *stc32) {
  __shared__ double E[3][kGEY][kGEX];
  __shared__ uint8_t DF[kGDY][kGDX];
  __shared__ uint8_t DC[kGCY][kGCX];
  constexpr int NT = kGX * kGY;
  const int t = threadIdx.x;
  const int I0 = blockIdx.x * kGX, J0 = blockIdx.y * kGY;
  for (int k = t; k < kGDX * kGDY; k += NT) {
    const int x = k % kGDX, y = k / kGDX;
    const int fi = 2 * I0 - 3 + x, fj = 2 * J0 - 3 + y;
    DF[y][x] = (fi < 0 || fj < 0 || fi >= nxf || fj >= nyf) ? 1 : dirf[(size_t)fj * nxf + fi];
  }
  for (int k = t; k < kGEX * kGEY; k += NT) {
    const int x = k % kGEX, y = k / kGEX;
    const int fi = min(max(2 * I0 - 2 + x, 0), nxf - 1), fj = min(max(2 * J0 - 2 + y, 0), nyf - 1);
    const size_t c = (size_t)fj * nxf + fi;
    E[0][y][x] = op.exx[c];
    E[1][y][x] = op.exy[c];
    E[2][y][x] = op.eyy[c];
  }
  __syncthreads();
  for (int k = t; k < kGCX * kGCY; k += NT) {
    const int x = k % kGCX, y = k / kGCX;
    const int I = I0 - 1 + x, J = J0 - 1 + y;
    uint8_t d = 1;
    if (I >= 0 && J >= 0 && I < nxc && J < nyc) {
      // on the ring the coarse node keeps the kind of the fine node under it
      // (Dirichlet, or free on a Neumann edge)
      d = (I == 0 || J == 0 || I == nxc - 1 || J == nyc - 1) && DF[2 * y + 1][2 * x + 1];
      if (!d) {
        bool all = true;
#pragma unroll
        for (int b = -1; b <= 1; ++b)
#pragma unroll
          for (int a = -1; a <= 1; ++a) all = all && DF[2 * y + 1 + b][2 * x + 1 + a];
        d = all;
      }
      if (x >= 1 && y >= 1 && x <= kGX && y <= kGY) dirc[(size_t)J * nxc + I] = d;
    }
    DC[y][x] = d;
  }
  __syncthreads();
  const int tx = t % kGX, ty = t / kGX;
  const int I = I0 + tx, J = J0 + ty;
  if (I >= nxc || J >= nyc) return;
  const size_t nc = (size_t)nxc * nyc, C = (size_t)J * nxc + I;
  double acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  if (DC[ty + 1][tx + 1]) {
    acc[4] = 1.0;
  } else {
#pragma unroll
    for (int b = -1; b <= 1; ++b)
#pragma unroll
      for (int a = -1; a <= 1; ++a) {
        const int dx = 2 * tx + a + 3, dy = 2 * ty + b + 3;  // fine node in the flag window
        const int ex = dx - 1, ey = dy - 1;                 // and in the tensor window
        double s[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) s[q] = 0.0;
        if (!DF[dy][dx]) {
          const double ax = E[0][ey][ex] * op.cx, ay = E[2][ey][ex] * op.cy;
          const double gx = (E[0][ey][ex + 1] - E[0][ey][ex - 1]) * op.qx +
                            (E[1][ey + 1][ex] - E[1][ey - 1][ex]) * op.qxy;
          const double gy = (E[2][ey + 1][ex] - E[2][ey - 1][ex]) * op.qy +
                            (E[1][ey][ex + 1] - E[1][ey][ex - 1]) * op.qxy;
          const double k1 = ax + gx, k3 = ax - gx, k4 = ay + gy, k5 = ay - gy;
          const double k6 = E[1][ey][ex] * op.hxy, k2 = 2.0 * (ax + ay);
          s[0] = k6;  s[1] = k5; s[2] = -k6;
          s[3] = k3;  s[4] = -k2; s[5] = k1;
          s[6] = -k6; s[7] = k4; s[8] = k6;
#pragma unroll
          for (int q = -1; q <= 1; ++q)
#pragma unroll
            for (int pp = -1; pp <= 1; ++pp)
              if (DF[dy + q][dx + pp]) s[(q + 1) * 3 + pp + 1] = 0.0;
        }
#pragma unroll
        for (int q = -1; q <= 1; ++q)
#pragma unroll
          for (int pp = -1; pp <= 1; ++pp) {
            const double v = s[(q + 1) * 3 + pp + 1];
            const int u = a + pp, w = b + q;
#pragma unroll
            for (int oj = -1; oj <= 1; ++oj)
#pragma unroll
              for (int oi = -1; oi <= 1; ++oi) {
                const int du = u - 2 * oi, dv = w - 2 * oj;
                if (du >= -1 && du <= 1 && dv >= -1 && dv <= 1)
                  acc[(oj + 1) * 3 + oi + 1] += (pw(a) * pw(b) * pw(du) * pw(dv)) * v;
              }
          }
      }
#pragma unroll
    for (int oj = -1; oj <= 1; ++oj)
#pragma unroll
      for (int oi = -1; oi <= 1; ++oi) {
        double &v = acc[(oj + 1) * 3 + oi + 1];
        v = DC[ty + 1 + oj][tx + 1 + oi] ? 0.0 : v * 0.25;
      }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) stc[k * nc + C] = acc[k];
  if (stc32) {
#pragma unroll
    for (int k = 0; k < 9; ++k) stc32[k * nc + C] = (float)acc[k];
  }
}

// Transfer weight along one axis of a semi-coarsened level: the linear
// weight pw along an axis that is halved, the identity along one that keeps
// every fine line.
__device__ __forceinline__ double tw(bool halved, int d) {
  return halved ? pw(d) : (d == 0 ? 1.0 : 0.0);
}

// Kind of coarse node (I, J) of a level with strides (sx, sy): Dirichlet
// outside the grid; on the ring the kind of the fine node under it;
// elsewhere Dirichlet when every fine node of its support is (its column of
// P would be empty).
__device__ bool coarse_fixed_semi(const uint8_t *dirf, int nxf, int nyf, int nxc, int nyc,
                                  int sx, int sy, int I, int J) {
  if (I < 0 || J < 0 || I >= nxc || J >= nyc) return true;
  const bool ring = I == 0 || J == 0 || I == nxc - 1 || J == nyc - 1;
  if (ring && dirf[(size_t)(sy * J) * nxf + sx * I]) return true;
  for (int b = -1; b <= 1; ++b)
    for (int a = -1; a <= 1; ++a) {
      if ((sx == 1 && a != 0) || (sy == 1 && b != 0)) continue;
      const int fi = sx * I + a, fj = sy * J + b;
      if (fi < 0 || fj < 0 || fi >= nxf || fj >= nyf) continue;
      if (!dirf[(size_t)fj * nxf + fi]) return false;
    }
  return true;
}

// Coarse Dirichlet flags of a semi-coarsened level, one thread per coarse
// node (the first of the level's two setup launches).
__global__ void k_coarse_flags_semi(const uint8_t *__restrict__ dirf, int nxf, int nyf, int nxc,
                                    int nyc, int sx, int sy, uint8_t *__restrict__ dirc) {
  const size_t nc = (size_t)nxc * nyc;
  for (size_t C = (size_t)blockIdx.x * blockDim.x + threadIdx.x; C < nc;
       C += (size_t)gridDim.x * blockDim.x) {
    const int J = (int)(C / (size_t)nxc), I = (int)(C - (size_t)J * nxc);
    dirc[C] = coarse_fixed_semi(dirf, nxf, nyf, nxc, nyc, sx, sy, I, J) ? 1 : 0;
  }
}

// Galerkin coarsening of a semi-coarsened level (an extension of eq. 23:
// one axis halved, strides sx, sy = 2 halved, 1 kept): A_H = (1/2) P^T A_h P
// with P linear along the halved axis and the identity along the other,
// restricted to the unknowns as in k_coarsen (zero rows at fine Dirichlet
// nodes, no columns at coarse Dirichlet nodes, identity rows there), with
// the coarse flags written by k_coarse_flags_semi.  One thread per coarse
// node: the fine stencils of its support (at most three nodes) come from
// the operator -- eq. 18 from the tensor on level 0, the stored stencil
// below -- and the products are summed in the order of the triple sum (fine
// node, its neighbour, coarse column).  Setup only.
template <class Op, int sx, int sy>
__global__ void k_coarsen_semi(Op opf, const uint8_t *__restrict__ dirf, int nxf, int nyf,
                               int nxc, int nyc, const uint8_t *__restrict__ dirc,
                               double *__restrict__ stc, float *__restrict__ stc32) {
  const size_t nc = (size_t)nxc * nyc;
  constexpr bool hx = sx == 2, hy = sy == 2;
  for (size_t C = (size_t)blockIdx.x * blockDim.x + threadIdx.x; C < nc;
       C += (size_t)gridDim.x * blockDim.x) {
    const int J = (int)(C / (size_t)nxc), I = (int)(C - (size_t)J * nxc);
    bool fixed[9];  // coarse neighbours outside the grid count as Dirichlet
#pragma unroll
    for (int oj = -1; oj <= 1; ++oj)
#pragma unroll
      for (int oi = -1; oi <= 1; ++oi) {
        const int KI = I + oi, KJ = J + oj;
        fixed[(oj + 1) * 3 + oi + 1] = KI < 0 || KJ < 0 || KI >= nxc || KJ >= nyc ||
                                       dirc[(size_t)KJ * nxc + KI] != 0;
      }
    double acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0.0;
    if (fixed[4]) {
      acc[4] = 1.0;
    } else {
#pragma unroll
      for (int b = -1; b <= 1; ++b)
#pragma unroll
        for (int a = -1; a <= 1; ++a) {
          const double wf = tw(hx, a) * tw(hy, b);
          if (wf == 0.0) continue;
          const int fi = sx * I + a, fj = sy * J + b;
          if (fi < 0 || fj < 0 || fi >= nxf || fj >= nyf) continue;
          const size_t f = (size_t)fj * nxf + fi;
          if (dirf[f]) continue;
          double sf[9];
          opf.full(f, sf);
#pragma unroll
          for (int q = -1; q <= 1; ++q)
#pragma unroll
            for (int pp = -1; pp <= 1; ++pp) {
              const int gi = fi + pp, gj = fj + q;
              if (gi < 0 || gj < 0 || gi >= nxf || gj >= nyf) continue;
              if (dirf[(size_t)gj * nxf + gi]) continue;
              const double afg = sf[(q + 1) * 3 + pp + 1];
#pragma unroll
              for (int oj = -1; oj <= 1; ++oj)
#pragma unroll
                for (int oi = -1; oi <= 1; ++oi) {
                  const double wg = tw(hx, gi - sx * (I + oi)) * tw(hy, gj - sy * (J + oj));
                  if (wg != 0.0 && !fixed[(oj + 1) * 3 + oi + 1])
                    acc[(oj + 1) * 3 + oi + 1] += wf * afg * wg;
                }
            }
        }
#pragma unroll
      for (int k = 0; k < 9; ++k) acc[k] *= 0.5;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) stc[k * nc + C] = acc[k];
    if (stc32) {
#pragma unroll
      for (int k = 0; k < 9; ++k) stc32[k * nc + C] = (float)acc[k];
    }
  }
}

// Coarse level rediscretised (TOMG_REDISCRETIZE): eq. 18 on the level's own
// grid, whose spacings are s dx, s dy (s = 2^l; the coefficients cx..hxy
// come with them), with the tensor of level 0 sampled at the coarse nodes --
// node (I, J) takes level 0's tensor at (s I, s J) -- and the Dirichlet set
// sampled the same way, plus the outer ring.  Dirichlet nodes get identity
// rows.  One thread per coarse node, grid-stride.
__global__ void k_rediscretize(const double *__restrict__ exx, const double *__restrict__ exy,
                               const double *__restrict__ eyy, const uint8_t *__restrict__ dir0,
                               int nx0, int s, int nxc, int nyc, double cx, double cy, double qx,
                               double qy, double qxy, double hxy, uint8_t *__restrict__ dirc,
                               double *__restrict__ stc, float *__restrict__ stc32) {
  const size_t nc = (size_t)nxc * nyc, row = (size_t)s * nx0;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc;
       c += (size_t)gridDim.x * blockDim.x) {
    const int J = (int)(c / (size_t)nxc), I = (int)(c - (size_t)J * nxc);
    const size_t f = (size_t)J * row + (size_t)s * I;
    const bool ring = I == 0 || J == 0 || I == nxc - 1 || J == nyc - 1;
    const bool d = ring || dir0[f];
    double a[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (d) {
      a[4] = 1.0;
    } else {
      const double ax = exx[f] * cx, ay = eyy[f] * cy;
      const double gx = (exx[f + s] - exx[f - s]) * qx + (exy[f + row] - exy[f - row]) * qxy;
      const double gy = (eyy[f + row] - eyy[f - row]) * qy + (exy[f + s] - exy[f - s]) * qxy;
      const double k6 = exy[f] * hxy;
      a[0] = k6;      a[1] = ay - gy; a[2] = -k6;
      a[3] = ax - gx; a[4] = -2.0 * (ax + ay); a[5] = ax + gx;
      a[6] = -k6;     a[7] = ay + gy; a[8] = k6;
    }
    dirc[c] = d ? 1 : 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) stc[k * nc + c] = a[k];
    if (stc32) {
#pragma unroll
      for (int k = 0; k < 9; ++k) stc32[k * nc + c] = (float)a[k];
    }
  }
}

constexpr int kInvThreads = 1024, kInvWaves = kInvThreads / 64;

// Coarsest level: index map of the free nodes and the explicit inverse of
// the coarsest matrix by Gauss-Jordan elimination with partial pivoting (one
// block).  cidx[ncoarse] receives the unknown count.
__device__ __forceinline__ void coarse_inverse_body(const double *st, const uint8_t *dir, int nx,
                                                    int ny, double *inv, int *cidx,
                                                    double *scal) {
  // Gauss-Jordan with partial pivoting on m <= kMaxCoarseUnknowns < 64
  // unknowns: lane t & 63 owns a column, wave t >> 6 every kInvWaves-th row
  // (sixteen waves: three or four rows each on 49 unknowns, so the
  // elimination of a pivot step is short next to its barriers); the pivot
  // search is a shuffle reduction in wave 0
  constexpr int M = kMaxCoarseUnknowns;
  __shared__ double A[M][M + 1], B[M][M + 1];
  __shared__ double fac[M], rowa[M], rowb[M];
  __shared__ int cid[81];
  __shared__ int sm;
  const int n = nx * ny, t = threadIdx.x, c = t & 63, w = t >> 6;
  if (t == 0) {
    int m = 0;
    for (int q = 0; q < n; ++q) cid[q] = dir[q] ? -1 : m++;
    sm = m;
    for (int q = 0; q < n; ++q) cidx[q] = cid[q];
    cidx[n] = m;
  }
  __syncthreads();
  const int m = sm;
  if (c < m)
    for (int r = w; r < m; r += kInvWaves) {
      A[r][c] = 0.0;
      B[r][c] = (r == c) ? 1.0 : 0.0;
    }
  __syncthreads();
  for (int q = t; q < n; q += kInvThreads) {
    const int row = cid[q];
    if (row < 0) continue;
    const int I = q % nx, J = q / nx;
    for (int dj = -1; dj <= 1; ++dj)
      for (int di = -1; di <= 1; ++di) {
        const int ii = I + di, jj = J + dj;
        if (ii < 0 || jj < 0 || ii >= nx || jj >= ny) continue;
        const int col = cid[jj * nx + ii];
        if (col >= 0) A[row][col] = st[(size_t)((dj + 1) * 3 + di + 1) * n + q];
      }
  }
  __syncthreads();
  // scale of the pivot test: the largest diagonal magnitude (wave 0, lanes
  // over rows); a pivot below 1e-12 of it marks the matrix singular (a
  // problem without Dirichlet nodes, for example: its operator annihilates
  // constants on every level)
  __shared__ double dscale;
  if (w == 0) {
    double d = c < m ? fabs(A[c][c]) : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) d = fmax(d, __shfl_xor(d, off, 64));
    if (c == 0) {
      dscale = d;
      scal[kSlotPivot] = 0.0;  // this setup's own verdict
    }
  }
  __syncthreads();
  const double tiny = 1e-12 * dscale;
  for (int k = 0; k < m; ++k) {
    if (w == 0) {
      // largest |A[r][k]| for r >= k, the first on ties
      double v = (c >= k && c < m) ? fabs(A[c][k]) : -1.0;
      int p = c;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int op = __shfl_xor(p, off, 64);
        if (ov > v || (ov == v && op < p)) {
          v = ov;
          p = op;
        }
      }
      if (c == 0 && !(v > tiny)) scal[kSlotPivot] = 1.0;
      if (p != k && c < m) {
        double u = A[k][c]; A[k][c] = A[p][c]; A[p][c] = u;
        u = B[k][c]; B[k][c] = B[p][c]; B[p][c] = u;
      }
    }
    __syncthreads();
    if (w == 0 && c < m) {
      const double pv = A[k][k];
      rowa[c] = A[k][c] / pv;
      rowb[c] = B[k][c] / pv;
      fac[c] = A[c][k];
    }
    __syncthreads();
    if (c < m) {
      const double ra = rowa[c], rb = rowb[c];
      for (int r = w; r < m; r += kInvWaves) {
        if (r == k) {
          A[k][c] = ra;
          B[k][c] = rb;
        } else {
          A[r][c] -= fac[r] * ra;
          B[r][c] -= fac[r] * rb;
        }
      }
    }
    __syncthreads();
  }
  // column-major: entry (r, c) of the inverse at c * m + r, so that the
  // coarsest solve's threads (one per row) read a column together
  if (c < m)
    for (int r = w; r < m; r += kInvWaves) inv[c * m + r] = B[r][c];
}

// A coarsest level of up to kMaxCoarseNodes nodes (a grid whose halving
// stops above 9 x 9): the matrix over its free nodes, numbered row-major, is
// banded with half-width bw = nx + 1.  One block factors it as A = L U in
// band storage (band[r * (2 bw + 1) + bw + c - r]) without row exchanges --
// the pivot test below flags a pivot that falls under 1e-12 of the largest
// diagonal magnitude, as the small kernel's does -- and then thread q forms
// row q of A^-1 by solving A^T z = e_q (U^T then L^T), every lane walking
// the same band rows; z goes to inv[c * m + q] (the same column-major layout
// as the small kernel's).
__device__ void coarse_inverse_band_body(const InvArgs &a) {
  __shared__ int cid[kMaxCoarseNodes];
  __shared__ int sm;
  __shared__ double dscale;
  const int nx = a.nx, n = nx * a.ny, t = threadIdx.x;
  const int bw = nx + 1, wd = 2 * bw + 1;
  if (t == 0) {
    int m = 0;
    for (int q = 0; q < n; ++q) cid[q] = a.dir[q] ? -1 : m++;
    sm = m;
    for (int q = 0; q < n; ++q) a.cidx[q] = cid[q];
    a.cidx[n] = m;
  }
  __syncthreads();
  const int m = sm;
  double *band = a.band;
  auto at = [&](int r, int c) -> double & { return band[(size_t)r * wd + bw + c - r]; };
  for (size_t q = t; q < (size_t)m * wd; q += blockDim.x) band[q] = 0.0;
  __syncthreads();
  double dmax = 0.0;
  for (int q = t; q < n; q += blockDim.x) {
    const int row = cid[q];
    if (row < 0) continue;
    const int I = q % nx, J = q / nx;
    for (int dj = -1; dj <= 1; ++dj)
      for (int di = -1; di <= 1; ++di) {
        const int ii = I + di, jj = J + dj;
        if (ii < 0 || jj < 0 || ii >= nx || jj >= a.ny) continue;
        const int col = cid[jj * nx + ii];
        if (col >= 0) at(row, col) = a.st[(size_t)((dj + 1) * 3 + di + 1) * n + q];
      }
    dmax = fmax(dmax, fabs(a.st[(size_t)4 * n + q]));
  }
  {  // largest diagonal magnitude over the block (waves, then wave maxima)
    __shared__ double wmax[kInvWaves];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
    if ((t & 63) == 0) wmax[t >> 6] = dmax;
    __syncthreads();
    if (t == 0) {
      double d = 0.0;
      for (int q = 0; q < (int)(blockDim.x >> 6); ++q) d = fmax(d, wmax[q]);
      dscale = d;
      a.scal[kSlotPivot] = 0.0;  // this setup's own verdict
    }
    __syncthreads();
  }
  const double tiny = 1e-12 * dscale;
  // band LU: at step k the rows k+1 .. k+bw take their multiplier, then the
  // trailing bw x bw block its update
  for (int k = 0; k < m; ++k) {
    const int hi = min(k + bw, m - 1), cnt = hi - k;
    const double pv = at(k, k);
    if (t == 0 && !(fabs(pv) > tiny)) a.scal[kSlotPivot] = 1.0;
    for (int r = k + 1 + t; r <= hi; r += blockDim.x) at(r, k) /= pv;
    __syncthreads();
    for (int q = t; q < cnt * cnt; q += blockDim.x) {
      const int r = k + 1 + q / cnt, c = k + 1 + q % cnt;
      at(r, c) -= at(r, k) * at(k, c);
    }
    __syncthreads();
  }
  // row q of the inverse: U^T w = e_q, then L^T z = w (unit diagonal)
  for (int q = t; q < m; q += blockDim.x) {
    double *z = a.inv;  // z[c] of this row at inv[c * m + q]
    for (int r = 0; r < m; ++r) {
      double v = r == q ? 1.0 : 0.0;
      if (r >= q)
        for (int k = max(q, r - bw); k < r; ++k) v -= at(k, r) * z[(size_t)k * m + q];
      z[(size_t)r * m + q] = r < q ? 0.0 : v / at(r, r);
    }
    for (int r = m - 1; r >= 0; --r) {
      double v = z[(size_t)r * m + q];
      for (int c = r + 1; c <= min(r + bw, m - 1); ++c) v -= at(c, r) * z[(size_t)c * m + q];
      z[(size_t)r * m + q] = v;
    }
  }
}

__global__ __launch_bounds__(kInvThreads) void k_coarse_inverse(InvArgs a) {
  coarse_inverse_body(a.st, a.dir, a.nx, a.ny, a.inv, a.cidx, a.scal);
}

// Batched form: one workgroup per problem.
__global__ __launch_bounds__(kInvThreads) void k_coarse_inverse_b(BatchTab tab) {
  const InvArgs a = *static_cast<const InvArgs *>(tab.e[blockIdx.x].args);
  coarse_inverse_body(a.st, a.dir, a.nx, a.ny, a.inv, a.cidx, a.scal);
}

__global__ __launch_bounds__(kInvThreads) void k_coarse_inverse_band(InvArgs a) {
  coarse_inverse_band_body(a);
}

// ---------------------------------------------------------------------------
// Cycle kernels
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_zero(T *x, size_t n) {
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x)
    x[c] = T(0);
}

// Words of host data carried to the device in a kernel's own arguments: the
// runtime copies the arguments when the launch is queued, so the upload
// needs neither pinned host memory nor a wait for the stream.
constexpr int kWordsPerStore = 240;  // 1920 bytes of argument per launch
struct WordChunk {
  uint64_t w[kWordsPerStore];
};

__global__ __launch_bounds__(256) void k_store_words(uint64_t *__restrict__ dst, WordChunk c,
                                                     int n) {
  if ((int)threadIdx.x < n) dst[threadIdx.x] = c.w[threadIdx.x];
}

// y = fl32(x), n elements.
__global__ void k_narrow(const double *__restrict__ x, float *__restrict__ y, size_t n) {
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x)
    y[c] = (float)x[c];
}

// One colour of four-colour Gauss-Seidel: nodes with i = i0 (mod 2),
// j = j0 (mod 2) that are not Dirichlet (ring nodes only on Neumann edges).
template <class Op, typename T>
__global__ void k_gs_colour(Op op, T *x, const T *b, const uint8_t *dir, int nx, int ny, int i0,
                            int j0) {
  const int i = i0 + 2 * (int)(blockIdx.x * blockDim.x + threadIdx.x);
  const int j = j0 + 2 * (int)(blockIdx.y * blockDim.y + threadIdx.y);
  if (i > nx - 1 || j > ny - 1) return;
  const size_t c = (size_t)j * nx + i;
  if (dir[c]) return;
  T off, dg;
  op.row(c, x, off, dg);
  x[c] = (b[c] - off) / dg;
}

// dst = src transposed: dst[i * ny + j] = src[j * nx + i], through a 32 x 32
// LDS tile so that both the reads and the writes are coalesced.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const T *__restrict__ src, T *__restrict__ dst,
                                                   int nx, int ny) {
  __shared__ T tile[32][33];
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + tx, j = j0 + r;
    if (i < nx && j < ny) tile[r][tx] = src[(size_t)j * nx + i];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int j = j0 + tx, i = i0 + r;
    if (i < nx && j < ny) dst[(size_t)i * ny + j] = tile[tx][r];
  }
}

template <typename T>
void transpose(tomg_problem *p, const T *src, T *dst, int nx, int ny) {
  hipLaunchKernelGGL((k_transpose<T>), dim3((nx + 31) / 32, (ny + 31) / 32), 256, 0, p->stream,
                     src, dst, nx, ny);
}

// Zebra x-line Gauss-Seidel, one parity of rows: block blk solves row
// j = parity + 2 blk exactly for its own nodes, the rows above and below
// held.  The row is a tridiagonal system: a free node keeps its W, C, E
// coefficients and moves b and the six off-row terms to the right; a
// Dirichlet node is the identity row holding its value.  It is cut into
// chunks of consecutive nodes, one per thread (2 to kZebraChunk nodes):
// each thread eliminates its chunk's other nodes in terms of the last node
// of the previous chunk and the last node of its own (Thomas elimination
// with three right-hand sides, in registers); the last nodes then satisfy
// one tridiagonal equation per chunk, solved by parallel cyclic reduction
// in LDS (one equation per thread, log2 of the chunk count steps), and each
// thread substitutes back (the partition method for tridiagonal systems).
// The row's equations are first formed with coalesced loads (consecutive
// threads, consecutive nodes) into LDS, padded by one element per 16 so
// that the chunk-strided reads spread over the banks; the new row goes back
// through LDS and is stored coalesced.  All reads of the row happen before
// the first barrier and all writes after the last, so the row is updated in
// place.
constexpr int kZebraThreads = 256, kZebraChunk = 17;
__host__ __device__ constexpr int zebra_pad(int i) { return i + (i >> 4); }
inline size_t zebra_shmem(int nx, size_t elem) { return 4 * (size_t)(zebra_pad(nx) + 1) * elem; }
static_assert(4 * (zebra_pad(kZebraMaxNx) + 1) * 8 <= 160 * 1024, "zebra row exceeds LDS");

template <class Op, typename T>
__global__ __launch_bounds__(kZebraThreads) void k_zebra_x(Op op, T *x, const T *b,
                                                           const uint8_t *dir, int nx, int ny,
                                                           int parity) {
  __shared__ T Fy[kZebraThreads], Fu[kZebraThreads], Fw[kZebraThreads];
  __shared__ T ra[kZebraThreads], rb[kZebraThreads], rc[kZebraThreads], rd[kZebraThreads];
  __shared__ T Ls[kZebraThreads + 1];  // Ls[t + 1]: last node of chunk t; Ls[0] = 0
  extern __shared__ unsigned char zebra_raw[];
  const int j = parity + 2 * (int)blockIdx.x;
  if (j > ny - 1) return;
  const int np = zebra_pad(nx) + 1;
  T *A = reinterpret_cast<T *>(zebra_raw), *C = A + np, *E = C + np, *D = E + np;
  const int t = threadIdx.x;
  const int nch = min(kZebraThreads, nx / 2);
  const int q = nx / nch, rem = nx % nch;
  const bool act = t < nch;
  const int m = act ? q + (t < rem ? 1 : 0) : 0;
  const int s = t * q + min(t, rem);
  const size_t row = (size_t)j * nx;
  const size_t dn = j > 0 ? (size_t)nx : 0, up = j < ny - 1 ? (size_t)nx : 0;

  // line equation of node i of the row: a x[i-1] + c x[i] + e x[i+1] = d
  auto coef = [&](int i, T &a, T &c, T &e, T &d) {
    const size_t ci = row + i;
    if (dir[ci]) {
      a = T(0);
      c = T(1);
      e = T(0);
      d = x[ci];
      return;
    }
    T s9[9];
    op.full(ci, s9);
    const size_t w = i > 0 ? ci - 1 : ci, ea = i < nx - 1 ? ci + 1 : ci;
    a = i > 0 ? s9[3] : T(0);
    c = s9[4];
    e = i < nx - 1 ? s9[5] : T(0);
    d = b[ci] - (s9[0] * x[w - dn] + s9[1] * x[ci - dn] + s9[2] * x[ea - dn]) -
        (s9[6] * x[w + up] + s9[7] * x[ci + up] + s9[8] * x[ea + up]);
  };

  for (int i = t; i < nx; i += kZebraThreads) {
    T a, c, e, d;
    coef(i, a, c, e, d);
    const int pi = zebra_pad(i);
    A[pi] = a;
    C[pi] = c;
    E[pi] = e;
    D[pi] = d;
  }
  __syncthreads();
  auto lds_coef = [&](int i, T &a, T &c, T &e, T &d) {
    const int pi = zebra_pad(i);
    a = A[pi];
    c = C[pi];
    e = E[pi];
    d = D[pi];
  };

  // chunk nodes k = 0 .. m-2 in terms of the outside unknowns:
  // x_k = Y_k + U_k Ls[t] + W_k Ls[t + 1]
  T cp[kZebraChunk], Y[kZebraChunk], U[kZebraChunk], W[kZebraChunk];
#pragma unroll
  for (int k = 0; k < kZebraChunk; ++k) cp[k] = Y[k] = U[k] = W[k] = T(0);
  T ym = T(0), um = T(0), wm = T(0);
  T aL = T(0), cL = T(1), eL = T(0), dL = T(0);
  if (act) {
#pragma unroll
    for (int k = 0; k < kZebraChunk - 1; ++k) {
      if (k < m - 1) {
        T a, c, e, d;
        lds_coef(s + k, a, c, e, d);
        const T ai = k == 0 ? T(0) : a;  // the first node's W neighbour is outside
        const T den = c - (k == 0 ? T(0) : ai * cp[k - 1]);
        const bool last = k == m - 2;    // its E neighbour is outside
        cp[k] = (last ? T(0) : e) / den;
        Y[k] = (d - (k == 0 ? T(0) : ai * Y[k - 1])) / den;
        U[k] = ((k == 0 ? -a : T(0)) - (k == 0 ? T(0) : ai * U[k - 1])) / den;
        W[k] = ((last ? -e : T(0)) - (k == 0 ? T(0) : ai * W[k - 1])) / den;
        if (last) {
          ym = Y[k];
          um = U[k];
          wm = W[k];
        }
      }
    }
#pragma unroll
    for (int k = kZebraChunk - 3; k >= 0; --k) {
      if (k <= m - 3) {
        Y[k] -= cp[k] * Y[k + 1];
        U[k] -= cp[k] * U[k + 1];
        W[k] -= cp[k] * W[k + 1];
      }
    }
    lds_coef(s + m - 1, aL, cL, eL, dL);
    Fy[t] = Y[0];
    Fu[t] = U[0];
    Fw[t] = W[0];
  }
  __syncthreads();
  if (act) {
    // equation of the chunk's last node with x[m-2] and the next chunk's
    // first node substituted: ra Ls[t] + rb Ls[t+1] + rc Ls[t+2] = rd
    const bool nxt = t + 1 < nch;
    ra[t] = aL * um;
    rb[t] = aL * wm + cL + (nxt ? eL * Fu[t + 1] : T(0));
    rc[t] = nxt ? eL * Fw[t + 1] : T(0);
    rd[t] = dL - aL * ym - (nxt ? eL * Fy[t + 1] : T(0));
  }
  __syncthreads();
  // parallel cyclic reduction: each step eliminates the couplings to the
  // equations sft away (outside the system: identity rows, zero right side)
  T pa = act ? ra[t] : T(0), pb = act ? rb[t] : T(1), pc = act ? rc[t] : T(0);
  T pd = act ? rd[t] : T(0);
  for (int sft = 1; sft < nch; sft <<= 1) {
    T am = T(0), bm = T(1), cm = T(0), dm = T(0), ap = T(0), bp = T(1), cq = T(0), dp = T(0);
    if (act && t - sft >= 0) {
      am = ra[t - sft];
      bm = rb[t - sft];
      cm = rc[t - sft];
      dm = rd[t - sft];
    }
    if (act && t + sft < nch) {
      ap = ra[t + sft];
      bp = rb[t + sft];
      cq = rc[t + sft];
      dp = rd[t + sft];
    }
    const T k1 = pa / bm, k2 = pc / bp;
    pb = pb - cm * k1 - ap * k2;
    pd = pd - dm * k1 - dp * k2;
    pa = -am * k1;
    pc = -cq * k2;
    __syncthreads();
    if (act) {
      ra[t] = pa;
      rb[t] = pb;
      rc[t] = pc;
      rd[t] = pd;
    }
    __syncthreads();
  }
  if (act) Ls[t + 1] = pd / pb;
  if (t == 0) Ls[0] = T(0);
  __syncthreads();
  if (act) {  // the new row into LDS (A is free since the forward sweep)
    const T lp = Ls[t], lt = Ls[t + 1];
#pragma unroll
    for (int k = 0; k < kZebraChunk - 1; ++k)
      if (k < m - 1) A[zebra_pad(s + k)] = Y[k] + U[k] * lp + W[k] * lt;
    A[zebra_pad(s + m - 1)] = lt;
  }
  __syncthreads();
  for (int i = t; i < nx; i += kZebraThreads) x[row + i] = A[zebra_pad(i)];
}

// r = b - A x at free nodes, 0 elsewhere (all nodes written).
template <class Op, typename T>
__global__ void k_residual(Op op, const T *x, const T *b, const uint8_t *dir, int nx, int ny,
                           T *r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= nx || j >= ny) return;
  const size_t c = (size_t)j * nx + i;
  T v = T(0);
  if (!dir[c]) {
    T off, dg;
    op.row(c, x, off, dg);
    v = b[c] - off - dg * x[c];
  }
  r[c] = v;
}

// Damped Jacobi update x += omega r / A_CC at free nodes.
template <class Op, typename T>
__global__ void k_jacobi_update(Op op, T *x, const T *r, const uint8_t *dir, int nx, int ny,
                                T omega) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= nx || j >= ny) return;
  const size_t c = (size_t)j * nx + i;
  if (dir[c]) return;
  x[c] += omega * r[c] / op.diag(c);
}

// Residual (eq. 20) and full-weighting restriction into the coarse
// right-hand side (eq. 23): weights 4, 2, 1 over 16.
// dirc (Neumann edges, else null): the coarse flags; a free coarse ring node
// sums the fine nodes of its support that lie inside the grid.
template <class Op, typename T>
__global__ void k_restrict(Op op, const T *x, const T *b, const uint8_t *dir, int nxf, T *bc,
                           int nxc, int nyc, const uint8_t *dirc) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y * blockDim.y + threadIdx.y;
  if (I >= nxc || J >= nyc) return;
  const int nyf = 2 * (nyc - 1) + 1;
  T s = T(0);
  const bool ring = I == 0 || J == 0 || I == nxc - 1 || J == nyc - 1;
  if (!ring || (dirc && !dirc[(size_t)J * nxc + I])) {
    for (int dj = -1; dj <= 1; ++dj)
      for (int di = -1; di <= 1; ++di) {
        const int fi = 2 * I + di, fj = 2 * J + dj;
        if (fi < 0 || fj < 0 || fi >= nxf || fj >= nyf) continue;
        const size_t f = (size_t)fj * nxf + fi;
        if (dir[f]) continue;
        T off, dg;
        op.row(f, x, off, dg);
        const T w = T((2 - abs(di)) * (2 - abs(dj))) * T(0.0625);
        s += w * (b[f] - off - dg * x[f]);
      }
  }
  bc[(size_t)J * nxc + I] = s;
}

// Full weighting (eq. 23) of a residual field already formed (zero at
// Dirichlet nodes) into the coarse right-hand side; a free coarse ring node
// (Neumann edge) sums the fine nodes of its support inside the grid, other
// ring nodes get zero.
template <typename T>
__global__ void k_full_weighting(const T *r, int nxf, int nyf, T *bc, int nxc, int nyc,
                                 const uint8_t *dirc) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y * blockDim.y + threadIdx.y;
  if (I >= nxc || J >= nyc) return;
  T s = T(0);
  const bool ring = I == 0 || J == 0 || I == nxc - 1 || J == nyc - 1;
  if (!ring || !dirc[(size_t)J * nxc + I]) {
    for (int dj = -1; dj <= 1; ++dj)
      for (int di = -1; di <= 1; ++di) {
        const int fi = 2 * I + di, fj = 2 * J + dj;
        if (fi < 0 || fj < 0 || fi >= nxf || fj >= nyf) continue;
        const T w = T((2 - abs(di)) * (2 - abs(dj))) * T(0.0625);
        s += w * r[(size_t)fj * nxf + fi];
      }
  }
  bc[(size_t)J * nxc + I] = s;
}

// Bilinear prolongation and correction (eq. 24) at free fine nodes.
template <typename T>
__global__ void k_prolong(const T *ec, int nxc, T *x, const uint8_t *dir, int nxf, int nyf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= nxf || j >= nyf) return;
  const size_t c = (size_t)j * nxf + i;
  if (dir[c]) return;
  const int I = i >> 1, J = j >> 1;
  const T *r0 = ec + (size_t)J * nxc;
  T e0 = (i & 1) ? T(0.5) * (r0[I] + r0[I + 1]) : r0[I];
  if (j & 1) {
    const T *r1 = r0 + nxc;
    const T e1 = (i & 1) ? T(0.5) * (r1[I] + r1[I + 1]) : r1[I];
    e0 = T(0.5) * (e0 + e1);
  }
  x[c] += e0;
}

// ---------------------------------------------------------------------------
// Level-0 reductions and the refinement kernels.  The block count of a
// reduction depends only on the grid size (red_blocks), so a problem reduces
// in the same order alone and in a batch.
// ---------------------------------------------------------------------------

// Level-0 reductions run over tiles of one wave by kRedTileH rows.  Lane k
// of a tile holds column i0 - 1 + k (clamped to the grid): lanes 1 .. 62
// compute, lanes 0 and 63 only carry the neighbouring columns, whose values
// reach the computing lanes by cross-lane shuffles, so each row costs one
// load per array.  A lane walks its column down the tile with the rows
// below, at and above the current one in registers and the next rows'
// loads in flight (the loop is unrolled whole, so every row stays in place
// in its registers).  Each lane sums its r^2 in row order and the tile's
// partial is the wave's sum over the lanes in lane order: the tiles depend
// only on the grid, so a problem reduces in the same order alone and in a
// batch.
//
// Modes: kRmNorm sum of r^2 of x; kRmNormZF the same with the values at free
// nodes taken as zero (the zero-interior start of the stopping test);
// kRmBegin both; kRmIrRes r32 = fl32(r) (zero at Dirichlet nodes) and its
// sum; kRmIrResB0 also the zero-interior sum; kRmIrStep the refinement
// update and residual together: v = x + e32 at free nodes (x at Dirichlet
// nodes) is written to xo and r = f - A v gives r32 and its sum.
enum { kRmNorm = 0, kRmNormZF, kRmBegin, kRmIrRes, kRmIrResB0, kRmIrStep };
constexpr int kRedCols = kRedTileW - 2;  // computed columns of a tile

template <int M> constexpr bool rm_zf() { return M == kRmNormZF || M == kRmBegin || M == kRmIrResB0; }
template <int M> constexpr bool rm_x() { return M != kRmNormZF; }

// One row as loaded at the lane's column.
template <bool ST>
struct RedRaw {
  double x, exx, exy, eyy, f;
  double st[ST ? 9 : 1];
  float e;
  uint8_t d;
};

// One row of the window: the values at columns i-1, i, i+1, the Dirichlet
// flags of the three (bits 0, 1, 2) and the row's own coefficients.
template <bool ST>
struct RedWin {
  double vl, vc, vr, exx, exy, eyy, f;
  double st[ST ? 9 : 1];
  uint32_t d;
};

template <int M, bool ST>
__device__ __forceinline__ void red_load(RedRaw<ST> &w, const RedArgs &a,
                                         const double *__restrict__ x, int i, int r) {
  const size_t c = (size_t)r * a.nx + i;
  w.x = x[c];
  w.d = a.dir[c];
  if constexpr (M == kRmIrStep) w.e = a.e32[c];
  w.f = a.f[c];
  if constexpr (ST) {
    const size_t n = (size_t)a.nx * a.ny;
#pragma unroll
    for (int k = 0; k < 9; ++k) w.st[k] = a.st0[k * n + c];
  } else {
    w.exx = a.exx[c];
    w.exy = a.exy[c];
    w.eyy = a.eyy[c];
  }
}

template <int M, bool ST>
__device__ __forceinline__ void red_enter(RedWin<ST> &w, const RedRaw<ST> &q) {
  double v = q.x;
  if constexpr (M == kRmIrStep) v = q.d ? q.x : q.x + (double)q.e;
  w.vc = v;
  w.vl = __shfl_up(v, 1, 64);
  w.vr = __shfl_down(v, 1, 64);
  const uint32_t dc = q.d ? 2u : 0u;
  w.d = dc | (__shfl_up(dc, 1, 64) >> 1) | (__shfl_down(dc, 1, 64) << 1);
  w.f = q.f;
  if constexpr (ST) {
#pragma unroll
    for (int k = 0; k < 9; ++k) w.st[k] = q.st[k];
  } else {
    w.exx = q.exx;
    w.exy = q.exy;
    w.eyy = q.eyy;
  }
}

// r = f - A v at the middle row from the rows below (S), at (C) and above
// (N): the operator of eq. 18 or the stored stencil; with Z the values at
// free nodes are taken as zero.
template <bool ST, bool Z>
__device__ __forceinline__ double red_resid(const RedArgs &a, const RedWin<ST> &S,
                                            const RedWin<ST> &C, const RedWin<ST> &N,
                                            double exxl, double exxr, double exyl, double exyr) {
  auto z = [](const RedWin<ST> &w, int k) {
    const double v = k == 0 ? w.vl : (k == 1 ? w.vc : w.vr);
    return (!Z || ((w.d >> k) & 1u)) ? v : 0.0;
  };
  if constexpr (ST) {
    const double *st = C.st;
    const double off = st[0] * z(S, 0) + st[1] * z(S, 1) + st[2] * z(S, 2) + st[3] * z(C, 0) +
                       st[5] * z(C, 2) + st[6] * z(N, 0) + st[7] * z(N, 1) + st[8] * z(N, 2);
    return C.f - off - st[4] * z(C, 1);
  } else {
    const double ax = C.exx * a.cx, ay = C.eyy * a.cy;
    const double gx = (exxr - exxl) * a.qx + (N.exy - S.exy) * a.qxy;
    const double gy = (N.eyy - S.eyy) * a.qy + (exyr - exyl) * a.qxy;
    const double k1 = ax + gx, k3 = ax - gx, k4 = ay + gy, k5 = ay - gy;
    const double k6 = C.exy * a.hxy, k2 = 2.0 * (ax + ay);
    const double off = k1 * z(C, 2) + k3 * z(C, 0) + k4 * z(N, 1) + k5 * z(S, 1) +
                       k6 * ((z(N, 2) - z(N, 0)) - (z(S, 2) - z(S, 0)));
    return C.f - off + k2 * z(C, 1);
  }
}

template <int M, bool ST>
__device__ __forceinline__ void red_tile(const RedArgs &a, const double *__restrict__ x,
                                         double *__restrict__ xo, int t) {
  constexpr int D = ST ? 1 : 3;  // rows loaded ahead of the window
  const int tx = (a.nx + kRedCols - 1) / kRedCols;
  const int lane = (int)threadIdx.x;
  const int i = (t % tx) * kRedCols - 1 + lane;  // this lane's column
  const int ic = i < 0 ? 0 : (i >= a.nx ? a.nx - 1 : i);
  const bool computes = lane >= 1 && lane <= kRedCols && i < a.nx;
  const int j0 = (t / tx) * kRedTileH, j1 = min(j0 + kRedTileH, a.ny);
  auto row = [&](int r) { return r < 0 ? 0 : (r >= a.ny ? a.ny - 1 : r); };
  float *__restrict__ r32 = a.r32;
  double s = 0.0, s0 = 0.0;
  RedWin<ST> w[3];
  RedRaw<ST> q[D];
  {
    RedRaw<ST> t0;
    red_load<M, ST>(t0, a, x, ic, row(j0 - 1));
    red_enter<M, ST>(w[0], t0);
    red_load<M, ST>(t0, a, x, ic, row(j0));
    red_enter<M, ST>(w[1], t0);
    red_load<M, ST>(t0, a, x, ic, row(j0 + 1));
    red_enter<M, ST>(w[2], t0);
  }
  // The walk has a fixed length (rows past the grid are clamped to its last
  // row), so the rows move through the window and the load slots without
  // control flow around them and stay in the registers they were loaded
  // into; only the arithmetic of rows outside the tile is skipped.
#pragma unroll
  for (int k = 0; k < D; ++k) red_load<M, ST>(q[k], a, x, ic, row(j0 + 2 + k));
#pragma unroll
  for (int u = 0; u < kRedTileH; ++u) {
    const int j = j0 + u;
    const RedWin<ST> &S = w[u % 3], &C = w[(u + 1) % 3], &N = w[(u + 2) % 3];
    double exxl = 0.0, exxr = 0.0, exyl = 0.0, exyr = 0.0;
    if constexpr (!ST) {
      exxl = __shfl_up(C.exx, 1, 64);
      exxr = __shfl_down(C.exx, 1, 64);
      exyl = __shfl_up(C.exy, 1, 64);
      exyr = __shfl_down(C.exy, 1, 64);
    }
    if (computes && j < j1) {
      const size_t c = (size_t)j * a.nx + i;
      double r = 0.0;
      if (!(C.d & 2u)) {
        // a free node on the ring exists only with a stored stencil
        // (Neumann edges), whose clamped neighbours carry zero coefficients
        if constexpr (rm_x<M>()) r = red_resid<ST, false>(a, S, C, N, exxl, exxr, exyl, exyr);
        if constexpr (rm_zf<M>()) {
          const double r0 = red_resid<ST, true>(a, S, C, N, exxl, exxr, exyl, exyr);
          if constexpr (M == kRmNormZF) r = r0;
          else s0 += r0 * r0;
        }
      }
      if constexpr (M == kRmIrRes || M == kRmIrResB0 || M == kRmIrStep) r32[c] = (float)r;
      if constexpr (M == kRmIrStep) xo[c] = C.vc;
      s += r * r;
    }
    // row j + 2 enters the window in place of the row below, and row
    // j + 2 + D is loaded into the freed slot (both only while the tile
    // still needs them: the conditions are fixed at compile time)
    if (u + 2 <= kRedTileH) red_enter<M, ST>(w[u % 3], q[u % D]);
    if (u + 2 + D <= kRedTileH) red_load<M, ST>(q[u % D], a, x, ic, row(j + 2 + D));
  }
  s = block_reduce<0>(s);
  if (threadIdx.x == 0) a.partials[t] = s;
  if constexpr (M == kRmBegin || M == kRmIrResB0) {
    s0 = block_reduce<0>(s0);
    if (threadIdx.x == 0) a.partials[a.nblk + t] = s0;
  }
}

// Refinement update alone: phi += e32 at free nodes (the tiles of the
// reductions, no partials).
__device__ __forceinline__ void ir_update_body(const RedArgs &a, double *phi, int t) {
  const int tx = (a.nx + kRedCols - 1) / kRedCols;
  const int lane = (int)threadIdx.x;
  const int i = (t % tx) * kRedCols - 1 + lane;
  const int j0 = (t / tx) * kRedTileH, j1 = min(j0 + kRedTileH, a.ny);
  if (lane < 1 || lane > kRedCols || i >= a.nx) return;
  // eight rows at a time: every load of the group is issued before the
  // first store
  constexpr int G = 8;
  for (int jg = j0; jg < j1; jg += G) {
    double v[G];
    float e[G];
    uint8_t d[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const size_t c = (size_t)min(jg + k, j1 - 1) * a.nx + i;
      v[k] = phi[c];
      e[k] = a.e32[c];
      d[k] = a.dir[c];
    }
#pragma unroll
    for (int k = 0; k < G; ++k)
      if (jg + k < j1 && !d[k]) phi[(size_t)(jg + k) * a.nx + i] = v[k] + (double)e[k];
  }
}

// phi = a.phi2 over the tile (the whole grid).
__device__ __forceinline__ void copy_back_body(const RedArgs &a, double *phi, int t) {
  const int tx = (a.nx + kRedCols - 1) / kRedCols;
  const int lane = (int)threadIdx.x;
  const int i = (t % tx) * kRedCols - 1 + lane;
  const int j0 = (t / tx) * kRedTileH, j1 = min(j0 + kRedTileH, a.ny);
  if (lane < 1 || lane > kRedCols || i >= a.nx) return;
#pragma unroll 8
  for (int j = j0; j < j1; ++j) {
    const size_t c = (size_t)j * a.nx + i;
    phi[c] = a.phi2[c];
  }
}

// The tile of block b among the n blocks [start, start + n) of a problem:
// the device hands blocks to its eight XCDs round-robin (block b to XCD
// b mod 8), so numbering each XCD's blocks consecutively gives each XCD a
// contiguous run of tiles, whose shared halo lines then come from that
// XCD's L2 once.  A bijection onto [0, n): each tile's partial sum, and so
// the reduction, is the same whatever block computes it.
__device__ __forceinline__ int xcd_tile_of(int b, int start, int n) {
  auto first = [&](int y) { return start + (((y - start) % 8) + 8) % 8; };
  auto count = [&](int y) {
    const int f = first(y);
    return f < start + n ? (start + n - 1 - f) / 8 + 1 : 0;
  };
  const int x = b & 7;
  int off = 0;
  for (int y = 0; y < x; ++y) off += count(y);
  return off + (b - first(x)) / 8;
}

// ST: the problem has a stored level-0 stencil (a.st0).
template <int M, bool ST>
__global__ void __launch_bounds__(kRedTileW) k_red(RedArgs a, const double *x, double *xo,
                                                   const double *skip) {
  if (skip && *skip != 0.0) return;
  red_tile<M, ST>(a, x, xo, xcd_tile_of(blockIdx.x, 0, gridDim.x));
}
__global__ void __launch_bounds__(kRedTileW) k_ir_update(RedArgs a, double *phi,
                                                         const double *skip) {
  if (skip && *skip != 0.0) return;
  ir_update_body(a, phi, xcd_tile_of(blockIdx.x, 0, gridDim.x));
}

__device__ __forceinline__ const BatchEntry &locate(const BatchTab &tab, int b) {
  int lo = 0, hi = tab.count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab.e[mid].start <= b) lo = mid; else hi = mid - 1;
  }
  return tab.e[lo];
}

// KIND: a reduction mode (kRm*), -1 for the refinement update alone, or -2
// for the copy of the iterate from the problem's second array back into the
// caller's.  With kRmIrStep the iterate moves between the caller's array and
// the second one (a.phi2): role 0 reads the caller's and writes the second,
// role 1 the other way round.
// ST: every problem of the launch has a stored level-0 stencil.
template <int KIND, bool ST>
__global__ void __launch_bounds__(kRedTileW) k_red_b(BatchTab tab) {
  const BatchEntry &e = locate(tab, blockIdx.x);
  const RedArgs &a = *static_cast<const RedArgs *>(e.args);
  const int t = xcd_tile_of(blockIdx.x, e.start, e.nbx);
  double *phi = static_cast<double *>(e.phi);
  if constexpr (KIND == -2) {
    copy_back_body(a, phi, t);
  } else if constexpr (KIND == -1) {
    ir_update_body(a, phi, t);
  } else if constexpr (KIND == kRmIrStep) {
    if (e.role) red_tile<KIND, ST>(a, a.phi2, phi, t);
    else red_tile<KIND, ST>(a, phi, a.phi2, t);
  } else {
    red_tile<KIND, ST>(a, phi, nullptr, t);
  }
}

// Batched finalize: one block per problem; sqrt of the fixed-order sum into
// scal[slot]; with rel != kRelNone, the relative residual and the
// convergence flag too, and a copy into out[e.out]; kRelBegin also records
// the starting iterate's residual (as k_finalize).
__global__ void k_finalize_b(BatchTab tab, int rel, double *out) {
  const BatchEntry &e = tab.e[blockIdx.x];
  const FinArgs a = *static_cast<const FinArgs *>(e.args);
  double v = 0.0;
  for (int k = threadIdx.x; k < a.n; k += blockDim.x) v += a.partials[k];
  v = block_reduce<0>(v);
  if (threadIdx.x == 0) {
    v = sqrt(v);
    a.scal[e.slot] = v;
    if (rel != kRelNone) {
      if (rel == kRelBegin) a.scal[kSlotR0] = v;
      double r = rel_residual(v, a.scal[kSlotB0], a.scal[kSlotR0]);
      // a setup that failed its checks (folded map, non-finite input,
      // singular coarsest matrix) or a non-finite new right-hand side
      // reports a non-finite residual
      if (!(a.scal[kSlotMinDet] > 0.0) || a.scal[kSlotBad] != 0.0 ||
          a.scal[kSlotPivot] != 0.0 || a.scal[kSlotBadRhs] != 0.0)
        r = NAN;
      a.scal[kSlotRel] = r;
      a.scal[kSlotDone] = (r <= a.scal[kSlotTol]) ? 1.0 : 0.0;
      if (rel == kRelBegin) a.scal[kSlotCycles] = 0.0;
      if (rel == kRelCycle) a.scal[kSlotCycles] += 1.0;
      record_history(a.scal, rel, r);
      out[e.out] = r;
    }
  }
}

// Coarsest solve x = A^-1 b with the explicit inverse (one block).
template <typename T>
__global__ void k_coarse_solve(const double *inv, const int *cidx, const T *b, T *x, int n) {
  __shared__ double bb[kMaxCoarseNodes];
  const int m = cidx[n];
  for (int c = threadIdx.x; c < n; c += blockDim.x)
    if (cidx[c] >= 0) bb[cidx[c]] = (double)b[c];
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const int k = cidx[c];
    double v = 0.0;
    if (k >= 0)
      for (int q = 0; q < m; ++q) v += inv[(size_t)q * m + k] * bb[q];
    x[c] = (T)v;
  }
}

// STREAM-style copy, 16 bytes per lane per iteration.
// Streaming copy used as the bandwidth reference beside the solver: four
// 16-byte loads in flight per thread, non-temporal loads and stores.
__global__ void k_copy16(const double2 *__restrict__ src, double2 *__restrict__ dst, size_t n) {
  constexpr int U = 4;
  const size_t stride = (size_t)gridDim.x * blockDim.x * U;
  for (size_t b = (size_t)blockIdx.x * blockDim.x * U + threadIdx.x; b < n; b += stride) {
    double2 v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const size_t c = b + (size_t)k * blockDim.x;
      if (c < n) {
        v[k].x = __builtin_nontemporal_load(&src[c].x);
        v[k].y = __builtin_nontemporal_load(&src[c].y);
      }
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const size_t c = b + (size_t)k * blockDim.x;
      if (c < n) {
        __builtin_nontemporal_store(v[k].x, &dst[c].x);
        __builtin_nontemporal_store(v[k].y, &dst[c].y);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Host-side helpers
// ---------------------------------------------------------------------------

inline dim3 grid2(int nx, int ny, dim3 blk) {
  return dim3((nx + blk.x - 1) / blk.x, (ny + blk.y - 1) / blk.y);
}
inline unsigned grid1(size_t n, unsigned cap = 4096) {
  size_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  return (unsigned)(g > cap ? cap : g);
}

template <typename T>
struct LevelView {
  T *x;
  T *b;
  const T *st;
  T *pong;  // second iterate buffer of the fused passes
};

template <class Op, typename T>
void smooth_level(tomg_problem *p, const Op &op, T *x, const T *b, const uint8_t *dir, int nx,
                  int ny, int sweeps) {
  const dim3 blk(64, 4);
  if (p->cfg.smoother == TOMG_ZEBRA_X) {
    for (int s = 0; s < sweeps; ++s)
      for (int parity = 0; parity < 2; ++parity)
        hipLaunchKernelGGL((k_zebra_x<Op, T>), (ny - parity + 1) / 2, kZebraThreads,
                           zebra_shmem(nx, sizeof(T)), p->stream, op, x, b, dir, nx, ny, parity);
    return;
  }
  if (p->cfg.smoother == TOMG_JACOBI) {
    T *r = reinterpret_cast<T *>(p->tmp);
    for (int s = 0; s < sweeps; ++s) {
      hipLaunchKernelGGL((k_residual<Op, T>), grid2(nx, ny, blk), blk, 0, p->stream, op, x, b,
                         dir, nx, ny, r);
      hipLaunchKernelGGL((k_jacobi_update<Op, T>), grid2(nx, ny, blk), blk, 0, p->stream, op, x,
                         r, dir, nx, ny, (T)p->cfg.jacobi_omega);
    }
    return;
  }
  const int cxn = (nx - 1) / 2 + 1, cyn = (ny - 1) / 2 + 1;
  for (int s = 0; s < sweeps; ++s)
    for (int col = 0; col < 4; ++col) {
      const int pi = col & 1, pj = col >> 1;
      const int i0 = pi, j0 = pj;
      hipLaunchKernelGGL((k_gs_colour<Op, T>), grid2(cxn, cyn, blk), blk, 0, p->stream, op, x, b,
                         dir, nx, ny, i0, j0);
    }
}

// Alternating zebra sweeps on stored stencils (FP64): an x-line sweep, then
// the y-line sweep as an x-line sweep of the transposed level (stencil and
// flags transposed at setup; iterate and right-hand side transposed in and
// the iterate back out).
void smooth_level_xy(tomg_problem *p, int l, const double *st, double *x, const double *b,
                     int sweeps) {
  const tomg::Level &v = p->lv[l];
  const StOpB<double> op = st_op_b<double>(st, v.nx, v.ny);
  const StOpB<double> opT = st_op_b<double>(v.stT, v.ny, v.nx);
  transpose<double>(p, b, v.bT, v.nx, v.ny);  // the right-hand side is fixed while smoothing
  for (int s = 0; s < sweeps; ++s) {
    for (int parity = 0; parity < 2; ++parity)
      hipLaunchKernelGGL((k_zebra_x<StOpB<double>, double>), (v.ny - parity + 1) / 2,
                         kZebraThreads, zebra_shmem(v.nx, sizeof(double)), p->stream, op, x, b,
                         (const uint8_t *)v.dir, v.nx, v.ny, parity);
    transpose<double>(p, x, v.xT, v.nx, v.ny);
    for (int parity = 0; parity < 2; ++parity)
      hipLaunchKernelGGL((k_zebra_x<StOpB<double>, double>), (v.nx - parity + 1) / 2,
                         kZebraThreads, zebra_shmem(v.ny, sizeof(double)), p->stream, opT, v.xT,
                         (const double *)v.bT, (const uint8_t *)v.dirT, v.ny, v.nx, parity);
    transpose<double>(p, (const double *)v.xT, x, v.ny, v.nx);
  }
}

// Smoothing on a stored-stencil level (the unfused cycle).
template <typename T>
void smooth_stored(tomg_problem *p, int l, const T *st, T *x, const T *b, int sweeps) {
  const tomg::Level &v = p->lv[l];
  if constexpr (std::is_same<T, double>::value) {
    if (p->cfg.smoother == TOMG_ZEBRA_XY) {
      smooth_level_xy(p, l, st, x, b, sweeps);
      return;
    }
  }
  smooth_level(p, st_op_b<T>(st, v.nx, v.ny), x, b, v.dir, v.nx, v.ny, sweeps);
}

template <class Op, typename T>
void restrict_level(tomg_problem *p, const Op &op, const T *x, const T *b, const uint8_t *dir,
                    int nxf, T *bc, int nxc, int nyc, const uint8_t *dirc = nullptr) {
  const dim3 blk(64, 4);
  hipLaunchKernelGGL((k_restrict<Op, T>), grid2(nxc, nyc, blk), blk, 0, p->stream, op, x, b, dir,
                     nxf, bc, nxc, nyc, dirc);
}

}  // namespace
// Threads of the coarsest solve: a wave for the small levels, up to 1024 for
// the large ones (one row of the inverse each).
static int coarse_solve_threads(const tomg_problem *p) {
  const long n = (long)p->lv[p->L - 1].nx * p->lv[p->L - 1].ny;
  return n <= 64 ? 64 : (n <= 256 ? 256 : 1024);
}

// First level handed to the single-workgroup tail: the first coarse level
// with at most tail_max_nodes() nodes and at most 4 levels below it.
int tail_level(const tomg_problem *p, bool batch) {
  // the tail gives each thread one node of its two coarsest levels: a large
  // coarsest level is solved on its own below the fused passes
  if (p->cband || (long)p->lv[p->L - 1].nx * p->lv[p->L - 1].ny > kSmallCoarseNodes)
    return p->L - 1;
  for (int l = 1; l < p->L; ++l)
    if ((long)p->lv[l].nx * p->lv[l].ny <= tail_max_nodes(batch) && p->L - l <= 4) return l;
  return p->L - 1;
}
namespace {

// One V(nu1, nu2) cycle on stored stencils (Neumann edges or the flux form):
// every level uses its stored stencil (level 0 included, with any Neumann
// ghost layer folded in) and its ring may hold free nodes, so the smoother covers the ring, the
// restriction fills free coarse ring nodes and the operator reads no node
// outside the grid.  One launch per colour, residual-restriction and
// prolongation.
template <typename T>
hipError_t run_vcycle_stored(tomg_problem *p, T *x0, const T *b0, const LevelView<T> *views,
                              bool zero0) {
  const int L = p->L;
  const dim3 blk(64, 4);
  for (int l = 0; l < L - 1; ++l) {
    const tomg::Level &lv = p->lv[l], &lc = p->lv[l + 1];
    T *x = l == 0 ? x0 : views[l].x;
    const T *b = l == 0 ? b0 : views[l].b;
    if (l > 0 || zero0) hipLaunchKernelGGL((k_zero<T>), grid1(lv.n), 256, 0, p->stream, x, lv.n);
    const StOpB<T> op = st_op_b<T>(views[l].st, lv.nx, lv.ny);
    smooth_stored<T>(p, l, views[l].st, x, b, p->cfg.nu1);
    // residual once per fine node, then its full weighting
    T *r = reinterpret_cast<T *>(p->tmp);
    hipLaunchKernelGGL((k_residual<StOpB<T>, T>), grid2(lv.nx, lv.ny, blk), blk, 0, p->stream, op,
                       (const T *)x, b, lv.dir, lv.nx, lv.ny, r);
    hipLaunchKernelGGL((k_full_weighting<T>), grid2(lc.nx, lc.ny, blk), blk, 0, p->stream,
                       (const T *)r, lv.nx, lv.ny, views[l + 1].b, lc.nx, lc.ny,
                       (const uint8_t *)lc.dir);
  }
  {
    const tomg::Level &lc = p->lv[L - 1];
    hipLaunchKernelGGL((k_coarse_solve<T>), 1, coarse_solve_threads(p), 0, p->stream, p->cinv, p->cidx,
                       (const T *)views[L - 1].b, views[L - 1].x, (int)lc.n);
  }
  for (int l = L - 2; l >= 0; --l) {
    const tomg::Level &lv = p->lv[l], &lc = p->lv[l + 1];
    T *x = l == 0 ? x0 : views[l].x;
    const T *b = l == 0 ? b0 : views[l].b;
    hipLaunchKernelGGL((k_prolong<T>), grid2(lv.nx, lv.ny, blk), blk, 0, p->stream,
                       (const T *)views[l + 1].x, lc.nx, x, lv.dir, lv.nx, lv.ny);
    smooth_stored<T>(p, l, views[l].st, x, b, p->cfg.nu2);
  }
  return hipGetLastError();
}

// Levels 1 .. L-1 of a four-colour cycle, between the level-0 passes: the
// fused down passes of levels 1 .. lc-1, the single-workgroup tail from
// level lc (or the coarsest solve alone), the fused up passes of levels
// lc-1 .. 1.
template <typename T>
static void coarse_levels(tomg_problem *p, const EpsOp<T> &op0, const LevelView<T> *views) {
  const int L = p->L;
  const int lc = p->lc;  // first level of the tail (the coarsest alone: no tail)
  for (int l = 1; l < lc; ++l)
    fused_down<T>(p, l, views[l].x, views[l].pong, views[l].b, op0.exx, op0.exy, op0.eyy,
                  views[l].st, views[l + 1].b, true);
  T *xs[kMaxLevels];
  T *bs[kMaxLevels];
  const T *sts[kMaxLevels];
  for (int l = 0; l < L; ++l) {
    xs[l] = views[l].x;
    bs[l] = views[l].b;
    sts[l] = views[l].st;
  }
  if (lc == L - 1)  // no tail: the coarsest solve alone
    hipLaunchKernelGGL((k_coarse_solve<T>), 1, coarse_solve_threads(p), 0, p->stream, p->cinv,
                       p->cidx, (const T *)views[L - 1].b, views[L - 1].x, (int)p->lv[L - 1].n);
  else
    tail_cycle<T>(p, lc, xs, bs, sts);
  for (int l = lc - 1; l >= 1; --l)
    fused_up<T>(p, l, views[l].pong, views[l].x, views[l].b, op0.exx, op0.exy, op0.eyy,
                views[l].st, views[l + 1].x, nullptr);
}

// k FP32 V-cycles of a refinement step from a zero start, the level-0 up
// pass of each cycle and the down pass of the next in one launch
// (fused_updown): the same relaxations in the same order as the cycles run
// one after another, so the same result bit for bit, with the level-0
// arrays moved once per cycle instead of twice.  The pre-smoothed level-0
// iterates alternate between e and e2 so that the last up pass leaves the
// correction in e.
static hipError_t run_inner_chain(tomg_problem *p, int k, float *e, float *e2, const float *b0,
                                  const EpsOp<float> &op0, const LevelView<float> *views) {
  auto pong = [&](int c) -> float * { return ((k - c) & 1) ? e : e2; };
  prof_begin(p, 0);
  fused_down<float>(p, 0, e, pong(1), b0, op0.exx, op0.exy, op0.eyy, views[0].st, views[1].b,
                    true);
  prof_end(p, 0);
  for (int c = 1; c <= k; ++c) {
    coarse_levels<float>(p, op0, views);
    if (c < k) {
      prof_begin(p, 2);
      fused_updown<float>(p, pong(c), pong(c + 1), b0, op0.exx, op0.exy, op0.eyy, views[0].st,
                          views[1].x, views[1].b);
      prof_end(p, 2);
    } else {
      prof_begin(p, 1);
      fused_up<float>(p, 0, pong(c), e, b0, op0.exx, op0.exy, op0.eyy, views[0].st, views[1].x,
                      nullptr);
      prof_end(p, 1);
    }
  }
  return hipGetLastError();
}

// One V(nu1, nu2) cycle in precision T.  x0/b0: level-0 iterate and rhs;
// op0: level-0 operator; coarse data from views[l].{x,b,st}.  zero0: the
// level-0 iterate starts at zero (not read).  With the four-colour smoother,
// every level above the tail is one fused down pass and one fused up pass
// and the small levels run in one workgroup; when partials is given, the
// level-0 up pass also leaves per-block sums of the squared final residual
// there (block count in *nblocks).
template <typename T>
hipError_t run_vcycle(tomg_problem *p, T *x0, const T *b0, const EpsOp<T> &op0,
                      const LevelView<T> *views, bool zero0, double *partials, int *nblocks) {
  const int L = p->L;
  const dim3 blk(64, 4);
  if (nblocks) *nblocks = 0;
  if (stored_level0(p->cfg) && p->cfg.smoother != TOMG_GS4)
    return run_vcycle_stored(p, x0, b0, views, zero0);
  if (p->cfg.smoother == TOMG_GS4) {
    prof_begin(p, 0);
    fused_down<T>(p, 0, x0, views[0].pong, b0, op0.exx, op0.exy, op0.eyy, views[0].st,
                  views[1].b, zero0);
    prof_end(p, 0);
    coarse_levels<T>(p, op0, views);
    prof_begin(p, 1);
    const int nb = fused_up<T>(p, 0, views[0].pong, x0, b0, op0.exx, op0.exy, op0.eyy,
                               views[0].st, views[1].x, partials);
    prof_end(p, 1);
    if (nblocks) *nblocks = partials ? nb : 0;
    return hipGetLastError();
  }
  // damped Jacobi: one launch per step
  for (int l = 0; l < L - 1; ++l) {
    const tomg::Level &lv = p->lv[l], &lc = p->lv[l + 1];
    T *x = l == 0 ? x0 : views[l].x;
    const T *b = l == 0 ? b0 : views[l].b;
    if (l > 0 || zero0) hipLaunchKernelGGL((k_zero<T>), grid1(lv.n), 256, 0, p->stream, x, lv.n);
    if (l > 0) {
      const StOp<T> op = st_op<T>(views[l].st, lv.nx, lv.ny);
      smooth_level(p, op, x, b, lv.dir, lv.nx, lv.ny, p->cfg.nu1);
      restrict_level(p, op, x, b, lv.dir, lv.nx, views[l + 1].b, lc.nx, lc.ny);
    } else {
      smooth_level(p, op0, x, b, lv.dir, lv.nx, lv.ny, p->cfg.nu1);
      restrict_level(p, op0, x, b, lv.dir, lv.nx, views[1].b, lc.nx, lc.ny);
    }
  }
  {
    const tomg::Level &lc = p->lv[L - 1];
    hipLaunchKernelGGL((k_coarse_solve<T>), 1, coarse_solve_threads(p), 0, p->stream, p->cinv, p->cidx,
                       (const T *)views[L - 1].b, views[L - 1].x, (int)lc.n);
  }
  for (int l = L - 2; l >= 0; --l) {
    const tomg::Level &lv = p->lv[l], &lc = p->lv[l + 1];
    T *x = l == 0 ? x0 : views[l].x;
    const T *b = l == 0 ? b0 : views[l].b;
    hipLaunchKernelGGL((k_prolong<T>), grid2(lv.nx, lv.ny, blk), blk, 0, p->stream,
                       (const T *)views[l + 1].x, lc.nx, x, lv.dir, lv.nx, lv.ny);
    if (l > 0) {
      const StOp<T> op = st_op<T>(views[l].st, lv.nx, lv.ny);
      smooth_level(p, op, x, b, lv.dir, lv.nx, lv.ny, p->cfg.nu2);
    } else {
      smooth_level(p, op0, x, b, lv.dir, lv.nx, lv.ny, p->cfg.nu2);
    }
  }
  return hipGetLastError();
}

EpsOp<double> op64(tomg_problem *p) {
  return eps_op<double>(p->exx, p->exy, p->eyy, p->cfg.nx, p->cfg.dx, p->cfg.dy);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------

hipError_t launch_setup(tomg_problem *p, const double *xp, const double *yp, const double *jac,
                        const double *epsp, const double *rho, const uint8_t *mask) {
  const int nx = p->cfg.nx, ny = p->cfg.ny;
  const bool f32 = p->cfg.precision == TOMG_FP32_IR;
  hipLaunchKernelGGL(k_setup, kRedBlocks, kRedThreads, 0, p->stream, nx, ny, p->cfg.dx,
                     p->cfg.dy, xp, yp, jac, epsp, rho, mask, p->exx, p->exy, p->eyy, p->det,
                     p->f, p->lv[0].dir, f32 ? p->exx32 : nullptr, f32 ? p->exy32 : nullptr,
                     f32 ? p->eyy32 : nullptr, p->partials, p->cfg.neumann);
  return finish_setup(p);
}

// After a level-0 setup kernel: its min-det and non-finite checks into the
// scalar block, and the stored level-0 stencil where the problem has one.
hipError_t finish_setup(tomg_problem *p) {
  const int ny = p->cfg.ny;
  const bool f32 = p->cfg.precision == TOMG_FP32_IR;
  hipLaunchKernelGGL((k_finalize<1>), 1, kRedThreads, 0, p->stream, p->partials, kRedBlocks, 2,
                     p->scal + kSlotMinDet, 0, p->scal, 0, nullptr);
  hipLaunchKernelGGL((k_finalize<0>), 1, kRedThreads, 0, p->stream, p->partials + 1, kRedBlocks,
                     2, p->scal + kSlotBad, 0, p->scal, 0, nullptr);
  if (stored_level0(p->cfg)) {
    hipLaunchKernelGGL(k_fold_stencil, kRedBlocks, kRedThreads, 0, p->stream, op64(p), ny,
                       (const uint8_t *)p->lv[0].dir, p->lv[0].st, p->cfg.flux);
    if (f32)  // the FP32 inner cycles relax with a rounded copy
      hipLaunchKernelGGL(k_narrow, 4096, 256, 0, p->stream, (const double *)p->lv[0].st,
                         p->lv[0].st32, 9 * p->lv[0].n);
  }
  return hipGetLastError();
}

hipError_t launch_setup_desc(tomg_problem *p, const tomg_map_desc &m, const tomg_source_desc &src,
                             double *phi_init) {
  const tomg_config &c = p->cfg;
  const bool f32 = c.precision == TOMG_FP32_IR;
#define TOMG_DESC(KIND)                                                                        \
  hipLaunchKernelGGL(k_setup_desc<KIND>, kRedBlocks, kRedThreads, 0, p->stream, c.nx, c.ny,     \
                     c.xi0, c.eta0, c.dx, c.dy, m, src, p->exx, p->exy, p->eyy, p->det, p->f,  \
                     p->lv[0].dir, f32 ? p->exx32 : nullptr, f32 ? p->exy32 : nullptr,         \
                     f32 ? p->eyy32 : nullptr, phi_init, p->partials, c.neumann)
  if (m.kind == TOMG_MAP_SINUSOIDAL) TOMG_DESC(TOMG_MAP_SINUSOIDAL);
  else if (m.kind == TOMG_MAP_POLAR) TOMG_DESC(TOMG_MAP_POLAR);
  else TOMG_DESC(TOMG_MAP_PERTURBED_CIRCLE);
#undef TOMG_DESC
  return finish_setup(p);
}

hipError_t launch_update_rhs_desc(tomg_problem *p, const tomg_map_desc &m,
                                  const tomg_source_desc &src) {
  const tomg_config &c = p->cfg;
#define TOMG_DESC(KIND)                                                                        \
  hipLaunchKernelGGL(k_update_rhs_desc<KIND>, kRedBlocks, kRedThreads, 0, p->stream, c.nx,      \
                     c.ny, c.xi0, c.eta0, c.dx, c.dy, m, src, (const double *)p->det, p->f,     \
                     p->partials)
  if (m.kind == TOMG_MAP_SINUSOIDAL) TOMG_DESC(TOMG_MAP_SINUSOIDAL);
  else if (m.kind == TOMG_MAP_POLAR) TOMG_DESC(TOMG_MAP_POLAR);
  else TOMG_DESC(TOMG_MAP_PERTURBED_CIRCLE);
#undef TOMG_DESC
  hipLaunchKernelGGL((k_finalize<0>), 1, kRedThreads, 0, p->stream, p->partials, kRedBlocks, 1,
                     p->scal + kSlotBadRhs, 0, p->scal, 0, nullptr);
  return hipGetLastError();
}

hipError_t launch_field(tomg_problem *p, const double *phi, const double *xp, const double *yp,
                        const double *jac, double *ex, double *ey) {
  hipLaunchKernelGGL(k_field, 2048, 256, 0, p->stream, p->cfg.nx, p->cfg.ny, p->cfg.dx, p->cfg.dy,
                     phi, xp, yp, jac, ex, ey);
  return hipGetLastError();
}

hipError_t upload_args(tomg_problem *p) {
  static_assert(sizeof(ArgsBlob) % sizeof(uint64_t) == 0, "blob of whole words");
  const int nw = (int)(sizeof(ArgsBlob) / sizeof(uint64_t));
  const uint64_t *src = reinterpret_cast<const uint64_t *>(&p->hargs);
  uint64_t *dst = reinterpret_cast<uint64_t *>(p->dargs);
  WordChunk c;
  for (int w0 = 0; w0 < nw; w0 += kWordsPerStore) {
    const int n = std::min(kWordsPerStore, nw - w0);
    std::memcpy(c.w, src + w0, n * sizeof(uint64_t));
    hipLaunchKernelGGL(k_store_words, 1, 256, 0, p->stream, dst + w0, c, n);
  }
  return hipGetLastError();
}

hipError_t launch_set_slots(tomg_problem *p, unsigned mask, double v) {
  hipLaunchKernelGGL(k_set_slots, 1, 64, 0, p->stream, p->scal, mask, v);
  return hipGetLastError();
}

hipError_t launch_zero(tomg_problem *p, double *x, size_t n) {
  hipLaunchKernelGGL((k_zero<double>), grid1(n), 256, 0, p->stream, x, n);
  return hipGetLastError();
}

hipError_t launch_setup_identity(tomg_problem *p, const uint8_t *mask) {
  const bool f32 = p->cfg.precision == TOMG_FP32_IR;
  hipLaunchKernelGGL(k_setup_identity, kRedBlocks, kRedThreads, 0, p->stream, p->cfg.nx,
                     p->cfg.ny, p->exx, p->exy, p->eyy, p->det, p->f, p->lv[0].dir, mask,
                     f32 ? p->exx32 : nullptr, f32 ? p->exy32 : nullptr,
                     f32 ? p->eyy32 : nullptr, p->partials);
  hipLaunchKernelGGL((k_finalize<1>), 1, kRedThreads, 0, p->stream, p->partials, kRedBlocks, 2,
                     p->scal + kSlotMinDet, 0, p->scal, 0, nullptr);
  hipLaunchKernelGGL((k_finalize<0>), 1, kRedThreads, 0, p->stream, p->partials + 1, kRedBlocks,
                     2, p->scal + kSlotBad, 0, p->scal, 0, nullptr);
  return hipGetLastError();
}

hipError_t launch_update_rhs(tomg_problem *p, const double *rho) {
  const size_t n = p->lv[0].n;
  hipLaunchKernelGGL(k_update_rhs, kRedBlocks, kRedThreads, 0, p->stream, rho, p->det, p->f, n,
                     p->partials);
  hipLaunchKernelGGL((k_finalize<0>), 1, kRedThreads, 0, p->stream, p->partials, kRedBlocks, 1,
                     p->scal + kSlotBadRhs, 0, p->scal, 0, nullptr);
  return hipGetLastError();
}

hipError_t launch_hierarchy(tomg_problem *p, bool defer_inverse) {
  const bool f32 = p->cfg.precision == TOMG_FP32_IR;
  for (int l = 1; l < p->L; ++l) {
    const tomg::Level &lf = p->lv[l - 1], &lc = p->lv[l];
    const dim3 grid((lc.nx + kGX - 1) / kGX, (lc.ny + kGY - 1) / kGY);
    float *st32 = f32 ? lc.st32 : nullptr;
    if (p->cfg.coarse_op == TOMG_REDISCRETIZE) {
      const double H = p->cfg.dx * (double)(1 << l), K = p->cfg.dy * (double)(1 << l);
      hipLaunchKernelGGL(k_rediscretize, grid1(lc.n), 256, 0, p->stream, (const double *)p->exx,
                         (const double *)p->exy, (const double *)p->eyy,
                         (const uint8_t *)p->lv[0].dir, p->cfg.nx, 1 << l, lc.nx, lc.ny,
                         1.0 / (H * H), 1.0 / (K * K), 0.25 / (H * H), 0.25 / (K * K),
                         0.25 / (H * K), 0.5 / (H * K), lc.dir, lc.st, st32);
    } else if (lf.ck != 0) {  // one axis halved
      const int sx = lf.ck == 1 ? 2 : 1, sy = lf.ck == 2 ? 2 : 1;
      hipLaunchKernelGGL(k_coarse_flags_semi, grid1(lc.n), 256, 0, p->stream,
                         (const uint8_t *)lf.dir, lf.nx, lf.ny, lc.nx, lc.ny, sx, sy, lc.dir);
      const uint8_t *df = lf.dir, *dc = lc.dir;
      if (l == 1 && !stored_level0(p->cfg)) {
        if (sx == 2)
          hipLaunchKernelGGL((k_coarsen_semi<EpsOp<double>, 2, 1>), grid1(lc.n), 256, 0,
                             p->stream, op64(p), df, lf.nx, lf.ny, lc.nx, lc.ny, dc, lc.st, st32);
        else
          hipLaunchKernelGGL((k_coarsen_semi<EpsOp<double>, 1, 2>), grid1(lc.n), 256, 0,
                             p->stream, op64(p), df, lf.nx, lf.ny, lc.nx, lc.ny, dc, lc.st, st32);
      } else {
        const StOp<double> op = st_op<double>(lf.st, lf.nx, lf.ny);
        if (sx == 2)
          hipLaunchKernelGGL((k_coarsen_semi<StOp<double>, 2, 1>), grid1(lc.n), 256, 0,
                             p->stream, op, df, lf.nx, lf.ny, lc.nx, lc.ny, dc, lc.st, st32);
        else
          hipLaunchKernelGGL((k_coarsen_semi<StOp<double>, 1, 2>), grid1(lc.n), 256, 0,
                             p->stream, op, df, lf.nx, lf.ny, lc.nx, lc.ny, dc, lc.st, st32);
      }
    } else if (l == 1 && !stored_level0(p->cfg))
      hipLaunchKernelGGL(k_coarsen_eps, grid, kGX * kGY, 0, p->stream, op64(p), lf.dir, lf.nx,
                         lf.ny, lc.nx, lc.ny, lc.dir, lc.st, st32);
    else
      hipLaunchKernelGGL((k_coarsen<StOp<double>>), grid, kGX * kGY, 0, p->stream,
                         st_op<double>(lf.st, lf.nx, lf.ny), lf.dir, lf.nx, lf.ny, lc.nx, lc.ny,
                         lc.dir, lc.st, st32);
  }
  p->inv_pending = true;
  if (!defer_inverse) {
    const hipError_t e = launch_coarse_inverse(p);
    if (e != hipSuccess) return e;
  }
  if (p->cfg.smoother == TOMG_ZEBRA_XY)
    // the transposed levels of the y-line sweeps: plane (di, dj) becomes (dj, di)
    for (int l = 0; l < p->L; ++l) {
      const tomg::Level &v = p->lv[l];
      for (int k = 0; k < 9; ++k) {
        const int di = k % 3 - 1, dj = k / 3 - 1, kt = (di + 1) * 3 + (dj + 1);
        transpose<double>(p, v.st + (size_t)k * v.n, v.stT + (size_t)kt * v.n, v.nx, v.ny);
      }
      transpose<uint8_t>(p, v.dir, v.dirT, v.nx, v.ny);
    }
  return hipGetLastError();
}

hipError_t launch_coarse_inverse(tomg_problem *p) {
  if (!p->inv_pending) return hipSuccess;
  if (p->cband)
    hipLaunchKernelGGL(k_coarse_inverse_band, 1, kInvThreads, 0, p->stream, p->hargs.inv);
  else
    hipLaunchKernelGGL(k_coarse_inverse, 1, kInvThreads, 0, p->stream, p->hargs.inv);
  p->inv_pending = false;
  return hipGetLastError();
}

void batch_coarse_inverse(tomg_problem *const *probs, const int *idx, int cnt, hipStream_t s) {
  BatchTab tab;
  tab.count = 0;
  auto flush = [&] {
    if (tab.count) hipLaunchKernelGGL(k_coarse_inverse_b, tab.count, kInvThreads, 0, s, tab);
    tab.count = 0;
  };
  for (int k = 0; k < cnt; ++k) {
    tomg_problem *p = probs[idx[k]];
    if (!p->inv_pending) continue;
    if (p->cband) {  // a large coarsest level: its own launch
      (void)launch_coarse_inverse(p);
      continue;
    }
    BatchEntry &e = tab.e[tab.count];
    e.args = &p->dargs->inv;
    e.phi = nullptr;
    e.role = 0;
    e.nbx = e.nby = 1;
    e.start = tab.count;
    e.slot = e.out = 0;
    ++tab.count;
    p->inv_pending = false;
    if (tab.count == kBatchMax) flush();
  }
  flush();
}

hipError_t launch_vcycle64(tomg_problem *p, double *phi, bool with_norm) {
  LevelView<double> v[kMaxLevels];
  for (int l = 0; l < p->L; ++l) v[l] = {p->lv[l].x, p->lv[l].b, p->lv[l].st, p->lv[l].x2};
  v[0].pong = p->tmp;
  int nb = 0;
  hipError_t e = run_vcycle<double>(p, phi, p->f, op64(p), v, false,
                                    with_norm ? p->partials : nullptr, &nb);
  if (e != hipSuccess || !with_norm) return e;
  if (nb > 0) {
    hipLaunchKernelGGL((k_finalize<0>), 1, kRedThreads, 0, p->stream, p->partials, nb, 1,
                       p->scal + kSlotRes, 1, p->scal, 2, p->skip);
    return hipGetLastError();
  }
  // no level-0 pass left norm partials (the Jacobi path): a separate norm
  const RedArgs &r = p->hargs.red;
  if (r.st0)
    hipLaunchKernelGGL((k_red<kRmNorm, true>), r.nblk, kRedTileW, 0, p->stream, r, phi, nullptr,
                       nullptr);
  else
    hipLaunchKernelGGL((k_red<kRmNorm, false>), r.nblk, kRedTileW, 0, p->stream, r, phi,
                       nullptr, nullptr);
  hipLaunchKernelGGL((k_finalize<0>), 1, kRedThreads, 0, p->stream, p->partials, r.nblk, 1,
                     p->scal + kSlotRes, 1, p->scal, 2, nullptr);
  return hipGetLastError();
}

int red_tiles(int nx, int ny) {
  return ((nx + kRedTileW - 3) / (kRedTileW - 2)) * ((ny + kRedTileH - 1) / kRedTileH);
}

void build_red_args(tomg_problem *p) {
  RedArgs &r = p->hargs.red;
  r.exx = p->exx;
  r.exy = p->exy;
  r.eyy = p->eyy;
  const double dx = p->cfg.dx, dy = p->cfg.dy;
  r.cx = 1.0 / (dx * dx);
  r.cy = 1.0 / (dy * dy);
  r.qx = 0.25 / (dx * dx);
  r.qy = 0.25 / (dy * dy);
  r.qxy = 0.25 / (dx * dy);
  r.hxy = 0.5 / (dx * dy);
  r.nx = p->cfg.nx;
  r.ny = p->cfg.ny;
  r.f = p->f;
  r.dir = p->lv[0].dir;
  r.partials = p->partials;
  r.r32 = p->r32;
  r.e32 = p->e32;
  r.tmp = p->tmp;
  r.st0 = stored_level0(p->cfg) ? p->lv[0].st : nullptr;
  r.phi2 = p->phi2;
  r.nblk = red_tiles(p->cfg.nx, p->cfg.ny);
  p->hargs.fin_red = {p->partials, p->scal, r.nblk};
  p->hargs.fin_red0 = {p->partials + r.nblk, p->scal, r.nblk};
  const PassArgs<double> &u = p->hargs.up64[0], &ub = p->hargs.up64b[0];
  p->hargs.fin_norm = {p->partials, p->scal, u.nbx * u.nby};
  p->hargs.fin_normb = {p->partials, p->scal, ub.nbx * ub.nby};
  const Level &lc = p->lv[p->L - 1];
  p->hargs.inv = {lc.st, lc.dir, p->cband, lc.nx, lc.ny, p->cinv, p->cidx, p->scal};
}

template <int M>
static void launch_red(tomg_problem *p, const double *x, double *xo, const double *skip) {
  const RedArgs &r = p->hargs.red;
  if (r.st0)
    hipLaunchKernelGGL((k_red<M, true>), r.nblk, kRedTileW, 0, p->stream, r, x, xo, skip);
  else
    hipLaunchKernelGGL((k_red<M, false>), r.nblk, kRedTileW, 0, p->stream, r, x, xo, skip);
}

hipError_t launch_ir_residual(tomg_problem *p, const double *phi) {
  const RedArgs &r = p->hargs.red;
  launch_red<kRmIrRes>(p, phi, nullptr, p->skip);
  hipLaunchKernelGGL((k_finalize<0>), 1, kRedThreads, 0, p->stream, p->partials, r.nblk, 1,
                     p->scal + kSlotRes, 1, p->scal, 2, p->skip);
  return hipGetLastError();
}

// Initial norms of a solve in one pass over level 0: |f - A phi0| into
// scal[kSlotB0] and the residual of phi into scal[kSlotRes] (and the
// relative residual); with ir also r32 (the refinement residual).
hipError_t launch_begin(tomg_problem *p, const double *phi, bool ir) {
  const RedArgs &r = p->hargs.red;
  if (ir)
    launch_red<kRmIrResB0>(p, phi, nullptr, nullptr);
  else
    launch_red<kRmBegin>(p, phi, nullptr, nullptr);
  hipLaunchKernelGGL((k_finalize<0>), 1, kRedThreads, 0, p->stream, p->partials + r.nblk,
                     r.nblk, 1, p->scal + kSlotB0, 1, p->scal, 0, nullptr);
  hipLaunchKernelGGL((k_finalize<0>), 1, kRedThreads, 0, p->stream, p->partials, r.nblk, 1,
                     p->scal + kSlotRes, 1, p->scal, 1, nullptr);
  return hipGetLastError();
}

// One refinement step after the inner cycles: phi += e32 and the new
// residual in one pass; the iterate moves from the caller's array to phi2
// (second = false) or back (second = true).
hipError_t launch_ir_step(tomg_problem *p, double *phi, bool second) {
  const RedArgs &r = p->hargs.red;
  if (second)
    launch_red<kRmIrStep>(p, p->phi2, phi, p->skip);
  else
    launch_red<kRmIrStep>(p, phi, p->phi2, p->skip);
  hipLaunchKernelGGL((k_finalize<0>), 1, kRedThreads, 0, p->stream, p->partials, r.nblk, 1,
                     p->scal + kSlotRes, 1, p->scal, 2, p->skip);
  return hipGetLastError();
}

hipError_t launch_ir_correct(tomg_problem *p, double *phi) {
  hipError_t e = launch_ir_inner(p);
  if (e != hipSuccess) return e;
  const RedArgs &r = p->hargs.red;
  hipLaunchKernelGGL(k_ir_update, r.nblk, kRedTileW, 0, p->stream, r, phi, p->skip);
  return hipGetLastError();
}

// The inner FP32 cycles of a refinement step: e32 from r32.
hipError_t launch_ir_inner(tomg_problem *p) {
  const int nx = p->cfg.nx;
  LevelView<float> v[kMaxLevels];
  for (int l = 0; l < p->L; ++l)
    v[l] = {p->lv[l].x32, p->lv[l].b32, p->lv[l].st32, p->lv[l].x2_32};
  v[0].pong = p->e32b;
  const EpsOp<float> o32 = eps_op<float>(p->exx32, p->exy32, p->eyy32, nx, p->cfg.dx, p->cfg.dy);
  if (chain_inner(p))
    return run_inner_chain(p, p->cfg.ir_inner_cycles, p->e32, p->e32b, p->r32, o32, v);
  for (int k = 0; k < p->cfg.ir_inner_cycles; ++k) {
    hipError_t e = run_vcycle<float>(p, p->e32, p->r32, o32, v, k == 0, nullptr, nullptr);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}


// ---- batched reductions ----------------------------------------------------

// roles (nullable, indexed like probs): the BatchEntry role of each problem.
template <int KIND>
static void batch_red(tomg_problem *const *probs, const int *idx, int cnt, double *const *phis,
                      hipStream_t s, const int *roles = nullptr) {
  BatchTab tab;
  for (int k0 = 0; k0 < cnt; k0 += kBatchMax) {
    tab.count = 0;
    int nb = 0;
    for (int k = k0; k < cnt && k < k0 + kBatchMax; ++k) {
      tomg_problem *p = probs[idx[k]];
      BatchEntry &e = tab.e[tab.count++];
      e.args = &p->dargs->red;
      e.phi = phis[idx[k]];
      e.role = roles ? roles[idx[k]] : 0;
      e.nbx = p->hargs.red.nblk;
      e.nby = 1;
      e.start = nb;
      e.slot = e.out = 0;
      nb += e.nbx;
    }
    if (!tab.count) continue;
    if (probs[idx[k0]]->hargs.red.st0)
      hipLaunchKernelGGL((k_red_b<KIND, true>), nb, kRedTileW, 0, s, tab);
    else
      hipLaunchKernelGGL((k_red_b<KIND, false>), nb, kRedTileW, 0, s, tab);
  }
}

void batch_resnorm(tomg_problem *const *probs, const int *idx, int cnt, bool zero_free,
                   double *const *phis, hipStream_t s) {
  if (zero_free)
    batch_red<kRmNormZF>(probs, idx, cnt, phis, s);
  else
    batch_red<kRmNorm>(probs, idx, cnt, phis, s);
}

void batch_ir_residual(tomg_problem *const *probs, const int *idx, int cnt, double *const *phis,
                       hipStream_t s) {
  batch_red<kRmIrRes>(probs, idx, cnt, phis, s);
}

void batch_begin_norms(tomg_problem *const *probs, const int *idx, int cnt, bool ir,
                       double *const *phis, hipStream_t s) {
  if (ir)
    batch_red<kRmIrResB0>(probs, idx, cnt, phis, s);
  else
    batch_red<kRmBegin>(probs, idx, cnt, phis, s);
}

void batch_ir_update(tomg_problem *const *probs, const int *idx, int cnt, double *const *phis,
                     hipStream_t s) {
  batch_red<-1>(probs, idx, cnt, phis, s);
}

void batch_ir_step(tomg_problem *const *probs, const int *idx, int cnt, double *const *phis,
                   const int *roles, hipStream_t s) {
  batch_red<kRmIrStep>(probs, idx, cnt, phis, s, roles);
}

void batch_copy_back(tomg_problem *const *probs, const int *idx, int cnt, double *const *phis,
                     hipStream_t s) {
  batch_red<-2>(probs, idx, cnt, phis, s);
}

void batch_finalize(tomg_problem *const *probs, const int *idx, int cnt, int kind, int slot,
                    int rel, double *out, hipStream_t s, bool by_index) {
  BatchTab tab;
  for (int k0 = 0; k0 < cnt; k0 += kBatchMax) {
    tab.count = 0;
    for (int k = k0; k < cnt && k < k0 + kBatchMax; ++k) {
      tomg_problem *p = probs[idx[k]];
      BatchEntry &e = tab.e[tab.count];
      e.args = kind == 0   ? (const void *)&p->dargs->fin_red
               : kind == 1 ? (const void *)&p->dargs->fin_normb
                           : (const void *)&p->dargs->fin_red0;
      e.phi = nullptr;
      e.role = 0;
      e.nbx = e.nby = 1;
      e.start = tab.count;
      e.slot = slot;
      e.out = by_index ? idx[k] : k;
      ++tab.count;
    }
    if (tab.count)
      hipLaunchKernelGGL(k_finalize_b, tab.count, kRedThreads, 0, s, tab, rel, out);
  }
}

hipError_t launch_smooth0(tomg_problem *p, double *phi, int sweeps) {
  if (p->cfg.smoother == TOMG_ZEBRA_XY)
    smooth_level_xy(p, 0, p->lv[0].st, phi, (const double *)p->f, sweeps);
  else if (stored_level0(p->cfg))
    smooth_level(p, st_op_b<double>(p->lv[0].st, p->cfg.nx, p->cfg.ny), phi,
                 (const double *)p->f, p->lv[0].dir, p->cfg.nx, p->cfg.ny, sweeps);
  else
    smooth_level(p, op64(p), phi, (const double *)p->f, p->lv[0].dir, p->cfg.nx, p->cfg.ny,
                 sweeps);
  return hipGetLastError();
}

hipError_t launch_copy_probe(const void *src, void *dst, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 16;
  hipLaunchKernelGGL(k_copy16, 2048, 256, 0, s, (const double2 *)src, (double2 *)dst, n);
  return hipGetLastError();
}

void prof_begin(tomg_problem *p, int kind) {
  if (!p->prof || p->nev[kind] >= tomg_problem::kMaxEv) return;
  (void)hipEventRecord(p->ev[kind][p->nev[kind]][0], p->stream);
}

void prof_end(tomg_problem *p, int kind) {
  if (!p->prof || p->nev[kind] >= tomg_problem::kMaxEv) return;
  (void)hipEventRecord(p->ev[kind][p->nev[kind]][1], p->stream);
  ++p->nev[kind];
}

// Called after the stream has been synchronised.
void prof_harvest(tomg_problem *p) {
  if (!p->prof) return;
  for (int kind = 0; kind < tomg_problem::kProfKinds; ++kind) {
    for (int e = 0; e < p->nev[kind]; ++e) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, p->ev[kind][e][0], p->ev[kind][e][1]) == hipSuccess) {
        p->prof_ms[kind] += ms;
        p->prof_cnt[kind] += 1.0;
      }
    }
    p->nev[kind] = 0;
  }
}

hipError_t launch_residual0(tomg_problem *p, const double *phi, double *r) {
  const dim3 blk(64, 4);
  if (stored_level0(p->cfg)) {
    hipLaunchKernelGGL((k_residual<StOpB<double>, double>), grid2(p->cfg.nx, p->cfg.ny, blk), blk,
                       0, p->stream, st_op_b<double>(p->lv[0].st, p->cfg.nx, p->cfg.ny), phi,
                       (const double *)p->f, p->lv[0].dir, p->cfg.nx, p->cfg.ny, r);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_residual<EpsOp<double>, double>), grid2(p->cfg.nx, p->cfg.ny, blk), blk,
                     0, p->stream, op64(p), phi, (const double *)p->f, p->lv[0].dir, p->cfg.nx,
                     p->cfg.ny, r);
  return hipGetLastError();
}

}  // namespace tomg

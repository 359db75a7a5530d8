// Fused level passes of the V-cycle (arXiv 2602.01888, Section 3), gfx950.
//
// One launch does, on one grid level, everything between two grid
// transfers:
//   down pass: [zero start] + nu four-colour Gauss-Seidel sweeps + residual
//              (eq. 20) + full-weighting restriction into the coarse
//              right-hand side (eq. 23);
//   up pass:   bilinear prolongation and correction on load (eq. 24) + nu
//              sweeps [+ partial sums of the final residual's squares].
//
// Block geometry: kBW threads own kBW consecutive columns (one each); the
// H = 4 nu + 2 outer columns on either side are halo, recomputed by the
// neighbouring block, so only W = kBW - 2H columns are written.  The block
// owns a band of CH rows and marches up it two rows at a time, starting
// HV = 2 nu + 3 rows below the band and stopping HV rows above it.  Node
// values of the rows in flight live in LDS; their stencil coefficients and
// right-hand side live in registers (a ring indexed by compile-time slots).
//
// The four-colour ordering (colour (i mod 2) + 2 (j mod 2), colours 0..3)
// is applied as a wavefront: at step k, sweep s relaxes colours 0 and 1 on
// even row 2k - 2s and then colours 2 and 3 on odd row 2k - 2s - 1.  An even
// row only reads odd rows that the current sweep has not reached yet and an
// odd row only reads even rows it has finished, so every node sees exactly
// the values the global colour-by-colour order gives it.  Each colour phase
// ends in a barrier.  Each sweep invalidates at most 4 halo columns and 2
// halo rows at the edges of the block, which is what H and HV cover.
#include <cmath>
#include <cstdlib>

#include "tomg_internal.h"

namespace tomg {
namespace {

#ifndef TOMG_BW
#define TOMG_BW 256
#endif
#ifndef TOMG_MIN_WAVES
#define TOMG_MIN_WAVES 1
#endif
constexpr int kBW = TOMG_BW;

template <typename T>
struct PassArgs {
  int nx, ny;
  const T *xin;             // level iterate read (unless ZERO)
  T *xout;                  // level iterate written (never the array read:
                            // neighbouring blocks read their halo from xin)
  const T *b;               // level right-hand side
  const uint8_t *dir;       // Dirichlet flags of the level
  const T *exx, *exy, *eyy; // level 0: permittivity tensor
  const T *st;              // coarse levels: 9-point stencil planes
  T cx, cy, qx, qy, qxy, hxy;
  const T *xc;              // up pass: coarse correction
  T *bc;                    // down pass: coarse right-hand side
  int nxc, nyc;
  double *partials;         // up pass with norm: one double per block
  int CH, W;
};

// Per-thread values of one row as loaded from global memory.
template <typename T, bool EPS>
struct Raw;
template <typename T>
struct Raw<T, true> {
  T x, f, xx, xy, yy, c00, c01, c10, c11;
  int d;
};
template <typename T>
struct Raw<T, false> {
  T x, f, a[9], c00, c01, c10, c11;
  int d;
};

// Coefficients of one row held in registers.  ik = 1 / diagonal, and 0 at
// Dirichlet nodes (which are never relaxed).
template <typename T, bool EPS>
struct Rec;
template <typename T>
struct Rec<T, true> {
  T ax, ay, gx, gy, k6, f, ik;
};
template <typename T>
struct Rec<T, false> {
  T a[9];
  T f, ik;
};

__device__ __forceinline__ int ring_slot(int o, int n) { return ((o % n) + n) % n; }

// Off-centre sum and diagonal of the node at LDS column t+1 of rows
// (lo, mid, hi) = (r-1, r, r+1): (A x)_c = off + dg x_c.
template <typename T>
__device__ __forceinline__ void apply_eps(const Rec<T, true> &c, const T *lo, const T *mid,
                                          const T *hi, int t, T &off, T &dg) {
  const T k1 = c.ax + c.gx, k3 = c.ax - c.gx, k4 = c.ay + c.gy, k5 = c.ay - c.gy;
  off = k1 * mid[t + 2] + k3 * mid[t] + k4 * hi[t + 1] + k5 * lo[t + 1] +
        c.k6 * ((hi[t + 2] - hi[t]) - (lo[t + 2] - lo[t]));
  dg = -T(2) * (c.ax + c.ay);
}
template <typename T>
__device__ __forceinline__ void apply_st(const Rec<T, false> &c, const T *lo, const T *mid,
                                         const T *hi, int t, T &off, T &dg) {
  off = c.a[0] * lo[t] + c.a[1] * lo[t + 1] + c.a[2] * lo[t + 2] + c.a[3] * mid[t] +
        c.a[5] * mid[t + 2] + c.a[6] * hi[t] + c.a[7] * hi[t + 1] + c.a[8] * hi[t + 2];
  dg = c.a[4];
}
template <typename T, bool EPS>
__device__ __forceinline__ void apply(const Rec<T, EPS> &c, const T *lo, const T *mid, const T *hi,
                                      int t, T &off, T &dg) {
  if constexpr (EPS)
    apply_eps<T>(c, lo, mid, hi, t, off, dg);
  else
    apply_st<T>(c, lo, mid, hi, t, off, dg);
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T *red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 1; k < kBW / 64; ++k) v += red[k];
  return v;
}

// Level 0 (EPS) prefetches the next row pair while it works on the current
// one; the stored-stencil levels load the current pair at the start of the
// step (their nine coefficient planes leave no registers for a second pair).
template <typename T, bool EPS, int NU, bool ZERO, bool PROLONG, bool RESTRICT, bool NORM>
__global__ __launch_bounds__(kBW, TOMG_MIN_WAVES) void k_pass(PassArgs<T> a) {
  constexpr int H = 4 * NU + 2;
  constexpr int HV = 2 * NU + 3;
  constexpr int NS = 2 * NU + 2;  // coefficient rows in flight: 2k-2NU .. 2k+1
  constexpr int NR = 2 * NU + 4;  // value rows in LDS:          2k-2NU-2 .. 2k+1
  __shared__ T L[NR][kBW + 2];
  __shared__ T xch[4][kBW + 2];
  __shared__ double red[kBW / 64];

  const int nx = a.nx, ny = a.ny;
  const int t = threadIdx.x;
  const int x0 = blockIdx.x * a.W;
  const int gi = x0 - H + t;
  const int gc = min(max(gi, 0), nx - 1);  // clamped column: loads never leave the array
  const bool inr = gi >= 0 && gi < nx;
  const bool updc = gi >= 1 && gi <= nx - 2;
  const bool outc = t >= H && t < H + a.W && gi < nx;
  const int odd = gi & 1;
  const int y0 = blockIdx.y * a.CH;
  const int y1 = min(ny, y0 + a.CH);
  const int ys = max(0, y0 - HV) & ~1;
  const int ye = min(ny - 1, y1 - 1 + HV);
  const int k0 = ys >> 1;
  const int k1 = (y1 - 1 + 2 * NU) >> 1;
  const size_t n = (size_t)nx * ny;
  const int Ic = gc >> 1;
  const int Ic1 = PROLONG ? min(Ic + 1, a.nxc - 1) : 0;

  for (int r = 0; r < NR; ++r) {
    L[r][t + 1] = T(0);
    if (t < 2) L[r][t * (kBW + 1)] = T(0);
  }
  if (t < 2)
    for (int r = 0; r < 4; ++r) xch[r][t * (kBW + 1)] = T(0);

  // all loads of a row are issued unconditionally from clamped addresses
  auto load_row = [&](int r, Raw<T, EPS> &w) {
    const int rc = min(max(r, 0), ny - 1);
    const size_t c = (size_t)rc * nx + gc;
    w.x = ZERO ? T(0) : a.xin[c];
    w.f = a.b[c];
    w.d = a.dir[c];
    if constexpr (EPS) {
      w.xx = a.exx[c];
      w.xy = a.exy[c];
      w.yy = a.eyy[c];
    } else {
#pragma unroll
      for (int z = 0; z < 9; ++z) w.a[z] = a.st[z * n + c];
    }
    if constexpr (PROLONG) {
      const int J = rc >> 1, J1 = min(J + 1, a.nyc - 1);
      const T *r0 = a.xc + (size_t)J * a.nxc;
      const T *r1 = a.xc + (size_t)J1 * a.nxc;
      w.c00 = r0[Ic];
      w.c01 = r0[Ic1];
      w.c10 = r1[Ic];
      w.c11 = r1[Ic1];
    }
  };
  // node value of a loaded row (plus the prolongated correction) into LDS
  auto commit_row = [&](int r, const Raw<T, EPS> &w) {
    const bool ld = r >= ys && r <= ye && inr;
    T v = ld ? w.x : T(0);
    if constexpr (PROLONG) {
      if (ld && !w.d && updc && r > 0 && r < ny - 1) {
        T e = odd ? T(0.5) * (w.c00 + w.c01) : w.c00;
        if (r & 1) {
          const T e1 = odd ? T(0.5) * (w.c10 + w.c11) : w.c10;
          e = T(0.5) * (e + e1);
        }
        v += e;
      }
    }
    L[ring_slot(r, NR)][t + 1] = v;
  };

  Rec<T, EPS> rec[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if constexpr (EPS) {
      rec[s].ax = rec[s].ay = rec[s].gx = rec[s].gy = rec[s].k6 = rec[s].f = T(0);
    } else {
#pragma unroll
      for (int q = 0; q < 9; ++q) rec[s].a[q] = T(0);
      rec[s].f = T(0);
    }
    rec[s].ik = T(0);
  }
  Raw<T, EPS> cur[2], nxt[2];
  // level 0: tensor values carried from earlier rows: row 2k-2 (eyy, exy)
  // and row 2k-1 (exx, exy, eyy, f, dir)
  T c_yy2 = T(0), c_xy2 = T(0), c_xx1 = T(0), c_xy1 = T(0), c_yy1 = T(0), c_f1 = T(0);
  int c_d1 = 1;
  (void)c_yy2; (void)c_xy2; (void)c_xx1; (void)c_xy1; (void)c_yy1; (void)c_f1; (void)c_d1;
  T rprev = T(0), acc = T(0);

  if constexpr (EPS) {  // prologue: the first row pair
    load_row(2 * k0, cur[0]);
    load_row(2 * k0 + 1, cur[1]);
    commit_row(2 * k0, cur[0]);
    commit_row(2 * k0 + 1, cur[1]);
  }
  __syncthreads();

  for (int kb = k0; kb <= k1; kb += NU + 1) {
#pragma unroll
    for (int ph = 0; ph <= NU; ++ph) {
      const int k = kb + ph;
      if (k <= k1) {
        const int ra = 2 * k;  // rows ra, ra+1 are the newest in the window
        if constexpr (EPS) {
          // prefetch the next pair; committed at the end of this step
          load_row(ra + 2, nxt[0]);
          load_row(ra + 3, nxt[1]);
          // coefficients of rows ra-1 and ra
          xch[0][t + 1] = c_xx1;
          xch[1][t + 1] = c_xy1;
          xch[2][t + 1] = cur[0].xx;
          xch[3][t + 1] = cur[0].xy;
          __syncthreads();
          {
            Rec<T, true> &R = rec[ring_slot(2 * ph - 1, NS)];
            R.ax = c_xx1 * a.cx;
            R.ay = c_yy1 * a.cy;
            R.gx = (xch[0][t + 2] - xch[0][t]) * a.qx + (cur[0].xy - c_xy2) * a.qxy;
            R.gy = (cur[0].yy - c_yy2) * a.qy + (xch[1][t + 2] - xch[1][t]) * a.qxy;
            R.k6 = c_xy1 * a.hxy;
            R.f = c_f1;
            R.ik = c_d1 ? T(0) : T(-1) / (T(2) * (R.ax + R.ay));
          }
          {
            Rec<T, true> &R = rec[ring_slot(2 * ph, NS)];
            R.ax = cur[0].xx * a.cx;
            R.ay = cur[0].yy * a.cy;
            R.gx = (xch[2][t + 2] - xch[2][t]) * a.qx + (cur[1].xy - c_xy1) * a.qxy;
            R.gy = (cur[1].yy - c_yy1) * a.qy + (xch[3][t + 2] - xch[3][t]) * a.qxy;
            R.k6 = cur[0].xy * a.hxy;
            R.f = cur[0].f;
            R.ik = cur[0].d ? T(0) : T(-1) / (T(2) * (R.ax + R.ay));
          }
        } else {
          load_row(ra, cur[0]);
          load_row(ra + 1, cur[1]);
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            Rec<T, false> &R = rec[ring_slot(2 * ph + q, NS)];
#pragma unroll
            for (int z = 0; z < 9; ++z) R.a[z] = cur[q].a[z];
            R.f = cur[q].f;
            R.ik = cur[q].d ? T(0) : T(1) / cur[q].a[4];
            commit_row(ra + q, cur[q]);
          }
          __syncthreads();
        }
        // ---------------- sweeps ----------------
#pragma unroll
        for (int s = 0; s < NU; ++s) {
#pragma unroll
          for (int half = 0; half < 2; ++half) {
            const int r = ra - 2 * s - half;  // even row first, then the odd row below
            const bool rowok = r >= 1 && r <= ny - 2 && r > ys && r < ye;
            const Rec<T, EPS> &R = rec[ring_slot(2 * ph - 2 * s - half, NS)];
            T *mid = L[ring_slot(r, NR)];
            const T *lo = L[ring_slot(r - 1, NR)];
            const T *hi = L[ring_slot(r + 1, NR)];
#pragma unroll
            for (int cp = 0; cp < 2; ++cp) {
              if (rowok && updc && odd == cp && R.ik != T(0)) {
                T off, dg;
                apply<T, EPS>(R, lo, mid, hi, t, off, dg);
                mid[t + 1] = (R.f - off) * R.ik;
              }
              __syncthreads();
            }
          }
        }
        // ------------- residual, output, restriction, norm -------------
        const int R0 = ra - 2 * NU;
        T res[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int r = R0 + q;
          const Rec<T, EPS> &R = rec[ring_slot(2 * ph - 2 * NU + q, NS)];
          const T *mid = L[ring_slot(r, NR)];
          res[q] = T(0);
          if (RESTRICT || NORM) {
            const bool rowok = r >= 1 && r <= ny - 2 && r > ys && r < ye;
            if (rowok && updc && R.ik != T(0)) {
              T off, dg;
              apply<T, EPS>(R, L[ring_slot(r - 1, NR)], mid, L[ring_slot(r + 1, NR)], t, off,
                            dg);
              res[q] = R.f - off - dg * mid[t + 1];
            }
          }
          if (r >= y0 && r < y1 && outc) {
            a.xout[(size_t)r * nx + gi] = mid[t + 1];
            if constexpr (NORM) acc += res[q] * res[q];
          }
        }
        if constexpr (RESTRICT) {
          const T rv = rprev + T(2) * res[0] + res[1];
          rprev = res[1];
          xch[0][t + 1] = rv;
          __syncthreads();
          const int J = k - NU;
          if (2 * J >= y0 && 2 * J < y1 && J < a.nyc && outc && !odd) {
            const int I = gi >> 1;
            const bool ring = I == 0 || J == 0 || I == a.nxc - 1 || J == a.nyc - 1;
            const T v = ring ? T(0)
                             : (xch[0][t] + T(2) * xch[0][t + 1] + xch[0][t + 2]) * T(0.0625);
            a.bc[(size_t)J * a.nxc + I] = v;
          }
        }
        __syncthreads();
        if constexpr (EPS) {
          // the prefetched pair enters the window; shift the carried rows
          commit_row(ra + 2, nxt[0]);
          commit_row(ra + 3, nxt[1]);
          c_yy2 = cur[0].yy;
          c_xy2 = cur[0].xy;
          c_xx1 = cur[1].xx;
          c_xy1 = cur[1].xy;
          c_yy1 = cur[1].yy;
          c_f1 = cur[1].f;
          c_d1 = cur[1].d;
          cur[0] = nxt[0];
          cur[1] = nxt[1];
        }
      }
    }
  }
  if constexpr (NORM) {
    const double s = block_sum<double>((double)acc, red);
    if (t == 0) a.partials[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

static int env_int(const char *name, int dflt) {
  const char *s = getenv(name);
  return (s && *s) ? atoi(s) : dflt;
}

// Rows per block: the tallest band (<= 128 rows) that still gives
// band_target blocks; never below band_min rows (halo rows are recomputed,
// so short bands cost redundant work).  TOMG_BAND_TARGET / TOMG_BAND_MIN
// override the defaults (tuning only).
static int pick_band(int nx, int ny, int W) {
  static const int target = env_int("TOMG_BAND_TARGET", 1024);
  static const int cmin = env_int("TOMG_BAND_MIN", 16);
  const int bx = (nx + W - 1) / W;
  int CH = 128;
  while (CH > cmin && CH > 8 && (long)bx * ((ny + CH - 1) / CH) < target) CH >>= 1;
  return CH;
}

// Upper bound of the block count of any pass on an nx x ny level (sizes the
// partial-sum buffer).
size_t fused_max_blocks(int nx, int ny) {
  const int Wmin = kBW - 2 * (4 * 4 + 2);
  return (size_t)((nx + Wmin - 1) / Wmin) * (size_t)((ny + 7) / 8);
}

template <typename T, bool EPS, int NU, bool ZERO, bool PROLONG, bool RESTRICT, bool NORM>
static void launch_pass_t(PassArgs<T> a, hipStream_t s, int *nblocks) {
  constexpr int H = 4 * NU + 2;
  a.W = kBW - 2 * H;
  a.CH = pick_band(a.nx, a.ny, a.W);
  dim3 grid((a.nx + a.W - 1) / a.W, (a.ny + a.CH - 1) / a.CH);
  if (nblocks) *nblocks = grid.x * grid.y;
  hipLaunchKernelGGL((k_pass<T, EPS, NU, ZERO, PROLONG, RESTRICT, NORM>), grid, dim3(kBW), 0, s,
                     a);
}

// Dispatch on the runtime sweep count (1..4).
template <typename T, bool EPS, bool ZERO, bool PROLONG, bool RESTRICT, bool NORM>
static void launch_pass_nu(int nu, const PassArgs<T> &a, hipStream_t s, int *nb) {
  switch (nu) {
    case 1: launch_pass_t<T, EPS, 1, ZERO, PROLONG, RESTRICT, NORM>(a, s, nb); break;
    case 2: launch_pass_t<T, EPS, 2, ZERO, PROLONG, RESTRICT, NORM>(a, s, nb); break;
    case 3: launch_pass_t<T, EPS, 3, ZERO, PROLONG, RESTRICT, NORM>(a, s, nb); break;
    default: launch_pass_t<T, EPS, 4, ZERO, PROLONG, RESTRICT, NORM>(a, s, nb); break;
  }
}

template <typename T>
static PassArgs<T> base_args(tomg_problem *p, int l, const T *xin, T *xout, const T *b,
                             const T *exx, const T *exy, const T *eyy, const T *st) {
  PassArgs<T> a{};
  a.nx = p->lv[l].nx;
  a.ny = p->lv[l].ny;
  a.xin = xin;
  a.xout = xout;
  a.b = b;
  a.dir = p->lv[l].dir;
  a.exx = exx;
  a.exy = exy;
  a.eyy = eyy;
  a.st = st;
  const double dx = p->cfg.dx, dy = p->cfg.dy;
  a.cx = T(1.0 / (dx * dx));
  a.cy = T(1.0 / (dy * dy));
  a.qx = T(0.25 / (dx * dx));
  a.qy = T(0.25 / (dy * dy));
  a.qxy = T(0.25 / (dx * dy));
  a.hxy = T(0.5 / (dx * dy));
  return a;
}

// Down pass on level l: nu1 sweeps of x (from zero when zero_start) written
// to pong, residual and restriction into bc (level l+1).
template <typename T>
void fused_down(tomg_problem *p, int l, const T *x, T *pong, const T *b, const T *exx,
                const T *exy, const T *eyy, const T *st, T *bc, bool zero_start) {
  PassArgs<T> a = base_args<T>(p, l, x, pong, b, exx, exy, eyy, st);
  a.bc = bc;
  a.nxc = p->lv[l + 1].nx;
  a.nyc = p->lv[l + 1].ny;
  const int nu = p->cfg.nu1;
  if (l == 0) {
    if (zero_start)
      launch_pass_nu<T, true, true, false, true, false>(nu, a, p->stream, nullptr);
    else
      launch_pass_nu<T, true, false, false, true, false>(nu, a, p->stream, nullptr);
  } else {
    if (zero_start)
      launch_pass_nu<T, false, true, false, true, false>(nu, a, p->stream, nullptr);
    else
      launch_pass_nu<T, false, false, false, true, false>(nu, a, p->stream, nullptr);
  }
}

// Up pass on level l: pong plus the prolongation of xc (level l+1), nu2
// sweeps, written to x; with partials, per-block sums of the squared final
// residual (returns the block count).
template <typename T>
int fused_up(tomg_problem *p, int l, const T *pong, T *x, const T *b, const T *exx,
             const T *exy, const T *eyy, const T *st, const T *xc, double *partials) {
  PassArgs<T> a = base_args<T>(p, l, pong, x, b, exx, exy, eyy, st);
  a.xc = xc;
  a.nxc = p->lv[l + 1].nx;
  a.nyc = p->lv[l + 1].ny;
  a.partials = partials;
  const int nu = p->cfg.nu2;
  int nb = 0;
  if (l == 0) {
    if (partials)
      launch_pass_nu<T, true, false, true, false, true>(nu, a, p->stream, &nb);
    else
      launch_pass_nu<T, true, false, true, false, false>(nu, a, p->stream, &nb);
  } else {
    launch_pass_nu<T, false, false, true, false, false>(nu, a, p->stream, &nb);
  }
  return nb;
}

template void fused_down<double>(tomg_problem *, int, const double *, double *, const double *,
                                 const double *, const double *, const double *, const double *,
                                 double *, bool);
template void fused_down<float>(tomg_problem *, int, const float *, float *, const float *,
                                const float *, const float *, const float *, const float *,
                                float *, bool);
template int fused_up<double>(tomg_problem *, int, const double *, double *, const double *,
                              const double *, const double *, const double *, const double *,
                              const double *, double *);
template int fused_up<float>(tomg_problem *, int, const float *, float *, const float *,
                             const float *, const float *, const float *, const float *,
                             const float *, double *);

}  // namespace tomg

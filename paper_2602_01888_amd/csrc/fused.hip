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
// Block geometry: BW threads own BW consecutive columns (one each); the
// H = 4 nu + 2 outer columns on either side are halo, recomputed by the
// neighbouring block, so only W = BW - 2H columns are written.  BW is 128
// (two waves), 64 (one wave) on the stored-stencil levels of a problem
// alone that are small enough to be bound by the chain of colour phases
// rather than by memory traffic, and 256 in the chained pass.  The block
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
#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include "tomg_internal.h"

namespace tomg {
namespace {

#ifndef TOMG_BW
#define TOMG_BW 128
#endif
#ifndef TOMG_MIN_WAVES
#define TOMG_MIN_WAVES 1
#endif
// Block widths.  A colour phase ends in a barrier over the block's waves, so
// narrower blocks shorten each step's chain of phases and give the device
// more blocks, at the cost of more recomputed halo columns (2H of BW).
// Measured per pass at 4097^2, FP64, four-wave -> two-wave blocks: level 0
// down 250 -> 232 us, up 272 -> 261, 2049^2 119 -> 112 and 101 -> 98; FP32
// level 0 138 -> 128 and 130 -> 129.  One-wave blocks on the stored levels
// up to 1025^2 (four-wave -> one-wave): 1025^2 44.7 -> 38.6 us, 513^2 25.9
// -> 21.6, 257^2 19.0 -> 16.2, 129^2 19.2 -> 13.7; on level 0 and at 2049^2
// they are slower (266 and 301 us at level 0).  The chained pass (four
// sweeps, H = 18) keeps four waves: 325 us against 344 with two.  Batched
// launches take two waves too (the 256-problem batch of sides 65 .. 1025:
// FP64 41.6 -> 36.8 ms, mixed 28.2 -> 26.4 ms).
#ifndef TOMG_BW_BATCH
#define TOMG_BW_BATCH 128
#endif
constexpr int kBW = TOMG_BW;
constexpr int kBWSmall = 64;
constexpr int kBWWide = 256;
constexpr int kBWBatch = TOMG_BW_BATCH;
constexpr long kSmallPassNodes = 2L << 20;  // largest level given one-wave blocks

// Streaming stores: the pass outputs are read back by the next pass, long
// after the caches have turned over, so they are written with the
// non-temporal hint.  Loads keep the default policy (halo rows are read
// again by the neighbouring band).
#ifndef TOMG_NT_STORE
#define TOMG_NT_STORE 1
#endif
#ifndef TOMG_NT_LOAD
#define TOMG_NT_LOAD 0
#endif
template <typename T>
__device__ __forceinline__ void st_out(T *p, T v) {
  if constexpr (TOMG_NT_STORE)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}
template <typename T>
__device__ __forceinline__ T ld_in(const T *p) {
  if constexpr (TOMG_NT_LOAD)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

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

template <typename T, int BW>
__device__ __forceinline__ T block_sum(T v, T *red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 1; k < BW / 64; ++k) v += red[k];
  return v;
}

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }

// One level pass.  A step takes P new row pairs: sweep s relaxes the even
// rows of the P pairs m-s, ..., m-s-P+1 (colours 0 then 1; even rows only
// read odd rows, so the P rows of a phase are independent) and then their
// odd rows (colours 2 then 3).  Four barriers per sweep and step, whatever
// P.  The level-0 pass loads the next step's rows while it works on the
// current ones; coarse levels issue a step's loads together at its start.
// CK is the grid transfer to the coarse level: 0 both axes halved (bilinear
// prolongation, full weighting), 1 x halved only, 2 y halved only
// (semi-coarsening: linear along the halved axis, the identity along the
// kept one, restriction (1/4) [1 2 1] along the halved axis).
template <typename T, bool EPS, int NU, int P, bool ZERO, bool PROLONG, bool RESTRICT, bool NORM,
          bool MIR, int CK, int BW>
__device__ __forceinline__ void pass_body(const PassArgs<T> &a, const int bx, const int by) {
  constexpr bool PF = EPS;  // level 0: the next step's rows are loaded during this step
  constexpr int H = 4 * NU + 2;
  constexpr int HV = 2 * NU + 3;
  constexpr int NS = 2 * NU + 2 * P;               // coefficient rows: R0 .. 2m+1
  constexpr int NR = NS + 2;                       // value rows in LDS
  constexpr int PER = NS / cgcd(2 * P, NS);        // steps until the slot ring repeats
  constexpr int NX = (4 * P > P + 1) ? 4 * P : P + 1;
  __shared__ T L[NR][BW + 2];
  __shared__ T xch[NX][BW + 2];
  __shared__ double red[BW / 64];

  const int nx = a.nx, ny = a.ny;
  const int t = threadIdx.x;
  const int x0 = bx * a.W;
  const int gi = x0 - H + t;
  const int gc = min(max(gi, 0), nx - 1);  // clamped column: loads never leave the array
  const bool inr = gi >= 0 && gi < nx;
  // every grid column may hold unknowns (a Neumann edge); Dirichlet nodes
  // are skipped by their zero 1/diagonal
  const bool updc = inr;
  const bool outc = t >= H && t < H + a.W && gi < nx;
  const int odd = gi & 1;
  // MIR: the block marches down its band.  It works in flipped row
  // coordinates (row r is grid row ny-1-r; ny is odd, so every row keeps its
  // parity and colour) and evaluates every sum in the order of the upward
  // march, so each node's arithmetic is the same either way.
  const int ya = by * a.CH, yb = min(ny, ya + a.CH);
  const int y0 = MIR ? ny - yb : ya;
  const int y1 = MIR ? ny - ya : yb;
  const int ys = max(0, y0 - HV) & ~1;
  const int ye = min(ny - 1, y1 - 1 + HV);
  const int m0 = (ys >> 1) + P - 1;  // newest pair of the first step
  const size_t n = (size_t)nx * ny;
  const int Ic = gc >> 1;
  const int Ic1 = (PROLONG && CK != 2) ? min(Ic + 1, a.nxc - 1) : 0;

  for (int r = 0; r < NR; ++r) {
    L[r][t + 1] = T(0);
    if (t < 2) L[r][t * (BW + 1)] = T(0);
  }
  if (t < 2)
    for (int r = 0; r < NX; ++r) xch[r][t * (BW + 1)] = T(0);

  auto slot = [&](int rel) { return ((rel % NS) + NS) % NS; };
  auto lrow = [&](int r) -> T * { return L[((r % NR) + NR) % NR]; };
  auto grow = [&](int r) { return MIR ? ny - 1 - r : r; };  // grid row of row r
  // rows with both neighbours loaded, and the grid's first and last rows
  // (their outer neighbour has a zero coefficient: Neumann, or Dirichlet
  // rows that are never relaxed)
  auto relaxable = [&](int r) {
    return r >= ys && r <= ye && (r > ys || r == 0) && (r < ye || r == ny - 1);
  };
  // the rows below and above row r on the grid
  auto below_row = [&](int r) -> T * { return lrow(MIR ? r + 1 : r - 1); };
  auto above_row = [&](int r) -> T * { return lrow(MIR ? r - 1 : r + 1); };

  // all loads of a row are issued unconditionally from clamped addresses
  auto load_row = [&](int r, Raw<T, EPS> &w) {
    const int rc = grow(min(max(r, 0), ny - 1));
    const size_t c = (size_t)rc * nx + gc;
    w.x = ZERO ? T(0) : ld_in(a.xin + c);
    w.f = ld_in(a.b + c);
    w.d = ld_in(a.dir + c);
    if constexpr (EPS) {
      w.xx = ld_in(a.exx + c);
      w.xy = ld_in(a.exy + c);
      w.yy = ld_in(a.eyy + c);
    } else {
#pragma unroll
      for (int z = 0; z < 9; ++z) w.a[z] = ld_in(a.st + z * n + c);
    }
    if constexpr (PROLONG && CK == 1) {  // x halved: coarse row rc, columns Ic, Ic + 1
      const T *r0 = a.xc + (size_t)rc * a.nxc;
      w.c00 = r0[Ic];
      w.c01 = r0[Ic1];
      w.c10 = w.c11 = T(0);
    } else if constexpr (PROLONG && CK == 2) {  // y halved: rows J, J + 1, column gc
      const int J = rc >> 1, J1 = min(J + 1, a.nyc - 1);
      w.c00 = a.xc[(size_t)J * a.nxc + gc];
      w.c10 = a.xc[(size_t)J1 * a.nxc + gc];
      w.c01 = w.c11 = T(0);
    } else if constexpr (PROLONG) {
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
      if (ld && !w.d && updc) {
        T e;
        if constexpr (CK == 2) {
          e = w.c00;
          if (r & 1) e = T(0.5) * (e + w.c10);
        } else {
          e = odd ? T(0.5) * (w.c00 + w.c01) : w.c00;
          if (CK == 0 && (r & 1)) {
            const T e1 = odd ? T(0.5) * (w.c10 + w.c11) : w.c10;
            e = T(0.5) * (e + e1);
          }
        }
        v += e;
      }
    }
    lrow(r)[t + 1] = v;
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
  Raw<T, EPS> cur[2 * P];
  Raw<T, EPS> nxt[PF ? 2 * P : 1];
  // level 0: tensor values carried from the two rows below the step's first
  // new row: row base-2 (eyy, exy) and row base-1 (exx, exy, eyy, f, dir)
  T c_yy2 = T(0), c_xy2 = T(0), c_xx1 = T(0), c_xy1 = T(0), c_yy1 = T(0), c_f1 = T(0);
  int c_d1 = 1;
  (void)c_yy2; (void)c_xy2; (void)c_xx1; (void)c_xy1; (void)c_yy1; (void)c_f1; (void)c_d1;
  (void)nxt;
  T rprev = T(0), acc = T(0);

  if constexpr (PF) {  // prologue: the rows of the first step
    const int base0 = 2 * (m0 - P + 1);
#pragma unroll
    for (int q = 0; q < 2 * P; ++q) load_row(base0 + q, cur[q]);
#pragma unroll
    for (int q = 0; q < 2 * P; ++q) commit_row(base0 + q, cur[q]);
  }
  __syncthreads();

  for (int sb = 0;; sb += PER) {
    bool more = true;
#pragma unroll
    for (int ph = 0; ph < PER; ++ph) {
      const int m = m0 + P * (sb + ph);
      const int R0 = 2 * (m - NU + 1 - P);  // first row of the residual batch
      if (more && R0 <= y1 - 1) {
        const int base = 2 * (m - P + 1);   // first new row of the step
        // relative row index of row 2m + o is rel0 + o
        const int rel0 = 2 * P * ph + 2 * P - 2;
        if constexpr (PF) {
#pragma unroll
          for (int q = 0; q < 2 * P; ++q) load_row(2 * m + 2 + q, nxt[q]);
        } else {
#pragma unroll
          for (int q = 0; q < 2 * P; ++q) load_row(base + q, cur[q]);
#pragma unroll
          for (int q = 0; q < 2 * P; ++q) commit_row(base + q, cur[q]);
        }
        if constexpr (EPS) {
          // coefficients of rows base-1 .. 2m (row 2m + 1 - 2P + v for v < 2P);
          // raw row u = 0 .. 2P+1 is row base-2+u: u = 0, 1 carried, u >= 2
          // loaded this step (cur[u-2])
          T ryy[2 * P + 2], rxy[2 * P + 2], rxx[2 * P + 2], rff[2 * P + 2];
          int rdd[2 * P + 2];
          ryy[0] = c_yy2;
          rxy[0] = c_xy2;
          rxx[0] = T(0);
          rff[0] = T(0);
          rdd[0] = 1;
          ryy[1] = c_yy1;
          rxy[1] = c_xy1;
          rxx[1] = c_xx1;
          rff[1] = c_f1;
          rdd[1] = c_d1;
#pragma unroll
          for (int q = 0; q < 2 * P; ++q) {
            ryy[q + 2] = cur[q].yy;
            rxy[q + 2] = cur[q].xy;
            rxx[q + 2] = cur[q].xx;
            rff[q + 2] = cur[q].f;
            rdd[q + 2] = cur[q].d;
          }
#pragma unroll
          for (int v = 0; v < 2 * P; ++v) {
            xch[2 * v][t + 1] = rxx[v + 1];
            xch[2 * v + 1][t + 1] = rxy[v + 1];
          }
          __syncthreads();
#pragma unroll
          for (int v = 0; v < 2 * P; ++v) {
            Rec<T, true> &R = rec[slot(rel0 + 1 - 2 * P + v)];
            R.ax = rxx[v + 1] * a.cx;
            R.ay = ryy[v + 1] * a.cy;
            // raw row v + 2 is the grid row above v + 1 (below it when MIR)
            const T dxy = MIR ? rxy[v] - rxy[v + 2] : rxy[v + 2] - rxy[v];
            const T dyy = MIR ? ryy[v] - ryy[v + 2] : ryy[v + 2] - ryy[v];
            R.gx = (xch[2 * v][t + 2] - xch[2 * v][t]) * a.qx + dxy * a.qxy;
            R.gy = dyy * a.qy + (xch[2 * v + 1][t + 2] - xch[2 * v + 1][t]) * a.qxy;
            R.k6 = rxy[v + 1] * a.hxy;
            R.f = rff[v + 1];
            R.ik = rdd[v + 1] ? T(0) : T(-1) / (T(2) * (R.ax + R.ay));
          }
        } else {
#pragma unroll
          for (int q = 0; q < 2 * P; ++q) {
            Rec<T, false> &R = rec[slot(rel0 + 2 - 2 * P + q)];
#pragma unroll
            for (int z = 0; z < 9; ++z) R.a[z] = cur[q].a[z];
            R.f = cur[q].f;
            R.ik = cur[q].d ? T(0) : T(1) / cur[q].a[4];
          }
          __syncthreads();
        }
        // ---------------- sweeps ----------------
#pragma unroll
        for (int s = 0; s < NU; ++s) {
#pragma unroll
          for (int half = 0; half < 2; ++half) {
#pragma unroll
            for (int cp = 0; cp < 2; ++cp) {
#pragma unroll
              for (int p = 0; p < P; ++p) {
                const int o = -2 * s - 2 * p - half;  // row 2m + o
                const int r = 2 * m + o;
                const bool rowok = relaxable(r);
                const Rec<T, EPS> &R = rec[slot(rel0 + o)];
                if (rowok && updc && odd == cp && R.ik != T(0)) {
                  T *mid = lrow(r);
                  T off, dg;
                  apply<T, EPS>(R, below_row(r), mid, above_row(r), t, off, dg);
                  mid[t + 1] = (R.f - off) * R.ik;
                }
              }
              __syncthreads();
            }
          }
        }
        // ------------- residual, output, restriction, norm -------------
        T res[2 * P];
#pragma unroll
        for (int q = 0; q < 2 * P; ++q) {
          const int r = R0 + q;
          const Rec<T, EPS> &R = rec[slot(rel0 + 2 - 2 * NU - 2 * P + q)];
          const T *mid = lrow(r);
          res[q] = T(0);
          if (RESTRICT || NORM) {
            const bool rowok = relaxable(r);
            if (rowok && updc && R.ik != T(0)) {
              T off, dg;
              apply<T, EPS>(R, below_row(r), mid, above_row(r), t, off, dg);
              res[q] = R.f - off - dg * mid[t + 1];
            }
          }
          if (r >= y0 && r < y1 && outc) {
            st_out(a.xout + (size_t)grow(r) * nx + gi, mid[t + 1]);
            if constexpr (NORM) acc += res[q] * res[q];
          }
        }
        if constexpr (RESTRICT && CK == 1) {
          // x halved: each residual row is a coarse row; (1/4) [1 2 1] along it
#pragma unroll
          for (int q = 0; q < 2 * P; ++q) xch[q][t + 1] = res[q];
          __syncthreads();
#pragma unroll
          for (int q = 0; q < 2 * P; ++q) {
            const int r = R0 + q;
            if (r >= y0 && r < y1 && outc && !odd) {
              const int I = gi >> 1, Jg = grow(r);
              const bool ring = I == 0 || Jg == 0 || I == a.nxc - 1 || Jg == a.nyc - 1;
              const bool fixed = ring && (!a.dirc || a.dirc[(size_t)Jg * a.nxc + I]);
              const T v = fixed ? T(0)
                               : (xch[q][t] + T(2) * xch[q][t + 1] + xch[q][t + 2]) * T(0.25);
              st_out(a.bc + (size_t)Jg * a.nxc + I, v);
            }
          }
        } else if constexpr (RESTRICT && CK == 2) {
          // y halved: (1/4) [1 2 1] across rows 2J-1, 2J, 2J+1 at every column
          T below[2 * P + 1];
          below[0] = rprev;
#pragma unroll
          for (int q = 0; q < 2 * P; ++q) below[q + 1] = res[q];
          rprev = res[2 * P - 1];
#pragma unroll
          for (int p = 0; p < P; ++p) {
            const int J = (R0 >> 1) + p;
            if (2 * J >= y0 && 2 * J < y1 && J < a.nyc && outc) {
              const int I = gi, Jg = MIR ? a.nyc - 1 - J : J;
              const bool ring = I == 0 || Jg == 0 || I == a.nxc - 1 || Jg == a.nyc - 1;
              const bool fixed = ring && (!a.dirc || a.dirc[(size_t)Jg * a.nxc + I]);
              const T sum = MIR ? res[2 * p + 1] + T(2) * res[2 * p] + below[2 * p]
                                : below[2 * p] + T(2) * res[2 * p] + res[2 * p + 1];
              st_out(a.bc + (size_t)Jg * a.nxc + I, fixed ? T(0) : sum * T(0.25));
            }
          }
        } else if constexpr (RESTRICT) {
          T below[2 * P + 1];
          below[0] = rprev;
#pragma unroll
          for (int q = 0; q < 2 * P; ++q) below[q + 1] = res[q];
#pragma unroll
          for (int p = 0; p < P; ++p)  // grid rows 2J-1, 2J, 2J+1 in that order
            xch[p][t + 1] = MIR ? res[2 * p + 1] + T(2) * res[2 * p] + below[2 * p]
                                : below[2 * p] + T(2) * res[2 * p] + res[2 * p + 1];
          rprev = res[2 * P - 1];
          __syncthreads();
#pragma unroll
          for (int p = 0; p < P; ++p) {
            const int J = (R0 >> 1) + p;
            if (2 * J >= y0 && 2 * J < y1 && J < a.nyc && outc && !odd) {
              const int I = gi >> 1, Jg = MIR ? a.nyc - 1 - J : J;
              const bool ring = I == 0 || Jg == 0 || I == a.nxc - 1 || Jg == a.nyc - 1;
              // a coarse ring node is Dirichlet unless its edge is Neumann
              const bool fixed = ring && (!a.dirc || a.dirc[(size_t)Jg * a.nxc + I]);
              const T v = fixed ? T(0)
                               : (xch[p][t] + T(2) * xch[p][t + 1] + xch[p][t + 2]) * T(0.0625);
              st_out(a.bc + (size_t)Jg * a.nxc + I, v);
            }
          }
        }
        __syncthreads();
        if constexpr (EPS) {
          // rows 2m and 2m+1 become the carried rows of the next step
          c_yy2 = cur[2 * P - 2].yy;
          c_xy2 = cur[2 * P - 2].xy;
          c_xx1 = cur[2 * P - 1].xx;
          c_xy1 = cur[2 * P - 1].xy;
          c_yy1 = cur[2 * P - 1].yy;
          c_f1 = cur[2 * P - 1].f;
          c_d1 = cur[2 * P - 1].d;
        }
        if constexpr (PF) {
#pragma unroll
          for (int q = 0; q < 2 * P; ++q) {
            commit_row(2 * m + 2 + q, nxt[q]);
            cur[q] = nxt[q];
          }
        }
      } else {
        more = false;
      }
    }
    if (!more) break;
  }
  if constexpr (NORM) {
    const double s = block_sum<double, BW>((double)acc, red);
    if (t == 0) a.partials[(size_t)by * a.nbx + bx] = s;
  }
}

// Odd bands march down (TOMG_MIRROR): then two neighbouring bands reach
// their common boundary at the same time -- at the start of the pass for one
// pair, at its end for the other -- and the halo rows both read are served
// by the cache instead of being fetched from memory twice.  FP64 passes
// only: the FP32 passes move half the bytes and gain nothing from it.
#ifndef TOMG_MIRROR
#define TOMG_MIRROR 1
#endif
template <typename T>
__device__ __forceinline__ bool mirrored(int by, int ny) {
  return TOMG_MIRROR && std::is_same<T, double>::value && (by & 1) && (ny & 1);
}

// Tile of a block of a one-dimensional launch.  Workgroups go to the eight
// XCDs in turn (XCD = linear id mod 8); each XCD is given one contiguous run
// of tiles in strip-fastest order, so the neighbouring strips of a band --
// which read each other's halo columns at about the same time -- share that
// XCD's L2 instead of fetching the halo twice from memory.
__device__ __forceinline__ void xcd_tile(int id, int nbx, int nby, int &bx, int &by) {
  const int n = nbx * nby, per = n >> 3, rem = n & 7;
  const int xcd = id & 7, q = id >> 3;
  const int tile = xcd * per + min(xcd, rem) + q;
  bx = tile % nbx;
  by = tile / nbx;
}

template <typename T, bool EPS, int NU, int P, bool ZERO, bool PROLONG, bool RESTRICT, bool NORM,
          int CK = 0, int BW = kBW>
__global__ __launch_bounds__(BW, TOMG_MIN_WAVES) void k_pass(PassArgs<T> a) {
  if (a.skip && *a.skip != 0.0) return;
  int bx = blockIdx.x, by = blockIdx.y;
  if (a.xcd_order) xcd_tile(blockIdx.x, a.nbx, a.nby, bx, by);
  if (mirrored<T>(by, a.ny))
    pass_body<T, EPS, NU, P, ZERO, PROLONG, RESTRICT, NORM, true, CK, BW>(a, bx, by);
  else
    pass_body<T, EPS, NU, P, ZERO, PROLONG, RESTRICT, NORM, false, CK, BW>(a, bx, by);
}

// Entry of a batched launch holding block b (entries sorted by start).
__device__ __forceinline__ const BatchEntry &batch_locate(const BatchTab &tab, int b) {
  int lo = 0, hi = tab.count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab.e[mid].start <= b) lo = mid; else hi = mid - 1;
  }
  return tab.e[lo];
}

// Batched form: each problem runs exactly the blocks it would run alone
// (one transfer kind per launch: the problems of a batch share their
// semi-coarsened levels).
template <typename T, bool EPS, int NU, int P, bool ZERO, bool PROLONG, bool RESTRICT, bool NORM,
          int CK = 0>
__global__ __launch_bounds__(kBWBatch, TOMG_MIN_WAVES) void k_pass_b(BatchTab tab) {
  const BatchEntry &e = batch_locate(tab, blockIdx.x);
  PassArgs<T> a = *static_cast<const PassArgs<T> *>(e.args);
  if (e.role == 1) a.xin = static_cast<const T *>(e.phi);
  if (e.role == 2) a.xout = static_cast<T *>(e.phi);
  const int local = blockIdx.x - e.start, bx = local % e.nbx, by = local / e.nbx;
  if (mirrored<T>(by, a.ny))
    pass_body<T, EPS, NU, P, ZERO, PROLONG, RESTRICT, NORM, true, CK, kBWBatch>(a, bx, by);
  else
    pass_body<T, EPS, NU, P, ZERO, PROLONG, RESTRICT, NORM, false, CK, kBWBatch>(a, bx, by);
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// Rows per block.  A pass is a set of blocks that each march up their band
// two rows per step, so its time is about (steps per block) x (rounds of
// blocks the device needs); halo rows are recomputed by both neighbours.
// The band is the shortest (fewest steps) that still lets all blocks of the
// pass be resident at once (slots = resident blocks per CU x CUs), and on
// levels above 2M nodes, where the pass is bound by memory traffic, at least
// three halo depths tall so that halo rows add at most two thirds to it.
//
// In a batch the other problems fill the device, so a problem's passes use
// taller bands than alone (less halo work), growing with the level's size:
// 16 rows below 257 rows, 24 from 257, 32 from 513, 40 from 1025.  Measured
// on the 256-problem batch (sides 65-1025, mixed precision): 30.5 ms with 16
// rows everywhere, 29.1 with 32, 31.8 with 64, 40.8 with 128, 28.2 with this
// table; on the serving stream (sides 129-2049) it raised the closed-loop
// capacity by 6 %.
constexpr int kMinBand = 2;
static int pick_band_batch(int nx, int ny, int W) {
  (void)nx;
  (void)W;
  const int c = ny >= 1025 ? 40 : (ny >= 513 ? 32 : (ny >= 257 ? 24 : 16));
  return c < ny ? c : ny;
}

static int pick_band(int nx, int ny, int W, long slots, int hv) {
  const long bx = (nx + W - 1) / W;
  int CH = (long)nx * ny > (2L << 20) ? 3 * hv + (3 * hv & 1) : kMinBand;
  while (CH < ny && bx * ((ny + CH - 1) / CH) > slots) CH += 2;
  return CH < ny ? CH : ny;
}

// Upper bound of the block count of any pass on an nx x ny level (sizes the
// partial-sum buffer).
size_t fused_max_blocks(int nx, int ny) {
  const int bw = (long)nx * ny <= kSmallPassNodes ? kBWSmall : (kBW < kBWBatch ? kBW : kBWBatch);
  const int Wmin = bw - 2 * (4 * 4 + 2);
  return (size_t)((nx + Wmin - 1) / Wmin) * (size_t)((ny + kMinBand - 1) / kMinBand);
}

#ifndef TOMG_PAIRS_EPS
#define TOMG_PAIRS_EPS 1
#endif
#ifndef TOMG_PAIRS_ST
#define TOMG_PAIRS_ST 1
#endif

// A one-wave-block pass (stored stencils only: no such variant of the
// level-0 pass that forms its coefficients from the tensor is built).
template <typename T, bool EPS, int NU, int P, bool ZERO, bool PROLONG, bool RESTRICT, bool NORM>
static void launch_small(const PassArgs<T> &a, dim3 grid, hipStream_t s) {
  if constexpr (!EPS)
    hipLaunchKernelGGL((k_pass<T, false, NU, P, ZERO, PROLONG, RESTRICT, NORM, 0, kBWSmall>), grid,
                       dim3(kBWSmall), 0, s, a);
}

// Sweep count, pair count and transfer kind are compile-time; dispatch on
// the runtime nu and a.ck (for a batched launch, that of its first problem:
// every problem of a batch has the same transfer at a given level).
template <typename T, bool EPS, bool ZERO, bool PROLONG, bool RESTRICT, bool NORM>
static void launch_pass(int nu, const PassArgs<T> &a, hipStream_t s, const BatchTab *tab,
                        int nblocks) {
  constexpr int P = EPS ? TOMG_PAIRS_EPS : TOMG_PAIRS_ST;
  const dim3 grid = a.xcd_order ? dim3(a.nbx * a.nby) : dim3(a.nbx, a.nby);
  // one-wave blocks: stored stencils, both axes halved, alone (make_args)
  const bool small = !EPS && !tab && a.bw == kBWSmall;
#define TOMG_LAUNCH(NU)                                                                          \
  do {                                                                                           \
    if (tab && a.ck == 1)                                                                        \
      hipLaunchKernelGGL((k_pass_b<T, EPS, NU, P, ZERO, PROLONG, RESTRICT, NORM, 1>),           \
                         dim3(nblocks), dim3(kBWBatch), 0, s, *tab);                                  \
    else if (tab && a.ck == 2)                                                                   \
      hipLaunchKernelGGL((k_pass_b<T, EPS, NU, P, ZERO, PROLONG, RESTRICT, NORM, 2>),           \
                         dim3(nblocks), dim3(kBWBatch), 0, s, *tab);                                  \
    else if (tab)                                                                                \
      hipLaunchKernelGGL((k_pass_b<T, EPS, NU, P, ZERO, PROLONG, RESTRICT, NORM>),              \
                         dim3(nblocks), dim3(kBWBatch), 0, s, *tab);                                  \
    else if (small)                                                                              \
      launch_small<T, EPS, NU, P, ZERO, PROLONG, RESTRICT, NORM>(a, grid, s);                   \
    else if (a.ck == 1)                                                                          \
      hipLaunchKernelGGL((k_pass<T, EPS, NU, P, ZERO, PROLONG, RESTRICT, NORM, 1>), grid,       \
                         dim3(kBW), 0, s, a);                                                    \
    else if (a.ck == 2)                                                                          \
      hipLaunchKernelGGL((k_pass<T, EPS, NU, P, ZERO, PROLONG, RESTRICT, NORM, 2>), grid,       \
                         dim3(kBW), 0, s, a);                                                    \
    else                                                                                         \
      hipLaunchKernelGGL((k_pass<T, EPS, NU, P, ZERO, PROLONG, RESTRICT, NORM>), grid,          \
                         dim3(kBW), 0, s, a);                                                    \
  } while (0)
  switch (nu) {
    case 1: TOMG_LAUNCH(1); break;
    case 2: TOMG_LAUNCH(2); break;
    case 3: TOMG_LAUNCH(3); break;
    default: TOMG_LAUNCH(4); break;
  }
#undef TOMG_LAUNCH
}

static int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  return cus;
}

// Blocks of one pass kernel that fit on a CU at once.
template <typename T, bool EPS, bool ZERO, bool PROLONG, bool RESTRICT, bool NORM, int BW = kBW>
static int pass_blocks_per_cu(int nu) {
  constexpr int P = EPS ? TOMG_PAIRS_EPS : TOMG_PAIRS_ST;
  const void *f;
  switch (nu) {
    case 1: f = reinterpret_cast<const void *>(k_pass<T, EPS, 1, P, ZERO, PROLONG, RESTRICT, NORM, 0, BW>); break;
    case 2: f = reinterpret_cast<const void *>(k_pass<T, EPS, 2, P, ZERO, PROLONG, RESTRICT, NORM, 0, BW>); break;
    case 3: f = reinterpret_cast<const void *>(k_pass<T, EPS, 3, P, ZERO, PROLONG, RESTRICT, NORM, 0, BW>); break;
    default: f = reinterpret_cast<const void *>(k_pass<T, EPS, 4, P, ZERO, PROLONG, RESTRICT, NORM, 0, BW>); break;
  }
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, BW, 0) != hipSuccess || nb < 1) nb = 1;
  return nb;
}

// Resident-block slots of the pass of level l (the variant a solve launches;
// eps0: level 0 forms its coefficients from the tensor; small: one-wave
// blocks on a stored stencil).
template <typename T>
static long pass_slots(int l, bool up, int nu, bool eps0, bool small) {
  constexpr bool F64 = std::is_same<T, double>::value;
  int nb;
  if (small) {
    nb = up ? (l == 0 ? pass_blocks_per_cu<T, false, false, true, false, F64, kBWSmall>(nu)
                      : pass_blocks_per_cu<T, false, false, true, false, false, kBWSmall>(nu))
            : (l == 0 ? pass_blocks_per_cu<T, false, false, false, true, false, kBWSmall>(nu)
                      : pass_blocks_per_cu<T, false, true, false, true, false, kBWSmall>(nu));
  } else if (l == 0 && !eps0) {
    nb = up ? pass_blocks_per_cu<T, false, false, true, false, F64>(nu)
            : pass_blocks_per_cu<T, false, false, false, true, false>(nu);
  } else if (l == 0) {
    if (up)
      nb = F64 ? pass_blocks_per_cu<T, true, false, true, false, F64>(nu)
               : pass_blocks_per_cu<T, true, false, true, false, false>(nu);
    else
      nb = pass_blocks_per_cu<T, true, false, false, true, false>(nu);
  } else {
    nb = up ? pass_blocks_per_cu<T, false, false, true, false, false>(nu)
            : pass_blocks_per_cu<T, false, true, false, true, false>(nu);
  }
  static const int cus = device_cus();
  return (long)nb * cus;
}

// The chained level-0 pass of the FP32 inner cycles (the up pass of a cycle
// and the down pass of the next): nu2 + nu1 in 2 .. 4 sweeps, prolongation
// on load and restriction of the final residual in the same launch.
template <typename T, bool EPS>
static int updown_blocks_per_cu(int nu) {
  constexpr int P = EPS ? TOMG_PAIRS_EPS : TOMG_PAIRS_ST;
  const void *f;
  switch (nu) {
    case 2: f = reinterpret_cast<const void *>(k_pass<T, EPS, 2, P, false, true, true, false, 0, kBWWide>); break;
    case 3: f = reinterpret_cast<const void *>(k_pass<T, EPS, 3, P, false, true, true, false, 0, kBWWide>); break;
    default: f = reinterpret_cast<const void *>(k_pass<T, EPS, 4, P, false, true, true, false, 0, kBWWide>); break;
  }
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kBWWide, 0) != hipSuccess || nb < 1) nb = 1;
  return nb;
}

template <typename T, bool EPS, int CK>
static void launch_updown_ck(int nu, const PassArgs<T> &a, hipStream_t s) {
  constexpr int P = EPS ? TOMG_PAIRS_EPS : TOMG_PAIRS_ST;
  const dim3 grid = a.xcd_order ? dim3(a.nbx * a.nby) : dim3(a.nbx, a.nby);
  switch (nu) {
    case 2:
      hipLaunchKernelGGL((k_pass<T, EPS, 2, P, false, true, true, false, CK, kBWWide>), grid,
                         dim3(kBWWide), 0, s, a);
      break;
    case 3:
      hipLaunchKernelGGL((k_pass<T, EPS, 3, P, false, true, true, false, CK, kBWWide>), grid,
                         dim3(kBWWide), 0, s, a);
      break;
    default:
      hipLaunchKernelGGL((k_pass<T, EPS, 4, P, false, true, true, false, CK, kBWWide>), grid,
                         dim3(kBWWide), 0, s, a);
      break;
  }
}

template <typename T, bool EPS>
static void launch_updown(int nu, const PassArgs<T> &a, hipStream_t s) {
  if (a.ck == 1)
    launch_updown_ck<T, EPS, 1>(nu, a, s);
  else if (a.ck == 2)
    launch_updown_ck<T, EPS, 2>(nu, a, s);
  else
    launch_updown_ck<T, EPS, 0>(nu, a, s);
}

// Chained only with a stored level-0 stencil (Neumann edges, the flux form):
// there the pass moves 49 B per node for its own 4-byte iterate and a
// chained pass saves half of them (Neumann semi-annulus at 4097^2, four
// inner cycles per step: 18.7 -> 17.2 ms).  With the coefficients formed
// from the tensor the level-0 pass is bound by its steps' phase chain, not
// by its bytes, and the chained pass's sixteen colour phases per step made
// it slower than the two passes it replaces (295 against 135 + 134 us).
bool chain_inner(const tomg_problem *p) {
  return p->cfg.precision == TOMG_FP32_IR && p->cfg.smoother == TOMG_GS4 && p->L >= 2 &&
         p->cfg.nu1 + p->cfg.nu2 <= 4 && stored_level0(p->cfg);
}

// Arguments of the down (up) pass of level l in precision T: the level
// iterate x_l is read (written) and its second buffer written (read).
template <typename T>
static PassArgs<T> make_args(tomg_problem *p, int l, bool up, bool batch, T *x0, T *pong0,
                             const T *b0, const T *exx, const T *exy, const T *eyy) {
  PassArgs<T> a{};
  const Level &v = p->lv[l];
  const bool f32 = std::is_same<T, float>::value;
  a.nx = v.nx;
  a.ny = v.ny;
  T *x = l == 0 ? x0 : (T *)(f32 ? (void *)v.x32 : (void *)v.x);
  T *pong = l == 0 ? pong0 : (T *)(f32 ? (void *)v.x2_32 : (void *)v.x2);
  a.xin = up ? pong : x;
  a.xout = up ? x : pong;
  a.b = l == 0 ? b0 : (const T *)(f32 ? (void *)v.b32 : (void *)v.b);
  a.dir = v.dir;
  a.exx = exx;
  a.exy = exy;
  a.eyy = eyy;
  const bool stored = stored_level0(p->cfg);  // level 0 stencil stored
  a.st = (l > 0 || stored) ? (const T *)(f32 ? (void *)v.st32 : (void *)v.st) : nullptr;
  const double dx = p->cfg.dx, dy = p->cfg.dy;
  a.cx = T(1.0 / (dx * dx));
  a.cy = T(1.0 / (dy * dy));
  a.qx = T(0.25 / (dx * dx));
  a.qy = T(0.25 / (dy * dy));
  a.qxy = T(0.25 / (dx * dy));
  a.hxy = T(0.5 / (dx * dy));
  const Level &c = p->lv[l + 1];
  a.nxc = c.nx;
  a.nyc = c.ny;
  a.xc = up ? (const T *)(f32 ? (void *)c.x32 : (void *)c.x) : nullptr;
  a.bc = up ? nullptr : (T *)(f32 ? (void *)c.b32 : (void *)c.b);
  a.dirc = stored ? c.dir : nullptr;
  a.partials = (up && l == 0) ? p->partials : nullptr;
  const int nu = up ? p->cfg.nu2 : p->cfg.nu1;
  const bool small = !batch && (l > 0 || stored) && v.ck == 0 &&
                     (long)a.nx * a.ny <= kSmallPassNodes;
  a.bw = batch ? kBWBatch : (small ? kBWSmall : kBW);
  a.W = a.bw - 2 * (4 * nu + 2);
  a.CH = batch ? pick_band_batch(a.nx, a.ny, a.W)
              : pick_band(a.nx, a.ny, a.W, pass_slots<T>(l, up, nu, !stored, small), 2 * nu + 3);
  a.nbx = (a.nx + a.W - 1) / a.W;
  a.nby = (a.ny + a.CH - 1) / a.CH;
  a.xcd_order = (!batch && a.nbx > 1) ? 1 : 0;
  a.ck = v.ck;
  return a;
}

// Pass arguments of every level, both directions (and FP32 copies for
// refinement problems).  The level-0 FP64 iterate is the caller's phi, set
// per launch (nullptr here).
void build_pass_args(tomg_problem *p) {
  ArgsBlob &g = p->hargs;
  for (int l = 0; l + 1 < p->L; ++l)
    for (int batch = 0; batch < 2; ++batch) {
      PassArgs<double> *d64 = batch ? g.down64b : g.down64, *u64 = batch ? g.up64b : g.up64;
      PassArgs<float> *d32 = batch ? g.down32b : g.down32, *u32 = batch ? g.up32b : g.up32;
      d64[l] = make_args<double>(p, l, false, batch, nullptr, p->tmp, p->f, p->exx, p->exy,
                                 p->eyy);
      u64[l] = make_args<double>(p, l, true, batch, nullptr, p->tmp, p->f, p->exx, p->exy,
                                 p->eyy);
      if (p->cfg.precision == TOMG_FP32_IR) {
        d32[l] = make_args<float>(p, l, false, batch, p->e32, p->e32b, p->r32, p->exx32,
                                  p->exy32, p->eyy32);
        u32[l] = make_args<float>(p, l, true, batch, p->e32, p->e32b, p->r32, p->exx32,
                                  p->exy32, p->eyy32);
      }
    }
  if (chain_inner(p)) {
    // the up pass's arguments (prolongation from level 1), with the
    // restriction into level 1's right-hand side and the blocking of
    // nu2 + nu1 sweeps
    PassArgs<float> a = make_args<float>(p, 0, true, false, p->e32, p->e32b, p->r32, p->exx32,
                                         p->exy32, p->eyy32);
    const int nu = p->cfg.nu1 + p->cfg.nu2;
    a.bc = p->lv[1].b32;
    a.partials = nullptr;
    a.bw = kBWWide;
    a.W = kBWWide - 2 * (4 * nu + 2);
    static const int cus = device_cus();
    const long slots = (long)updown_blocks_per_cu<float, false>(nu) * cus;
    a.CH = pick_band(a.nx, a.ny, a.W, slots, 2 * nu + 3);
    a.nbx = (a.nx + a.W - 1) / a.W;
    a.nby = (a.ny + a.CH - 1) / a.CH;
    a.xcd_order = a.nbx > 1 ? 1 : 0;
    g.updown32 = a;
  }
}

template <typename T>
static void launch_down(int nu, bool eps, bool zero, const PassArgs<T> &a, hipStream_t s,
                        const BatchTab *tab, int nb) {
  if (eps) {
    if (zero) launch_pass<T, true, true, false, true, false>(nu, a, s, tab, nb);
    else launch_pass<T, true, false, false, true, false>(nu, a, s, tab, nb);
  } else {
    if (zero) launch_pass<T, false, true, false, true, false>(nu, a, s, tab, nb);
    else launch_pass<T, false, false, false, true, false>(nu, a, s, tab, nb);
  }
}

template <typename T>
static void launch_up(int nu, bool eps, bool norm, const PassArgs<T> &a, hipStream_t s,
                      const BatchTab *tab, int nb) {
  if (eps) {
    if (norm) launch_pass<T, true, false, true, false, true>(nu, a, s, tab, nb);
    else launch_pass<T, true, false, true, false, false>(nu, a, s, tab, nb);
  } else {
    if (norm) launch_pass<T, false, false, true, false, true>(nu, a, s, tab, nb);
    else launch_pass<T, false, false, true, false, false>(nu, a, s, tab, nb);
  }
}

// Down pass on level l: nu1 sweeps of x (from zero when zero_start) written
// to pong, residual and restriction into the level l+1 right-hand side.
template <typename T>
void fused_down(tomg_problem *p, int l, const T *x, T *pong, const T *b, const T *exx,
                const T *exy, const T *eyy, const T *st, T *bc, bool zero_start) {
  PassArgs<T> a = std::is_same<T, float>::value ? *(PassArgs<T> *)(void *)&p->hargs.down32[l]
                                                : *(PassArgs<T> *)(void *)&p->hargs.down64[l];
  a.xin = x;
  a.xout = pong;
  a.b = b;
  a.exx = exx;
  a.exy = exy;
  a.eyy = eyy;
  a.st = st;
  a.bc = bc;
  a.skip = p->skip;
  launch_down<T>(p->cfg.nu1, l == 0 && !stored_level0(p->cfg), zero_start, a, p->stream,
                 nullptr, 0);
}

// Up pass on level l: pong plus the prolongation of xc (level l+1), nu2
// sweeps, written to x; with partials, per-block sums of the squared final
// residual (returns the block count).
template <typename T>
int fused_up(tomg_problem *p, int l, const T *pong, T *x, const T *b, const T *exx,
             const T *exy, const T *eyy, const T *st, const T *xc, double *partials) {
  PassArgs<T> a = std::is_same<T, float>::value ? *(PassArgs<T> *)(void *)&p->hargs.up32[l]
                                                : *(PassArgs<T> *)(void *)&p->hargs.up64[l];
  a.xin = pong;
  a.xout = x;
  a.b = b;
  a.exx = exx;
  a.exy = exy;
  a.eyy = eyy;
  a.st = st;
  a.xc = xc;
  a.partials = partials;
  a.skip = p->skip;
  launch_up<T>(p->cfg.nu2, l == 0 && !stored_level0(p->cfg), partials != nullptr, a, p->stream,
               nullptr, 0);
  return a.nbx * a.nby;
}

template <typename T>
void fused_updown(tomg_problem *p, const T *pong, T *out, const T *b, const T *exx,
                  const T *exy, const T *eyy, const T *st, const T *xc, T *bc) {
  static_assert(std::is_same<T, float>::value, "chained passes run the FP32 inner cycles");
  PassArgs<T> a = p->hargs.updown32;
  a.xin = pong;
  a.xout = out;
  a.b = b;
  a.exx = exx;
  a.exy = exy;
  a.eyy = eyy;
  a.st = st;
  a.xc = xc;
  a.bc = bc;
  a.partials = nullptr;
  a.skip = p->skip;
  launch_updown<T, false>(p->cfg.nu1 + p->cfg.nu2, a, p->stream);  // stored level 0 only
}
template void fused_updown<float>(tomg_problem *, const float *, float *, const float *,
                                  const float *, const float *, const float *, const float *,
                                  const float *, float *);

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

// ---------------------------------------------------------------------------
// Batched passes: one launch covers level l of up to kBatchMax problems.
// ---------------------------------------------------------------------------

template <typename T>
static void batch_pass(tomg_problem *const *probs, const int *idx, int cnt, int l, bool up,
                       bool flag, double *const *phis, hipStream_t s) {
  const bool f32 = std::is_same<T, float>::value;
  BatchTab tab;
  for (int k0 = 0; k0 < cnt; k0 += kBatchMax) {
    tab.count = 0;
    int nb = 0;
    const PassArgs<T> *first = nullptr;
    for (int k = k0; k < cnt && k < k0 + kBatchMax; ++k) {
      tomg_problem *p = probs[idx[k]];
      const PassArgs<T> *h = f32 ? (const PassArgs<T> *)(void *)(up ? &p->hargs.up32b[l]
                                                                      : &p->hargs.down32b[l])
                                 : (const PassArgs<T> *)(void *)(up ? &p->hargs.up64b[l]
                                                                      : &p->hargs.down64b[l]);
      const PassArgs<T> *d = f32 ? (const PassArgs<T> *)(void *)(up ? &p->dargs->up32b[l]
                                                                      : &p->dargs->down32b[l])
                                 : (const PassArgs<T> *)(void *)(up ? &p->dargs->up64b[l]
                                                                      : &p->dargs->down64b[l]);
      if (!first) first = h;
      BatchEntry &e = tab.e[tab.count++];
      e.args = d;
      e.phi = (!f32 && l == 0) ? (void *)phis[idx[k]] : nullptr;
      e.role = (!f32 && l == 0) ? (up ? 2 : 1) : 0;
      e.nbx = h->nbx;
      e.nby = h->nby;
      e.start = nb;
      e.slot = e.out = 0;
      nb += h->nbx * h->nby;
    }
    if (!tab.count) continue;
    const tomg_problem *p0 = probs[idx[k0]];
    const int nu = up ? p0->cfg.nu2 : p0->cfg.nu1;
    // a batch has one level-0 operator form (on-the-fly or stored) for all
    const bool eps = l == 0 && !stored_level0(p0->cfg);
    if (up)
      launch_up<T>(nu, eps, flag, *first, s, &tab, nb);
    else
      launch_down<T>(nu, eps, flag, *first, s, &tab, nb);
  }
}

void batch_down(tomg_problem *const *probs, const int *idx, int cnt, int l, bool fp32, bool zero0,
                double *const *phis, hipStream_t s) {
  const bool zero = l > 0 || zero0;
  if (fp32)
    batch_pass<float>(probs, idx, cnt, l, false, zero, phis, s);
  else
    batch_pass<double>(probs, idx, cnt, l, false, zero, phis, s);
}

void batch_up(tomg_problem *const *probs, const int *idx, int cnt, int l, bool fp32, bool norm,
              double *const *phis, hipStream_t s) {
  if (fp32)
    batch_pass<float>(probs, idx, cnt, l, true, norm && l == 0, phis, s);
  else
    batch_pass<double>(probs, idx, cnt, l, true, norm && l == 0, phis, s);
}

}  // namespace tomg

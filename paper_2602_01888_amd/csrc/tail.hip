// The smallest levels of the V-cycle in one workgroup (arXiv 2602.01888,
// Section 3).
//
// Below a few thousand nodes per level, a level pass is bound by latency: a
// launch per pass, or a band-marching pass with a barrier per colour phase
// and row pair, costs far more than its work.  One 1024-thread workgroup
// runs the sub-cycle from level lc (zero start, right-hand side from the
// level above) down to the coarsest level and back, with the iterates of
// all tail levels and one residual array in LDS, so a colour phase is an
// LDS read-modify-write between two barriers.
//
// Levels are counted from the coarsest (r = 0).  The two coarsest (at most
// 17 x 17 nodes) give each thread one node whose stencil row and right-hand
// side stay in registers.  Levels r >= 2 (at most 65 x 65 nodes, five nodes
// per thread) stream their stencil rows from global memory, where they stay
// in the L2 cache; in each colour phase a thread already loads the stencil
// of its node of the next phase, so the load latency overlaps the barrier.
// Their right-hand side is the global array for the first tail level and an
// LDS array below it.  Arithmetic per node is that of the other kernels:
// four-colour Gauss-Seidel on the stored 9-point stencil, full weighting,
// bilinear prolongation, explicit coarsest inverse.
#include <type_traits>

#include "tomg_internal.h"

namespace tomg {
namespace {

constexpr int kTailThreads = 1024;
constexpr int kTailMaxNodes = 65 * 65;  // per level: at most five nodes per thread
// LDS per workgroup, less the static arrays (the coarsest right-hand side)
constexpr int kTailLdsMax = 160 * 1024 - 9 * 1024;

template <typename T>
struct Own {
  T a[9];
  T b, ik;  // ik = 1 / diagonal, 0 where the node is not relaxed
  int c;    // node index in the level, -1 when not owned
  int col;  // colour (i mod 2) + 2 (j mod 2)
};

// Interior node k of colour col (i = pi + 2u, j = pj + 2w), or -1.
__device__ __forceinline__ int colour_node(int nx, int ny, int col, int k) {
  const int i0 = (col & 1) ? 1 : 2, j0 = (col >> 1) ? 1 : 2;
  const int cu = nx - 2 >= i0 ? (nx - 2 - i0) / 2 + 1 : 0;
  const int cw = ny - 2 >= j0 ? (ny - 2 - j0) / 2 + 1 : 0;
  if (k >= cu * cw) return -1;
  return (j0 + 2 * (k / cu)) * nx + i0 + 2 * (k % cu);
}

template <typename T>
__device__ __forceinline__ void tail_body(const TailArgs<T> &a) {
  extern __shared__ unsigned char smem_raw[];
  T *X = reinterpret_cast<T *>(smem_raw);
  __shared__ double bb[kMaxCoarseNodes];
  const int t = threadIdx.x;
  const int nl = a.nl;
  int total = 0, rmax = 0;
  for (int q = 0; q < nl; ++q) {
    const int n = a.lv[q].nx * a.lv[q].ny;
    total += n;
    if (q < nl - 1) rmax = max(rmax, n);
  }
  T *Rb = X + total;  // residual of the level being restricted
  T *Bs = Rb + rmax;  // right-hand sides of streamed levels below the first
  auto lvl = [&](int r) -> const TailLevel<T> & { return a.lv[nl - 1 - r]; };

  for (int q = 0; q < nl; ++q) {
    const TailLevel<T> &v = a.lv[q];
    for (int c = t; c < v.nx * v.ny; c += kTailThreads) X[v.off + c] = T(0);
  }
  Own<T> own[2];  // levels r = 0 (coarsest) and r = 1
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    Own<T> &o = own[r];
    o.c = -1;
    o.b = o.ik = T(0);
    o.col = 0;
#pragma unroll
    for (int z = 0; z < 9; ++z) o.a[z] = T(0);
    if (r >= nl) continue;
    const TailLevel<T> &v = lvl(r);
    const int n = v.nx * v.ny;
    if (t >= n) continue;
    const int i = t % v.nx, j = t / v.nx;
    o.c = t;
    o.col = (i & 1) + 2 * (j & 1);
    const bool interior = i > 0 && j > 0 && i < v.nx - 1 && j < v.ny - 1;
    if (r > 0 && interior && !v.dir[t]) {
#pragma unroll
      for (int z = 0; z < 9; ++z) o.a[z] = v.st[(size_t)z * n + t];
      o.ik = T(1) / o.a[4];
    }
    if (r == nl - 1) o.b = v.b[t];
  }
  __syncthreads();

  // off-centre part of A x at node c of level v, from a stencil row s9
  auto offc = [&](const TailLevel<T> &v, const T *s9, int c) -> T {
    const T *x = X + v.off;
    const int w = v.nx;
    return s9[0] * x[c - w - 1] + s9[1] * x[c - w] + s9[2] * x[c - w + 1] + s9[3] * x[c - 1] +
           s9[5] * x[c + 1] + s9[6] * x[c + w - 1] + s9[7] * x[c + w] + s9[8] * x[c + w + 1];
  };
  auto load_row = [&](const TailLevel<T> &v, int c, T s9[9]) {
    const size_t n = (size_t)v.nx * v.ny;
#pragma unroll
    for (int z = 0; z < 9; ++z) s9[z] = v.st[z * n + c];
  };
  auto rhs = [&](const TailLevel<T> &v, int c) -> T { return v.boff < 0 ? v.b[c] : Bs[v.boff + c]; };

  auto smooth = [&](int r, int sweeps) {
    const TailLevel<T> &v = lvl(r);
    if (r >= 2) {
      // the node k = t of each colour, its stencil loaded one phase ahead
      T s9n[9];
      int cn = colour_node(v.nx, v.ny, 0, t), dn = 1;
      if (cn >= 0) {
        dn = v.dir[cn];
        load_row(v, cn, s9n);
      }
      for (int s = 0; s < sweeps; ++s)
        for (int col = 0; col < 4; ++col) {
          T s9[9];
#pragma unroll
          for (int z = 0; z < 9; ++z) s9[z] = s9n[z];
          const int c = cn, d = dn;
          if (s + 1 < sweeps || col < 3) {
            cn = colour_node(v.nx, v.ny, (col + 1) & 3, t);
            if (cn >= 0) {
              dn = v.dir[cn];
              load_row(v, cn, s9n);
            }
          }
          if (c >= 0 && !d) X[v.off + c] = (rhs(v, c) - offc(v, s9, c)) * (T(1) / s9[4]);
          for (int k = t + kTailThreads;; k += kTailThreads) {  // nodes beyond the first
            const int c2 = colour_node(v.nx, v.ny, col, k);
            if (c2 < 0) break;
            if (v.dir[c2]) continue;
            T s2[9];
            load_row(v, c2, s2);
            X[v.off + c2] = (rhs(v, c2) - offc(v, s2, c2)) * (T(1) / s2[4]);
          }
          __syncthreads();
        }
    } else {
      const Own<T> &o = own[r & 1];
      for (int s = 0; s < sweeps; ++s)
        for (int col = 0; col < 4; ++col) {
          if (o.c >= 0 && o.col == col && o.ik != T(0))
            X[v.off + o.c] = (o.b - offc(v, o.a, o.c)) * o.ik;
          __syncthreads();
        }
    }
  };

#pragma unroll
  for (int r = kTailLevels - 1; r >= 1; --r) {
    if (r > nl - 1) continue;
    const TailLevel<T> &v = lvl(r), &cv = lvl(r - 1);
    smooth(r, a.nu1);
    // residual into Rb, then full weighting into the coarse right-hand side
    if (r >= 2) {
      const int n = v.nx * v.ny;
      for (int c = t; c < n; c += kTailThreads) {
        const int i = c % v.nx, j = c / v.nx;
        T res = T(0);
        if (i > 0 && j > 0 && i < v.nx - 1 && j < v.ny - 1 && !v.dir[c]) {
          T s9[9];
          load_row(v, c, s9);
          res = rhs(v, c) - offc(v, s9, c) - s9[4] * X[v.off + c];
        }
        Rb[c] = res;
      }
    } else {
      const Own<T> &o = own[r & 1];
      if (o.c >= 0)
        Rb[o.c] = o.ik != T(0) ? o.b - offc(v, o.a, o.c) - o.a[4] * X[v.off + o.c] : T(0);
    }
    __syncthreads();
    const int nc = cv.nx * cv.ny;
    for (int C = t; C < nc; C += kTailThreads) {
      const int I = C % cv.nx, J = C / cv.nx;
      T s = T(0);
      if (I > 0 && J > 0 && I < cv.nx - 1 && J < cv.ny - 1) {
        const int f = (2 * J) * v.nx + 2 * I, w = v.nx;
        const T e = Rb[f - w] + T(2) * Rb[f] + Rb[f + w];
        const T ww = Rb[f - w - 1] + T(2) * Rb[f - 1] + Rb[f + w - 1];
        const T ee = Rb[f - w + 1] + T(2) * Rb[f + 1] + Rb[f + w + 1];
        s = (ww + T(2) * e + ee) * T(0.0625);
      }
      if (r - 1 >= 2)
        Bs[cv.boff + C] = s;
      else
        own[(r - 1) & 1].b = s;  // C == t: the level has at most 289 nodes
    }
    __syncthreads();
  }
  {  // coarsest level: x = A^-1 b
    const TailLevel<T> &v = lvl(0);
    const int n = v.nx * v.ny, m = a.cidx[n];
    if (t < n) {
      const int k = a.cidx[t];
      if (k >= 0) bb[k] = (double)own[0].b;
    }
    __syncthreads();
    if (t < n) {
      const int k = a.cidx[t];
      double s = 0.0;
      if (k >= 0)
        for (int q = 0; q < m; ++q) s += a.cinv[(size_t)q * m + k] * bb[q];
      X[v.off + t] = (T)s;
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 1; r < kTailLevels; ++r) {
    if (r > nl - 1) continue;
    const TailLevel<T> &v = lvl(r), &cv = lvl(r - 1);
    const T *xc = X + cv.off;
    const int n = v.nx * v.ny;
    for (int c = t; c < n; c += kTailThreads) {
      const int i = c % v.nx, j = c / v.nx;
      if (i == 0 || j == 0 || i == v.nx - 1 || j == v.ny - 1 || v.dir[c]) continue;
      const int I = i >> 1, J = j >> 1;
      const T *r0 = xc + J * cv.nx;
      T e0 = (i & 1) ? T(0.5) * (r0[I] + r0[I + 1]) : r0[I];
      if (j & 1) {
        const T *r1 = r0 + cv.nx;
        const T e1 = (i & 1) ? T(0.5) * (r1[I] + r1[I + 1]) : r1[I];
        e0 = T(0.5) * (e0 + e1);
      }
      X[v.off + c] += e0;
    }
    __syncthreads();
    smooth(r, a.nu2);
  }
  // iterates of every tail level back to global memory
  for (int q = 0; q < nl; ++q) {
    const TailLevel<T> &v = a.lv[q];
    for (int c = t; c < v.nx * v.ny; c += kTailThreads) v.x[c] = X[v.off + c];
  }
}

template <typename T>
__global__ __launch_bounds__(kTailThreads) void k_tail(TailArgs<T> a) {
  if (a.skip && *a.skip != 0.0) return;
  tail_body<T>(a);
}

// Batched form: one workgroup per problem.
template <typename T>
__global__ __launch_bounds__(kTailThreads) void k_tail_b(BatchTab tab) {
  const TailArgs<T> &a = *static_cast<const TailArgs<T> *>(tab.e[blockIdx.x].args);
  tail_body<T>(a);
}

}  // namespace

// Number of nodes a level may have to be handled by the tail.  A problem
// alone hands the tail its levels from 33 x 33 down: the fused passes of
// one-wave blocks on the 65 x 65 level cost less than that level in the
// single workgroup (129^2 FP64 solve 0.651 -> 0.567 ms, 4097^2 11.83 ->
// 11.68 ms).  In a batch the tail takes over from 65 x 65: there the
// batched passes of that level cost more than the tail (the 256-problem
// batch 26.5 -> 27.2 ms mixed with the tail from 33 x 33).
int tail_max_nodes(bool batch) { return batch ? kTailMaxNodes : 33 * 33; }

// Largest tail LDS footprint for the node limits above: the first level at
// kTailMaxNodes, three more each at most a quarter of the previous plus a
// ring, one residual array and the streamed right-hand sides.
static_assert((kTailMaxNodes * 2 + 1100 + 300 + 100 + 1100) * 8 <= kTailLdsMax,
              "tail LDS exceeds the workgroup limit");

template <typename T>
static TailArgs<T> make_tail_args(tomg_problem *p, int lc) {
  TailArgs<T> a{};
  const bool f32 = std::is_same<T, float>::value;
  a.lc = lc;
  a.nl = p->L - lc;
  a.nu1 = p->cfg.nu1;
  a.nu2 = p->cfg.nu2;
  a.cinv = p->cinv;
  a.cidx = p->cidx;
  int off = 0, rmax = 0, boff = 0;
  for (int q = 0; q < a.nl; ++q) {
    const Level &v = p->lv[lc + q];
    a.lv[q].nx = v.nx;
    a.lv[q].ny = v.ny;
    a.lv[q].st = (const T *)(f32 ? (void *)v.st32 : (void *)v.st);
    a.lv[q].x = (T *)(f32 ? (void *)v.x32 : (void *)v.x);
    a.lv[q].b = (const T *)(f32 ? (void *)v.b32 : (void *)v.b);
    a.lv[q].dir = v.dir;
    a.lv[q].off = off;
    const int n = v.nx * v.ny;
    a.lv[q].boff = -1;
    if (q > 0 && q < a.nl - 2) {  // streamed level below the first
      a.lv[q].boff = boff;
      boff += n;
    }
    off += n;
    if (q < a.nl - 1) rmax = rmax > n ? rmax : n;
  }
  a.shmem = (off + rmax + boff) * (int)sizeof(T);
  return a;
}

void build_tail_args(tomg_problem *p) {
  p->hargs.tail64 = make_tail_args<double>(p, p->lc);
  p->hargs.tail64b = make_tail_args<double>(p, p->lcb);
  if (p->cfg.precision == TOMG_FP32_IR) {
    p->hargs.tail32 = make_tail_args<float>(p, p->lc);
    p->hargs.tail32b = make_tail_args<float>(p, p->lcb);
  }
}

// Levels lc..L-1 in one workgroup; xs/bs/sts give the per-level correction,
// right-hand side and stencil arrays of precision T (indexed by level).
template <typename T>
void tail_cycle(tomg_problem *p, int lc, T *const *xs, T *const *bs, const T *const *sts) {
  TailArgs<T> a = make_tail_args<T>(p, lc);
  for (int q = 0; q < a.nl; ++q) {
    a.lv[q].st = sts[lc + q];
    a.lv[q].x = xs[lc + q];
    a.lv[q].b = bs[lc + q];
  }
  a.skip = p->skip;
  hipLaunchKernelGGL((k_tail<T>), 1, kTailThreads, a.shmem, p->stream, a);
}

template void tail_cycle<double>(tomg_problem *, int, double *const *, double *const *,
                                 const double *const *);
template void tail_cycle<float>(tomg_problem *, int, float *const *, float *const *,
                                const float *const *);

void batch_tail(tomg_problem *const *probs, const int *idx, int cnt, bool fp32, hipStream_t s) {
  BatchTab tab;
  for (int k0 = 0; k0 < cnt; k0 += kBatchMax) {
    tab.count = 0;
    int shmem = 0;
    for (int k = k0; k < cnt && k < k0 + kBatchMax; ++k) {
      tomg_problem *p = probs[idx[k]];
      BatchEntry &e = tab.e[tab.count];
      e.args = fp32 ? (const void *)&p->dargs->tail32b : (const void *)&p->dargs->tail64b;
      e.phi = nullptr;
      e.role = 0;
      e.nbx = e.nby = 1;
      e.start = tab.count;
      e.slot = e.out = 0;
      const int sh = fp32 ? p->hargs.tail32b.shmem : p->hargs.tail64b.shmem;
      shmem = shmem > sh ? shmem : sh;
      ++tab.count;
    }
    if (!tab.count) continue;
    if (fp32)
      hipLaunchKernelGGL(k_tail_b<float>, tab.count, kTailThreads, shmem, s, tab);
    else
      hipLaunchKernelGGL(k_tail_b<double>, tab.count, kTailThreads, shmem, s, tab);
  }
}

}  // namespace tomg

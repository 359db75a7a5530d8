// Internal declarations shared by the HIP translation units of libtomg.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "tomg.h"

namespace tomg {

constexpr int kMaxLevels = 16;
constexpr int kMaxCoarseUnknowns = 49;  // coarsest grid <= 9 x 9 nodes
// A grid whose halving stops above 9 x 9 (5 x 5 with Neumann edges) keeps a
// coarsest level of at most this many nodes (the 201 x 201 family: 26 x 26),
// inverted through a band LU factorisation.
constexpr int kMaxCoarseNodes = 1024;
constexpr int kSmallCoarseNodes = 81;
constexpr int kRedBlocks = 1024;        // fixed grid of every reduction kernel
constexpr int kRedThreads = 256;
constexpr int kRedTileW = 64, kRedTileH = 32;  // level-0 reduction tiles (columns x rows)

// Slots of the device scalar block.
enum Slot {
  kSlotB0 = 0,      // ||f - A phi0||_2
  kSlotRes = 1,     // last residual norm
  kSlotMinDet = 2,  // min det J over non-corner nodes (setup)
  kSlotBad = 3,     // count of non-finite values (setup)
  kSlotPivot = 4,   // nonzero when the coarsest matrix is singular
  kSlotRel = 5,     // last relative residual
  kSlotDone = 6,    // convergence flag (1.0 when rel <= tol)
  kSlotTol = 7,     // stopping tolerance used by the device-side check
  kSlotCycles = 8,  // cycles whose norm was finalized (counted on the device)
  kSlotBadRhs = 9,  // count of non-finite right-hand-side values (update_rhs)
  kSlotR0 = 10,     // residual norm of the solve's starting iterate (the
                    // denominator of the relative residual when kSlotB0 is 0)
  kNumSlots = 16
};
// After the slots: the relative residual at the start of the last solve and
// after each of its cycles (the first kHistMax), for tomg_residual_history.
enum {
  kHistMax = 256
};

// Modes of the relative-residual bookkeeping of a finalize: none; the
// initial norms of a solve (also records kSlotR0); after a cycle.
enum { kRelNone = 0, kRelBegin = 1, kRelCycle = 2 };

struct Level {
  int nx = 0, ny = 0;
  int ck = 0;  // transfer to the next level: 0 both axes halved, 1 x only, 2 y only
  size_t n = 0;
  double *st = nullptr;  // 9 planes (levels >= 1)
  double *x = nullptr;   // correction (levels >= 1)
  double *b = nullptr;   // right-hand side (levels >= 1)
  double *x2 = nullptr;  // second iterate buffer of the fused passes (levels >= 1)
  uint8_t *dir = nullptr;
  float *st32 = nullptr, *x32 = nullptr, *b32 = nullptr, *x2_32 = nullptr;  // FP32 (IR)
  // alternating zebra: the level transposed (node (i, j) at i * ny + j)
  double *stT = nullptr, *xT = nullptr, *bT = nullptr;
  uint8_t *dirT = nullptr;
};

// ---- per-problem launch arguments (device copies live in the workspace) ----

// One fused level pass (fused.hip).
template <typename T>
struct PassArgs {
  int nx, ny;
  const T *xin;              // level iterate read (unless the pass starts at zero)
  T *xout;                   // level iterate written (never the array read)
  const T *b;                // level right-hand side
  const uint8_t *dir;        // Dirichlet flags of the level
  const T *exx, *exy, *eyy;  // level 0: permittivity tensor
  const T *st;               // coarse levels: 9-point stencil planes
  T cx, cy, qx, qy, qxy, hxy;
  const T *xc;               // up pass: coarse correction
  T *bc;                     // down pass: coarse right-hand side
  const uint8_t *dirc;       // coarse flags where the coarse ring may hold
                             // unknowns (Neumann edges), else null
  int nxc, nyc;
  double *partials;          // up pass with norm: one double per block
  int CH, W;                 // band height, owned columns per block
  int nbx, nby;              // block grid
  int xcd_order;             // tiles in XCD-contiguous order (one-dimensional grid)
  int ck;                    // transfer to the coarse level: 0 both axes halved, 1 x, 2 y
  int bw;                    // threads (columns) per block
  const double *skip;        // nonzero *skip: the launch does nothing (solve()
                             // queues cycles past convergence as no-ops)
};

// One level of the single-workgroup tail (tail.hip).
template <typename T>
struct TailLevel {
  int nx, ny;
  const T *st;
  T *x;
  const T *b;
  const uint8_t *dir;
  int off;   // offset of the level's iterate in the LDS array
  int boff;  // offset of its right-hand side in LDS (levels after the first
             // with more nodes than the tail has threads), else -1
};
constexpr int kTailLevels = 4;
template <typename T>
struct TailArgs {
  int lc, nl, nu1, nu2;  // levels lc .. lc+nl-1 (the last is the coarsest)
  const double *cinv;
  const int *cidx;
  int shmem;             // dynamic LDS bytes
  const double *skip;    // as in PassArgs
  TailLevel<T> lv[kTailLevels];
};

// Level-0 residual reductions and the refinement kernels (kernels.hip).
struct RedArgs {
  const double *exx, *exy, *eyy;
  double cx, cy, qx, qy, qxy, hxy;
  int nx, ny;
  const double *f;
  const uint8_t *dir;
  double *partials;
  float *r32, *e32;
  double *tmp;
  const double *st0;  // level-0 stencil (Neumann edges only, else null)
  double *phi2;       // second array of the iterate (refinement), else null
  int nblk;  // tiles of the reduction (a function of the grid size only)
};

// Coarsest inverse of one problem (its launch may be deferred and batched).
struct InvArgs {
  const double *st;
  const uint8_t *dir;
  double *band;  // band LU workspace of a coarsest level above kSmallCoarseNodes
  int nx, ny;
  double *inv;
  int *cidx;
  double *scal;
};

// Fixed-order reduction of partials into the scalar block.
struct FinArgs {
  const double *partials;
  double *scal;
  int n;
};

struct ArgsBlob {
  PassArgs<double> down64[kMaxLevels], up64[kMaxLevels];
  PassArgs<float> down32[kMaxLevels], up32[kMaxLevels];
  // the same passes as launched in a batch: taller bands, since the other
  // problems of the batch fill the device
  PassArgs<double> down64b[kMaxLevels], up64b[kMaxLevels];
  PassArgs<float> down32b[kMaxLevels], up32b[kMaxLevels];
  // level 0 of the FP32 inner cycles: the up pass of a cycle and the down
  // pass of the next in one launch (nu2 + nu1 sweeps)
  PassArgs<float> updown32;
  TailArgs<double> tail64;
  TailArgs<float> tail32;
  TailArgs<double> tail64b;  // the tail as launched in a batch (from level lcb)
  TailArgs<float> tail32b;
  RedArgs red;
  FinArgs fin_red, fin_norm, fin_red0;  // partials of the reductions, the up pass,
                                        // and the second half of a two-norm pass
  FinArgs fin_normb;                    // the up pass as launched in a batch
  InvArgs inv;                          // the coarsest inverse
};

// One problem's share of a batched launch: blocks [start, start + nbx*nby).
// phi/role: the level-0 iterate of this solve (role 1: the array the pass
// reads, 2: the array it writes).  slot/out: where a finalize writes.
struct BatchEntry {
  const void *args;
  void *phi;
  int role, nbx, nby, start, slot, out;
};
constexpr int kBatchMax = 96;
struct BatchTab {
  int count;
  BatchEntry e[kBatchMax];
};
constexpr int kMaxBatch = 4096;  // problems per tomg_solve_batch call

// Byte offsets of every array inside the caller's workspace.
struct Layout {
  int L = 0;
  int nx[kMaxLevels], ny[kMaxLevels];
  int ck[kMaxLevels];  // transfer kind to the next level (0 full, 1 x halved, 2 y halved)
  size_t exx, exy, eyy, det, f, tmp, partials, scal, cinv, cidx, cband;
  size_t dir[kMaxLevels], st[kMaxLevels], x[kMaxLevels], b[kMaxLevels], x2[kMaxLevels];
  size_t exx32, exy32, eyy32, e32, e32b, r32, phi2;
  size_t st32[kMaxLevels], x32[kMaxLevels], b32[kMaxLevels], x2_32[kMaxLevels];
  size_t stT[kMaxLevels], xT[kMaxLevels], bT[kMaxLevels], dirT[kMaxLevels];
  size_t args, bout;  // device copy of the launch arguments; batch results
  size_t total = 0;
};

// Level shapes of a configuration; ck[l] (nullable) receives the kind of
// the transfer from level l to l + 1: 0 both axes halved, 1 x only, 2 y only.
int level_shapes(const tomg_config &c, int *nxs, int *nys, int *ck);

// The level-0 operator is stored as a 9-point stencil (Neumann edges, or the
// flux form) and every cycle runs the unfused kernels on stored stencils.
// Longest line of the zebra smoothers: four padded FP64 rows of LDS fit in
// 160 KB.
constexpr int kZebraMaxNx = 4225;

inline bool stored_level0(const tomg_config &c) {
  return c.neumann != 0 || c.flux != 0 || c.smoother == TOMG_ZEBRA_XY;
}
bool make_layout(const tomg_config &cfg, Layout *lay);

}  // namespace tomg

struct tomg_problem {
  tomg_config cfg;
  tomg::Layout lay;
  hipStream_t stream = nullptr;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  int L = 0;
  tomg::Level lv[tomg::kMaxLevels];
  double *exx = nullptr, *exy = nullptr, *eyy = nullptr, *det = nullptr, *f = nullptr;
  double *tmp = nullptr, *partials = nullptr, *scal = nullptr, *cinv = nullptr;
  double *phi2 = nullptr;  // refinement: second array of the iterate
  double *cband = nullptr; // band LU of a large coarsest level
  int *cidx = nullptr;
  float *exx32 = nullptr, *exy32 = nullptr, *eyy32 = nullptr, *e32 = nullptr, *r32 = nullptr;
  float *e32b = nullptr;
  tomg::ArgsBlob *dargs = nullptr;  // device copy of hargs
  tomg::ArgsBlob hargs;             // host copy (source of the upload)
  double *bout = nullptr;           // batch results (used when this problem leads a batch)
  int lc = 0;                       // first level of the tail
  int lcb = 0;                      // the same in a batched launch
  int m_coarse = 0;
  const double *skip = nullptr;     // device convergence flag while solve() queues cycles
  double up[2] = {0.0, 0.0};        // source of the tolerance/cycle-count upload
  bool unchecked = false;           // setup issued without its host-side check
  double last_rate = 0.0;           // mean contraction per cycle of the last converged
                                    // solve (0: none yet)
  double last_rel0 = 1.0;           // the initial relative residual of that solve
  bool inv_pending = false;         // coarsest inverse of the last setup not launched yet
  bool has_map = false;             // the last setup came from a map descriptor
  tomg_map_desc map{};              // ... this one (for tomg_update_rhs_desc)
  bool ready = false;
  // level-0 pass timing (tomg_profile): event pairs recorded since the last
  // harvest, per kind (0 down, 1 up)
  static constexpr int kMaxEv = 64;
  static constexpr int kProfKinds = 3;  // level-0 down, up, and chained up-down passes
  bool prof = false;
  hipEvent_t ev[kProfKinds][kMaxEv][2] = {};
  int nev[kProfKinds] = {0, 0, 0};
  double prof_ms[kProfKinds] = {0, 0, 0};
  double prof_cnt[kProfKinds] = {0, 0, 0};
  char err[512];
};

namespace tomg {

// ---- launch wrappers (kernels.hip); each returns hipSuccess or the error ----
hipError_t launch_setup(tomg_problem *p, const double *xp, const double *yp, const double *jac,
                        const double *epsp, const double *rho, const uint8_t *mask);
hipError_t launch_update_rhs(tomg_problem *p, const double *rho);
hipError_t finish_setup(tomg_problem *p);
hipError_t launch_setup_desc(tomg_problem *p, const tomg_map_desc &m, const tomg_source_desc &src,
                             double *phi_init);
hipError_t launch_update_rhs_desc(tomg_problem *p, const tomg_map_desc &m,
                                  const tomg_source_desc &src);
// Galerkin (or rediscretised) levels; the coarsest inverse too unless
// defer_inverse (then it is launched by launch_coarse_inverse or, batched,
// by batch_coarse_inverse before the problem's next cycle).
hipError_t launch_hierarchy(tomg_problem *p, bool defer_inverse = false);
// The problem's pending coarsest inverse, if any, on its stream.
hipError_t launch_coarse_inverse(tomg_problem *p);
// The pending coarsest inverses of probs[idx[0..cnt)] in one launch per up to
// kBatchMax problems (one workgroup each) on stream s.
void batch_coarse_inverse(tomg_problem *const *probs, const int *idx, int cnt, hipStream_t s);
hipError_t launch_vcycle64(tomg_problem *p, double *phi, bool with_norm);

// fused level passes (fused.hip)
template <typename T>
void fused_down(tomg_problem *p, int l, const T *x, T *pong, const T *b, const T *exx,
                const T *exy, const T *eyy, const T *st, T *bc, bool zero_start);
template <typename T>
int fused_up(tomg_problem *p, int l, const T *pong, T *x, const T *b, const T *exx,
             const T *exy, const T *eyy, const T *st, const T *xc, double *partials);
size_t fused_max_blocks(int nx, int ny);
// Whether the FP32 inner cycles run chained (fused_updown): four-colour
// smoother, nu1 + nu2 <= 4, the level-0 stencil stored.
bool chain_inner(const tomg_problem *p);
// Level-0 up pass of an FP32 inner cycle and down pass of the next in one
// launch: pong (plus the prolongation of xc) in, nu2 + nu1 sweeps, the
// result to out, the residual restricted into bc.
template <typename T>
void fused_updown(tomg_problem *p, const T *pong, T *out, const T *b, const T *exx,
                  const T *exy, const T *eyy, const T *st, const T *xc, T *bc);

// levels lc..L-1 of the cycle in one workgroup (tail.hip)
template <typename T>
void tail_cycle(tomg_problem *p, int lc, T *const *xs, T *const *bs, const T *const *sts);
int tail_max_nodes(bool batch);
hipError_t launch_ir_residual(tomg_problem *p, const double *phi);
hipError_t launch_ir_correct(tomg_problem *p, double *phi);
hipError_t launch_ir_inner(tomg_problem *p);
hipError_t launch_ir_step(tomg_problem *p, double *phi, bool second);
hipError_t launch_begin(tomg_problem *p, const double *phi, bool ir);
hipError_t launch_setup_identity(tomg_problem *p, const uint8_t *mask);
hipError_t launch_zero(tomg_problem *p, double *x, size_t n);
// scal[k] = v for every bit k of mask (a fill kernel on the problem's stream)
hipError_t launch_set_slots(tomg_problem *p, unsigned mask, double v);
// Queues the copy of p->hargs into p->dargs on p->stream (no host wait).
hipError_t upload_args(tomg_problem *p);
hipError_t launch_field(tomg_problem *p, const double *phi, const double *xp, const double *yp,
                        const double *jac, double *ex, double *ey);
hipError_t launch_smooth0(tomg_problem *p, double *phi, int sweeps);
hipError_t launch_residual0(tomg_problem *p, const double *phi, double *r);
hipError_t launch_copy_probe(const void *src, void *dst, size_t bytes, hipStream_t s);

// launch arguments of every stage, built once per problem (fused.hip,
// tail.hip, kernels.hip) and uploaded by tomg_create
void build_pass_args(tomg_problem *p);
void build_tail_args(tomg_problem *p);
void build_red_args(tomg_problem *p);
int red_tiles(int nx, int ny);
int tail_level(const tomg_problem *p, bool batch);

// batched stages over problems probs[idx[0..cnt-1]] (one launch per up to
// kBatchMax problems); phis: the level-0 iterate of each problem (indexed
// like probs)
void batch_down(tomg_problem *const *probs, const int *idx, int cnt, int l, bool fp32, bool zero0,
                double *const *phis, hipStream_t s);
void batch_up(tomg_problem *const *probs, const int *idx, int cnt, int l, bool fp32, bool norm,
              double *const *phis, hipStream_t s);
void batch_tail(tomg_problem *const *probs, const int *idx, int cnt, bool fp32, hipStream_t s);
void batch_resnorm(tomg_problem *const *probs, const int *idx, int cnt, bool zero_free,
                   double *const *phis, hipStream_t s);
void batch_ir_residual(tomg_problem *const *probs, const int *idx, int cnt, double *const *phis,
                       hipStream_t s);
// both initial norms (and r32 with ir) in one pass: partials of the iterate's
// residual in fin_red, of the zero-interior residual in fin_red0
void batch_begin_norms(tomg_problem *const *probs, const int *idx, int cnt, bool ir,
                       double *const *phis, hipStream_t s);
void batch_ir_update(tomg_problem *const *probs, const int *idx, int cnt, double *const *phis,
                     hipStream_t s);
// update and residual in one pass (launch_ir_step); roles[k] (indexed like
// probs): 0 the iterate moves from phis[k] to the problem's phi2, 1 back
void batch_ir_step(tomg_problem *const *probs, const int *idx, int cnt, double *const *phis,
                   const int *roles, hipStream_t s);
// phis[k] = the problem's phi2
void batch_copy_back(tomg_problem *const *probs, const int *idx, int cnt, double *const *phis,
                     hipStream_t s);
// kind 0: the reduction partials (fin_red), 1: the level-0 up-pass partials
// (fin_norm), 2: the second half of a two-norm pass (fin_red0); slot: scalar
// slot written; rel (kRel*): also write rel and done, and copy the value into
// out[k] for entry k (out = the leading problem's bout), or into out[idx[k]]
// with by_index
void batch_finalize(tomg_problem *const *probs, const int *idx, int cnt, int kind, int slot,
                    int rel, double *out, hipStream_t s, bool by_index = false);

// Pass timing around level-0 passes (no-ops unless p->prof).
void prof_begin(tomg_problem *p, int kind);
void prof_end(tomg_problem *p, int kind);
void prof_harvest(tomg_problem *p);

}  // namespace tomg

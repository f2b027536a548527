// device.hpp -- shared device-side types and helpers of the gfx950 kernels.
//
// Layout and launch conventions used by every grid kernel:
//   * vectors are lexicographic, x fastest (index i + nx j + nx ny k);
//   * a thread owns "groups" of VEC consecutive x-values (VEC = 4 when nx % 4 == 0,
//     else 1), so a group never straddles an x-row;
//   * a block owns a contiguous range of nit*TPB groups; the block index is remapped so
//     that the 8 XCDs (each with its own L2) each own one contiguous eighth of the grid
//     (hardware dispatch sends block b to XCD b % 8), which keeps stencil halo planes of
//     neighbouring blocks in the same L2;
//   * reductions are deterministic: per-thread partial -> wave64 shuffle tree -> fixed-order
//     block sum -> per-block partials -> per-group sums (groups of 64 blocks, summed by the
//     group's last block) -> the last group to finish adds the group sums in group order in
//     FP64 and computes the dependent scalars (see reduce_to_last).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>

namespace mprk {

typedef _Float16 half_t;

constexpr int TPB = 256;             // threads per block of every grid kernel
constexpr int NWAVE = TPB / 64;
constexpr int MAXM = 32;             // max GMRES cycle length
constexpr int MAXD = MAXM + 1;       // max simultaneous dot products
constexpr int MAXRED = MAXD + 2;     // max values of one grid reduction (dots + two norms)
constexpr int MAXS = 8;              // max RK stages
constexpr int BJ_MAX = 8;            // max block-Jacobi block size

struct Geo {
  int nx, ny, nz, bc;  // bc: 0 zero Dirichlet, 1 periodic
  int N, plane;        // nx*ny*nz, nx*ny
};

struct Launch {
  int ng;   // number of groups (N / VEC, or rows for CSR kernels)
  int nit;  // groups per thread
  int G;    // blocks (a multiple of 8)
};

// 7-point stencil coefficients: w = c v + xm v[x-1] + xp v[x+1] + ym v[y-1] + ...
template <typename C>
struct Coef {
  C c, xm, xp, ym, yp, zm, zp;
};

template <typename C>
__host__ __device__ inline Coef<C> coef_cast(const Coef<double>& a) {
  return Coef<C>{(C)a.c, (C)a.xm, (C)a.xp, (C)a.ym, (C)a.yp, (C)a.zm, (C)a.zp};
}

// stencil of M = I - sigma K from the stencil of K
__host__ __device__ inline Coef<double> coef_stage(const Coef<double>& K, double sigma) {
  return Coef<double>{1.0 - sigma * K.c, -sigma * K.xm, -sigma * K.xp, -sigma * K.ym,
                      -sigma * K.yp,     -sigma * K.zm, -sigma * K.zp};
}

struct Csr {
  const int* rowptr;
  const int* col;
};

// The terms of f(y) = K y + g + R(y) besides the operator, evaluated in FP64 with it: the
// constant forcing g (N doubles, or null) and the pointwise reaction R(y) = r1 y + r2 y^2 +
// r3 y^3 (react = 0: none).
struct FTerms {
  const double* g;
  double r1, r2, r3;
  int react;
  __device__ __forceinline__ double R(double y) const { return y * (r1 + y * (r2 + y * r3)); }
};

constexpr int MAXPASS = 32;  // passes whose iteration counts are recorded
constexpr int MAXSTG = 8;    // stages whose head records a replayed step keeps on the device

// Kernel classes counted for profiling (launches that did work).
enum KClass {
  KC_STAGE_RHS = 0, KC_RESIDUAL, KC_CG_BEGIN, KC_CG_DIR, KC_CG_UPD, KC_PROMOTE,
  KC_GM_BEGIN, KC_GM_PREC, KC_GM_MATVEC, KC_GM_ORTH, KC_GM_FINISH, KC_KEPS, KC_COMBINE,
  KC_APPLY64, KC_CG_RZ, KC_FDM, KC_GM_REORTH, KC_GM_STEP, KC_GM_CLOSE, KC_COUNT
};

// Device control record of one solve context (one per problem).  The first 64 bytes
// are the head the host polls.
struct Ctl {
  // ---- head polled by the host (64 bytes) ----
  int outer_done;     // stage finished (converged, pass limit, or non-finite)
  int inner_done;     // current LP solve finished
  int passes;         // LP solves completed in this stage
  int iters;          // Krylov iterations of the current LP solve
  int total_iters;    // Krylov iterations of this stage (all passes)
  int nonfinite;      // a non-finite FP64 residual was seen in this stage
  int converged;      // outer residual reached outer_tol
  int J;              // GMRES: Arnoldi vectors in the current cycle
  double outer_rel;   // ||res|| / ||rhs|| of the last FP64 residual
  double res_norm;    // ||res||_2
  long long good_steps;  // steps whose combination was applied
  int bad_steps;         // steps skipped because of a non-finite residual
  int step_nonfinite;    // sticky for the current step (gates the combination)
  // ---- body ----
  long long life_iters;   // Krylov iterations since bind
  long long life_passes;  // LP solves since bind
  long long missed;       // stages finished without reaching their tolerance, since bind
  long long held_steps;   // strict: steps not combined because a stage missed its tolerance
  int inner_conv;         // the current LP solve stopped because it reached its tolerance
  int step_held;          // strict: a stage of the current step missed (gates the combination)
  int halt;               // strict: a stage missed in this call; its remaining stages are skipped
  double rhs_norm;    // ||rhs||_2
  double scale;       // LP right-hand side = res / scale (scale = ||res||_2 / sqrt(N))
  double tol;         // inner stopping tolerance in LP units
  double rz, pq, alpha, beta, rr;
  double hcol[MAXD];                 // current Hessenberg column (latest Gram-Schmidt pass)
  double hacc[MAXD];                 // its coefficients from the step's earlier pass (CGS2)
  double H[(MAXM + 1) * MAXM];       // Hessenberg matrix, column-major (MAXM+1 rows)
  double cs[MAXM], sn[MAXM];         // Givens rotations
  double g[MAXM + 1];                // rotated right-hand side
  double ysol[MAXM];                 // least-squares solution of the cycle
  double vscale[MAXM + 1];           // basis vector i = vscale[i] * stored vector i
  double zc;     // fused GMRES step: the stored product of the pending column is zc times the
                 // product of the normalised basis vector
  double znext;  // fused GMRES step: scale of the next step's stencil input (an estimate of the
                 // inverse norm of the next stored basis vector, which keeps values O(1))
  int pass_iters[MAXPASS];           // Krylov iterations of each pass of the current stage
  long long worked[KC_COUNT];        // launches per kernel class that did work (profiling)
  long long units[KC_COUNT];         // basis vectors touched (GMRES kernels), else launches
  long long srec[MAXSTG][8];         // steps replayed from a graph: each stage's final head
};

__device__ __forceinline__ void count_work(Ctl* ctl, int kc, int units = 1) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->worked[kc] += 1;
    ctl->units[kc] += units;
  }
}

// The host polls this prefix of Ctl.
struct CtlHead {
  int outer_done, inner_done, passes, iters, total_iters, nonfinite, converged, J;
  double outer_rel, res_norm;
  long long good_steps;
  int bad_steps, step_nonfinite;
};
static_assert(sizeof(CtlHead) == 64, "poll head must be 64 bytes");


// k_stage_rhs reset flags: a new stage, a new step, a new library call (clears the halt)
enum { RESET_STAGE = 1, RESET_STEP = 2, RESET_CALL = 4 };

struct SolveCfg {
  double sigma;        // tau a_ii
  double outer_tol;
  int max_passes;      // LP solves per stage (>= 1)
  int paper_mode;      // refine_max == 0
  int outer_stop;      // inner solves also stop at the outer target (outer loop only)
  int strict;          // a stage that misses its tolerance fails the step (u is not updated)
  double rtol, atol;
  int maxit;           // Krylov iterations per LP solve
  int m;               // GMRES cycle length
  double sqrtN;
  double invN;
};

// Inner stopping target from the outer test: the update y += scale x leaves an FP64 residual
// of about unit times the LP residual's norm, so an LP residual below half of
// outer_tol ||rhs|| / unit already meets the outer tolerance and further iterations are not
// needed (the inner rtol stays the bound on them).  Only where outer_stop is set (by default
// with LP storage and the outer loop: the one-solve mode has no outer test, and an FP64 inner
// solve's own tolerance is the accuracy asked for).  unit: the FP64 norm of one unit of the LP norm (scale for the
// 2-norm, scale sqrt N for the RMS norm).
__device__ __forceinline__ double outer_target(const SolveCfg& cfg, const Ctl* ctl, double unit) {
  return cfg.outer_stop ? 0.5 * cfg.outer_tol * ctl->rhs_norm / unit : 0.0;
}

template <typename T, int V>
struct alignas(sizeof(T) * V) Vec {
  T v[V];
};

template <typename C, typename S, int V>
__device__ __forceinline__ void loadv(const S* __restrict__ p, C (&o)[V]) {
  Vec<S, V> t = *reinterpret_cast<const Vec<S, V>*>(p);
#pragma unroll
  for (int i = 0; i < V; ++i) o[i] = (C)t.v[i];
}

template <typename S, typename C, int V>
__device__ __forceinline__ void storev(S* __restrict__ p, const C (&o)[V]) {
  Vec<S, V> t;
#pragma unroll
  for (int i = 0; i < V; ++i) t.v[i] = (S)o[i];
  *reinterpret_cast<Vec<S, V>*>(p) = t;
}

// round a compute value through the storage type (what a store + reload would give)
template <typename S, typename C>
__device__ __forceinline__ C rnd(C x) {
  return (C)(S)x;
}

__device__ __forceinline__ int xcd_block(int G) {
  const int b = blockIdx.x;
  return (b & 7) * (G >> 3) + (b >> 3);
}

// One DPP step: v + (v moved by the DPP pattern CTRL; 0 where the pattern has no source or the
// row is masked off).  A double moves as its two 32-bit halves.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  const long long m = ((long long)hi << 32) | (unsigned int)lo;
  return v + __builtin_bit_cast(double, m);
}

// Sum over the 64 lanes of a wave, in a fixed order, returned to every lane: an inclusive scan
// inside each row of 16 lanes (row_shr 1, 2, 4, 8), then row 0's total added into row 1 and
// row 2's into row 3 (row_bcast15), then rows 0-1 into rows 2-3 (row_bcast31); lane 63 then
// holds the total, which is read back as a scalar.  Only DPP moves: no LDS round trips.
__device__ __forceinline__ double wave_sum(double v) {
  v = dpp_add<0x111, 0xf>(v);  // row_shr:1
  v = dpp_add<0x112, 0xf>(v);  // row_shr:2
  v = dpp_add<0x114, 0xf>(v);  // row_shr:4
  v = dpp_add<0x118, 0xf>(v);  // row_shr:8
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Workspace of a grid reduction.  Level 1: one partial per block, p1[d * s1 + L]; level 2: one
// sum per group of RGRP consecutive blocks, p2[d * s2 + group].  Counters: tick[0] counts the
// groups done, tick[TSTRIDE * (1 + group)] the blocks of a group done (256 bytes apart, so that
// concurrent tickets of different groups do not share a line).  All counters are zero between
// launches (each is reset by the block that completes it).
constexpr int RGRP = 64;
constexpr int TSTRIDE = 64;

struct Red {
  double* p1;
  double* p2;
  unsigned int* tick;
  int s1, s2;
};

// Number of counters a reduction over at most G blocks needs.
__host__ __device__ inline size_t red_ticks(long G) {
  return (size_t)TSTRIDE * (size_t)(1 + (G + RGRP - 1) / RGRP);
}

// Publish the calling wave's device-scope partial stores, then take a ticket.  The partials are
// written with device-scope atomic stores, which are coherent across the XCDs once complete;
// s_waitcnt 0 waits for their completion before the ticket is taken, so whoever draws the last
// ticket reads (with device-scope loads) every published value.  No L2 writeback is needed:
// only these partials cross blocks, never the kernel's plain data stores.
__device__ __forceinline__ unsigned int publish_ticket(unsigned int* ctr) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  return __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double load_dev(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid reduction of nd (<= ND <= 64) per-thread values in fixed order: wave64 shuffle tree,
// block sum over the waves, one partial per block; the last block of each group of RGRP blocks
// sums the group's partials (one wave, lane = block within the group); the last group to finish
// sums the group sums.  Returns true in that final block, where tot[0..nd) (shared memory)
// holds the totals.  The order of every addition depends only on G and the block indices, so
// results are bitwise reproducible for a given launch shape.
template <int ND>
__device__ bool reduce_to_last(const double (&v)[ND], int nd, const Red& red, int L, int G,
                               double* tot) {
  static_assert(ND <= 64, "one wave publishes all values of a block");
  __shared__ double wsum[NWAVE][ND];
  __shared__ int stage;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    if (d < nd) {
      double s = wave_sum(v[d]);
      if (lane == 0) wsum[wave][d] = s;
    }
  }
  __syncthreads();
  const int grp = L / RGRP, g0 = grp * RGRP, gn = min(RGRP, G - g0);
  const int ngrp = (G + RGRP - 1) / RGRP;
  if (wave == 0) {
    if (lane < nd) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < NWAVE; ++w) s += wsum[w][lane];
      store_dev(red.p1 + (size_t)lane * red.s1 + L, s);
    }
    if (lane == 0) stage = publish_ticket(red.tick + TSTRIDE * (1 + grp)) == (unsigned)(gn - 1);
  }
  __syncthreads();
  if (!stage) return false;
  // last block of its group: group sums (wave 0, lane = block of the group)
  if (wave == 0) {
    double x[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d)
      x[d] = (d < nd && lane < gn) ? load_dev(red.p1 + (size_t)d * red.s1 + g0 + lane) : 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      if (d < nd) {
        const double s = wave_sum(x[d]);
        if (lane == d) store_dev(red.p2 + (size_t)d * red.s2 + grp, s);
      }
    }
    if (lane == 0) {
      __hip_atomic_store(red.tick + TSTRIDE * (1 + grp), 0u, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      stage = publish_ticket(red.tick) == (unsigned)(ngrp - 1) ? 2 : 0;
    }
  }
  __syncthreads();
  if (stage != 2) return false;
  // final block: every thread sums a strided slice of each value's group sums, then a fixed
  // shuffle tree and a fixed-order combine of the waves
  __shared__ double wtot[NWAVE][ND];
  for (int d = 0; d < nd; ++d) {
    const double* p = red.p2 + (size_t)d * red.s2;
    double s = 0.0;
    for (int b = threadIdx.x; b < ngrp; b += TPB) s += load_dev(p + b);
    s = wave_sum(s);
    if (lane == 0) wtot[wave][d] = s;
  }
  __syncthreads();
  if (threadIdx.x < nd) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) s += wtot[w][threadIdx.x];
    tot[threadIdx.x] = s;
  }
  if (threadIdx.x == 0) __hip_atomic_store(red.tick, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return true;
}

// Neighbour indices of the group starting at element e (x0 = e % nx, ...); -1 = outside
// a zero-Dirichlet boundary.
struct Nbr {
  int xm, xp, ym, yp, zm, zp;
};

template <int VEC>
__device__ __forceinline__ Nbr neighbours(const Geo& g, int e) {
  const int x0 = e % g.nx;
  const int t = e / g.nx;
  const int y = t % g.ny;
  const int z = t / g.ny;
  const bool per = g.bc == 1;
  Nbr n;
  n.xm = x0 > 0 ? e - 1 : (per ? e + g.nx - 1 : -1);
  n.xp = x0 + VEC < g.nx ? e + VEC : (per ? e + VEC - g.nx : -1);
  n.ym = y > 0 ? e - g.nx : (per ? e + (g.ny - 1) * g.nx : -1);
  n.yp = y < g.ny - 1 ? e + g.nx : (per ? e - (g.ny - 1) * g.nx : -1);
  n.zm = z > 0 ? e - g.plane : (per ? e + (g.nz - 1) * g.plane : -1);
  n.zp = z < g.nz - 1 ? e + g.plane : (per ? e - (g.nz - 1) * g.plane : -1);
  return n;
}

// Apply a 7-point stencil to the group at e.  `F` supplies input values:
//   F::vec(idx, C (&)[VEC]) -- VEC consecutive values starting at idx (aligned group)
//   F::one(idx) -> C        -- one value
// With a loader `pre` (possibly empty), the caller's other independent loads are issued right
// after the seven and a scheduling barrier keeps them in flight together (the compiler would
// otherwise sink a single-value load behind waits for the others: a second memory round trip).
struct NoPre {
  __device__ __forceinline__ void operator()() const {}
};
template <typename C, int VEC, typename F, typename P = NoPre>
__device__ __forceinline__ void stencil_group(const Geo& g, const Coef<C>& k, int e, const F& f,
                                              C (&ctr)[VEC], C (&out)[VEC], const P& pre = P()) {
  const Nbr n = neighbours<VEC>(g, e);
  // every load is issued unconditionally (a missing Dirichlet neighbour reads the group itself)
  // and masked afterwards, so the seven loads are in flight together
  C l = f.one(n.xm >= 0 ? n.xm : e);
  C r = f.one(n.xp >= 0 ? n.xp : e);
  C ym[VEC], yp[VEC], zm[VEC], zp[VEC];
  f.vec(e, ctr);
  f.vec(n.ym >= 0 ? n.ym : e, ym);
  f.vec(n.yp >= 0 ? n.yp : e, yp);
  f.vec(n.zm >= 0 ? n.zm : e, zm);
  f.vec(n.zp >= 0 ? n.zp : e, zp);
  if constexpr (!std::is_same<P, NoPre>::value) {
    pre();
    __builtin_amdgcn_sched_barrier(0);
  }
  if (n.xm < 0) l = C(0);
  if (n.xp < 0) r = C(0);
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    if (n.ym < 0) ym[v] = C(0);
    if (n.yp < 0) yp[v] = C(0);
    if (n.zm < 0) zm[v] = C(0);
    if (n.zp < 0) zp[v] = C(0);
  }
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    const C left = v > 0 ? ctr[v - 1] : l;
    const C right = v < VEC - 1 ? ctr[v + 1] : r;
    C acc = k.c * ctr[v];
    acc += k.xm * left;
    acc += k.xp * right;
    acc += k.ym * ym[v];
    acc += k.yp * yp[v];
    acc += k.zm * zm[v];
    acc += k.zp * zp[v];
    out[v] = acc;
  }
}

// Input functor: plain array in storage type S, converted to C.
template <typename C, typename S, int VEC>
struct In1 {
  const S* __restrict__ a;
  __device__ __forceinline__ void vec(int i, C (&o)[VEC]) const { loadv<C, S, VEC>(a + i, o); }
  __device__ __forceinline__ C one(int i) const { return (C)a[i]; }
};

// Input functor: a + beta * b (CG search direction), with rounding through S so that every
// reader sees exactly the values the owner stores.
template <typename C, typename S, int VEC>
struct InAxpy {
  const S* __restrict__ a;
  const S* __restrict__ b;
  C beta;
  int use_b;
  __device__ __forceinline__ void vec(int i, C (&o)[VEC]) const {
    loadv<C, S, VEC>(a + i, o);
    if (use_b) {
      C t[VEC];
      loadv<C, S, VEC>(b + i, t);
#pragma unroll
      for (int v = 0; v < VEC; ++v) o[v] = rnd<S, C>(o[v] + beta * t[v]);
    }
  }
  __device__ __forceinline__ C one(int i) const {
    C o = (C)a[i];
    if (use_b) o = rnd<S, C>(o + beta * (C)b[i]);
    return o;
  }
};

// Input functor: s * a (a scaled stored vector)
template <typename C, typename S, int VEC>
struct InScaled {
  const S* __restrict__ a;
  C s;
  __device__ __forceinline__ void vec(int i, C (&o)[VEC]) const {
    loadv<C, S, VEC>(a + i, o);
#pragma unroll
    for (int v = 0; v < VEC; ++v) o[v] *= s;
  }
  __device__ __forceinline__ C one(int i) const { return s * (C)a[i]; }
};

// Block-Jacobi inverses.  mode 0: one stored inverse per block (row r's BS entries at
// inv[r * BS]); mode 1: a table of distinct inverses and idx[block] selecting one; mode 2: a
// single inverse shared by every block (constant-coefficient operators with BS | nx); mode 3:
// one inverse per block, rows interleaved for kernels whose lanes own VEC consecutive rows:
// row r = VEC g + q is the chunk ((g / 64) VEC + q) 64 + g % 64 (chunks of BS entries), so the
// q-th row load of the 64 lanes of a wave reads one contiguous 64-chunk run.
template <int VEC>
__host__ __device__ __forceinline__ size_t bj_chunk(int r) {
  const int g = r / VEC, q = r % VEC;
  return ((size_t)(g >> 6) * VEC + q) * 64 + (g & 63);
}

// Rows the interleaved layout spans for nrows rows: whole 64-lane runs of VEC rows.
__host__ __device__ inline size_t bj_chunks(long nrows, int vec) {
  const long groups = (nrows + vec - 1) / vec;
  return (size_t)((groups + 63) / 64) * 64 * vec;
}
// Mode 4 (adaptive precision): the rows of each chunk of 64 lane groups (the interleave unit
// of mode 3) are stored in one type chosen per chunk, tag[c] = 0 FP8 E4M3, 1 FP16, 2 FP32,
// 3 FP64, from byte offset aoff[c] of the inverse area; within a chunk, row r = VEC g + q of the
// lane group g is at entry (q * 64 + g % 64) * BS of the chunk's type.
struct BJDesc {
  const void* inv;
  const int* idx;
  int mode;
  const int* tag;
  const long long* aoff;
};

template <typename S>
struct BJ {
  const S* __restrict__ inv;
  const int* __restrict__ idx;
  int mode;
  const int* __restrict__ tag;
  const long long* __restrict__ aoff;
};

template <typename S>
__host__ __device__ inline BJ<S> bj_typed(const BJDesc& d) {
  return BJ<S>{(const S*)d.inv, d.idx, d.mode, d.tag, d.aoff};
}

// One row of an adaptive-precision inverse, converted to the compute type (tag 0 FP8 E4M3,
// 1 FP16, 2 FP32, 3 FP64).
template <typename C, int BS>
__device__ __forceinline__ void bj_row_adaptive(const void* base, int tag, size_t ent, C (&w)[BS]) {
  if (tag == 0) {
    const unsigned char* pb = (const unsigned char*)base + ent;
    if constexpr (BS >= 4) {
#pragma unroll
      for (int q = 0; q < BS / 4; ++q) {
        const int word = *reinterpret_cast<const int*>(pb + 4 * q);
        w[4 * q + 0] = (C)__builtin_amdgcn_cvt_f32_fp8(word, 0);
        w[4 * q + 1] = (C)__builtin_amdgcn_cvt_f32_fp8(word, 1);
        w[4 * q + 2] = (C)__builtin_amdgcn_cvt_f32_fp8(word, 2);
        w[4 * q + 3] = (C)__builtin_amdgcn_cvt_f32_fp8(word, 3);
      }
    } else {
      int word = 0;
#pragma unroll
      for (int k = 0; k < BS; ++k) word |= (int)pb[k] << (8 * k);
      w[0] = (C)__builtin_amdgcn_cvt_f32_fp8(word, 0);
      if constexpr (BS > 1) w[1] = (C)__builtin_amdgcn_cvt_f32_fp8(word, 1);
    }
  } else if (tag == 1) {
    const Vec<half_t, BS> t = *reinterpret_cast<const Vec<half_t, BS>*>((const half_t*)base + ent);
#pragma unroll
    for (int k = 0; k < BS; ++k) w[k] = (C)t.v[k];
  } else if (tag == 2) {
    const Vec<float, BS> t = *reinterpret_cast<const Vec<float, BS>*>((const float*)base + ent);
#pragma unroll
    for (int k = 0; k < BS; ++k) w[k] = (C)t.v[k];
  } else {
    const Vec<double, BS> t = *reinterpret_cast<const Vec<double, BS>*>((const double*)base + ent);
#pragma unroll
    for (int k = 0; k < BS; ++k) w[k] = (C)t.v[k];
  }
}

// Offsets (in entries) of the stored inverse rows of this lane's VEC rows e .. e+VEC-1; an
// invalid lane gets offset 0 (the first stored row) so that its loads stay in bounds.
template <typename S, int VEC, int BS>
__device__ __forceinline__ void bj_offsets(const BJ<S>& dinv, int e, bool valid, size_t (&off)[VEC]) {
  if (dinv.mode == 3) {
#pragma unroll
    for (int i = 0; i < VEC; ++i) off[i] = bj_chunk<VEC>(e + i) * BS;
  } else if (dinv.mode == 0) {
#pragma unroll
    for (int i = 0; i < VEC; ++i) off[i] = (size_t)(e + i) * BS;
  } else {
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
      const int row = e + i;
      const int b = (dinv.mode == 2 || !valid) ? 0 : dinv.idx[row / BS];
      off[i] = ((size_t)b * BS + (row & (BS - 1))) * BS;
    }
  }
#pragma unroll
  for (int i = 0; i < VEC; ++i) off[i] = valid ? off[i] : 0;
}

// Row q (0 <= q < NR, lane row i0 + q) of the lane's block-Jacobi product, from its stored
// inverse row `row` and the lane's inputs r (BS <= VEC) or the block's gathered inputs rb.
template <typename C, typename S, int VEC, int BS>
__device__ __forceinline__ C bj_row_dot(const Vec<S, BS>& row, int q, const C (&r)[VEC],
                                        const C* rb) {
  C acc = C(0);
  if constexpr (BS > VEC) {
#pragma unroll
    for (int k = 0; k < BS; ++k) acc += (C)row.v[k] * rb[k];
  } else {
    const int sb = q / BS;  // block within the lane
#pragma unroll
    for (int k = 0; k < BS; ++k) acc += (C)row.v[k] * r[sb * BS + k];
  }
  return acc;
}

// The BS inputs of the block of this lane's rows when a block spans BS/VEC lanes (every lane
// of the wave must call this).
template <typename C, int VEC, int BS>
__device__ __forceinline__ void bj_gather(const C (&r)[VEC], C (&rb)[BS > VEC ? BS : 1]) {
  if constexpr (BS > VEC) {
    constexpr int LPB = BS / VEC;  // lanes per block
    const int lane = threadIdx.x & 63;
    const int base = lane & ~(LPB - 1);
#pragma unroll
    for (int k = 0; k < BS; ++k) rb[k] = __shfl(r[k % VEC], base + k / VEC);
  }
}

// Block-Jacobi rows of one lane, loaded ahead of the values they multiply.
template <typename S, int VEC, int BS>
struct BJRows {
  Vec<S, BS> row[VEC];
  bool late;  // mode 4, chunk stored in a wider type than S: rows are loaded where applied
  int tag;    // mode 4: type tag of the rows held (a narrower type's rows are kept as raw bits)
};

// Type tag of the storage type S in the adaptive layout (0 FP8 E4M3, 1 FP16, 2 FP32, 3 FP64).
template <typename S>
__host__ __device__ constexpr int bj_type_tag() {
  return sizeof(S) == 2 ? 1 : sizeof(S) == 4 ? 2 : 3;
}

// Rows of a chunk stored in a narrower type than S (W 32-bit words per row), kept as raw bits
// in the first W words of each row of S.
template <typename S, int VEC, int BS, int W>
__device__ __forceinline__ void bj_load_narrow(const char* base, int g, BJRows<S, VEC, BS>& R) {
  if constexpr (W > 0 && W * 4 <= (int)sizeof(S) * BS && (W * 4) % BS == 0) {
    constexpr int NW = (int)sizeof(S) * BS / 4;
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
      const Vec<unsigned, W> u =
          *reinterpret_cast<const Vec<unsigned, W>*>(base + ((size_t)i * 64 + (g & 63)) * (W * 4));
      Vec<unsigned, NW> full{};
#pragma unroll
      for (int k = 0; k < W; ++k) full.v[k] = u.v[k];
      R.row[i] = __builtin_bit_cast(Vec<S, BS>, full);
    }
  }
}

// The BS entries of a row held as raw bits of the narrower type of tag (0 FP8 E4M3, 1 FP16,
// 2 FP32), converted to the compute type.
template <typename C, typename S, int BS>
__device__ __forceinline__ void bj_decode_narrow(const Vec<S, BS>& row, int tag, C (&w)[BS]) {
  constexpr int NW = (int)sizeof(S) * BS / 4;
#pragma unroll
  for (int k = 0; k < BS; ++k) w[k] = C(0);
  if constexpr (NW == 0 || (int)sizeof(S) * BS % 4 != 0) {
    return;  // no narrower row fits (never loaded as such)
  } else {
    const Vec<unsigned, NW> u = __builtin_bit_cast(Vec<unsigned, NW>, row);
    if (tag == 0) {
      if constexpr (BS % 4 == 0 && BS / 4 <= NW) {
#pragma unroll
        for (int q = 0; q < BS / 4; ++q) {
          w[4 * q + 0] = (C)__builtin_amdgcn_cvt_f32_fp8((int)u.v[q], 0);
          w[4 * q + 1] = (C)__builtin_amdgcn_cvt_f32_fp8((int)u.v[q], 1);
          w[4 * q + 2] = (C)__builtin_amdgcn_cvt_f32_fp8((int)u.v[q], 2);
          w[4 * q + 3] = (C)__builtin_amdgcn_cvt_f32_fp8((int)u.v[q], 3);
        }
      }
    } else if (tag == 1) {
      if constexpr (BS % 2 == 0 && BS / 2 <= NW) {
#pragma unroll
        for (int q = 0; q < BS / 2; ++q) {
          const Vec<half_t, 2> h = __builtin_bit_cast(Vec<half_t, 2>, u.v[q]);
          w[2 * q + 0] = (C)h.v[0];
          w[2 * q + 1] = (C)h.v[1];
        }
      }
    } else {
      if constexpr (BS <= NW) {
#pragma unroll
        for (int k = 0; k < BS; ++k) w[k] = (C)__builtin_bit_cast(float, u.v[k]);
      }
    }
  }
}

// AD = 1: the adaptive-precision layout (mode 4) is possible; kernels are instantiated apart for
// it, so that its conversions cost the other layouts no registers.
template <typename S, int VEC, int BS, int AD = 0>
__device__ __forceinline__ void bj_load(const BJ<S>& dinv, int e, bool valid, BJRows<S, VEC, BS>& R) {
  R.late = false;
  if (AD && dinv.mode == 4) {
    // adaptive precision: a chunk stored in the storage type or a narrower one is loaded here
    // (a narrower row's bits fill the first bytes of a row of S); a wider one where the rows are
    // applied
    constexpr int TS = bj_type_tag<S>();
    const int g = valid ? e / VEC : 0;
    const int ch = g >> 6;
    const int tag = dinv.tag[ch];
    R.tag = tag;
    const char* base = (const char*)dinv.inv + dinv.aoff[ch];
    if (tag == TS) {
#pragma unroll
      for (int i = 0; i < VEC; ++i)
        R.row[i] = *reinterpret_cast<const Vec<S, BS>*>((const S*)base +
                                                         ((size_t)i * 64 + (g & 63)) * BS);
    } else if (tag == 0 && TS > 0 && BS % 4 == 0) {
      bj_load_narrow<S, VEC, BS, BS / 4>(base, g, R);
    } else if (tag == 1 && TS > 1 && BS % 2 == 0) {
      bj_load_narrow<S, VEC, BS, BS / 2>(base, g, R);
    } else if (tag == 2 && TS > 2) {
      bj_load_narrow<S, VEC, BS, BS>(base, g, R);
    } else {
      R.late = true;
    }
    return;
  }
  size_t off[VEC];
  bj_offsets<S, VEC, BS>(dinv, e, valid, off);
#pragma unroll
  for (int i = 0; i < VEC; ++i) R.row[i] = *reinterpret_cast<const Vec<S, BS>*>(dinv.inv + off[i]);
}

// z = D^{-1} r with rows loaded by bj_load, or (mode 4) loaded here (every lane of the wave
// must call this).
template <typename C, typename S, int VEC, int BS>
__device__ __forceinline__ void bj_mul(const BJRows<S, VEC, BS>& R, bool valid, const C (&r)[VEC],
                                       C (&z)[VEC]);
template <typename C, typename S, int VEC, int BS, int AD = 0>
__device__ __forceinline__ void bj_apply_lane(const BJ<S>& dinv, int e, bool valid,
                                              const C (&r)[VEC], C (&z)[VEC]);
template <typename C, typename S, int VEC, int BS, int AD = 0>
__device__ __forceinline__ void bj_mul(const BJ<S>& dinv, int e, const BJRows<S, VEC, BS>& R,
                                       bool valid, const C (&r)[VEC], C (&z)[VEC]) {
  if (AD && dinv.mode == 4 && R.late) {
    bj_apply_lane<C, S, VEC, BS, AD>(dinv, e, valid, r, z);
  } else if (AD && dinv.mode == 4 && R.tag != bj_type_tag<S>()) {
    C rb[BS > VEC ? BS : 1];
    bj_gather<C, VEC, BS>(r, rb);
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      C w[BS];
      bj_decode_narrow<C, S, BS>(R.row[q], R.tag, w);
      C acc = C(0);
      if constexpr (BS > VEC) {
#pragma unroll
        for (int k = 0; k < BS; ++k) acc += w[k] * rb[k];
      } else {
        const int sb = q / BS;
#pragma unroll
        for (int k = 0; k < BS; ++k) acc += w[k] * r[sb * BS + k];
      }
      z[q] = valid ? acc : C(0);
    }
  } else {
    bj_mul<C, S, VEC, BS>(R, valid, r, z);
  }
}

template <typename C, typename S, int VEC, int BS>
__device__ __forceinline__ void bj_mul(const BJRows<S, VEC, BS>& R, bool valid, const C (&r)[VEC],
                                       C (&z)[VEC]) {
  C rb[BS > VEC ? BS : 1];
  bj_gather<C, VEC, BS>(r, rb);
#pragma unroll
  for (int q = 0; q < VEC; ++q) {
    const C acc = bj_row_dot<C, S, VEC, BS>(R.row[q], q, r, rb);
    z[q] = valid ? acc : C(0);
  }
}

// Block-Jacobi: z = D^{-1} r for the VEC rows of this lane (rows e .. e+VEC-1).  Blocks of BS
// rows; when BS > VEC a block spans BS/VEC consecutive lanes whose values are exchanged by
// shuffles (every lane of the wave must call this).  Inverse rows are loaded without branches,
// RCH rows in flight at a time.  Mode 4 reads each row in its chunk's type.
template <typename C, typename S, int VEC, int BS, int AD>
__device__ __forceinline__ void bj_apply_lane(const BJ<S>& dinv, int e, bool valid,
                                              const C (&r)[VEC], C (&z)[VEC]) {
  C rb[BS > VEC ? BS : 1];
  bj_gather<C, VEC, BS>(r, rb);
  if (AD && dinv.mode == 4) {
    const int g = valid ? e / VEC : 0;  // an invalid lane reads chunk 0 and discards the result
    const int ch = g >> 6;
    const int tag = dinv.tag[ch];
    const void* base = (const char*)dinv.inv + dinv.aoff[ch];
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      C w[BS];
      bj_row_adaptive<C, BS>(base, tag, ((size_t)q * 64 + (g & 63)) * BS, w);
      C acc = C(0);
      if constexpr (BS > VEC) {
#pragma unroll
        for (int k = 0; k < BS; ++k) acc += w[k] * rb[k];
      } else {
        const int sb = q / BS;
#pragma unroll
        for (int k = 0; k < BS; ++k) acc += w[k] * r[sb * BS + k];
      }
      z[q] = valid ? acc : C(0);
    }
    return;
  }
  size_t off[VEC];
  bj_offsets<S, VEC, BS>(dinv, e, valid, off);
  constexpr int RCH = VEC < 4 ? VEC : 4;
#pragma unroll
  for (int i0 = 0; i0 < VEC; i0 += RCH) {
    Vec<S, BS> row[RCH];
#pragma unroll
    for (int i = 0; i < RCH; ++i) row[i] = *reinterpret_cast<const Vec<S, BS>*>(dinv.inv + off[i0 + i]);
#pragma unroll
    for (int i = 0; i < RCH; ++i) {
      const C acc = bj_row_dot<C, S, VEC, BS>(row[i], i0 + i, r, rb);
      z[i0 + i] = valid ? acc : C(0);
    }
  }
}

}  // namespace mprk

// batch.hip -- batched form of include/mprk.h: many independent heat / advection-diffusion
// problems of uneven size advanced together, one persistent kernel launch per RK stage.
//
// Each problem owns a contiguous group of workgroups (its "CTA group").  Inside the stage
// kernel a group runs the whole implicit stage on its own: stage right-hand side (FP64),
// the FP64 residual loop, and preconditioned CG in the LP storage type, with group barriers
// between phases and group reductions (per-workgroup partials, double-buffered, summed in fixed
// order by every workgroup of the group, so all workgroups take identical decisions).  The
// last stage ends with the FP64 step combination.  One step = s launches, captured once as a
// hipGraph and replayed.  All workgroups of the launch must be co-resident: the grid is sized
// from the occupancy query, and every barrier wait is bounded (a timeout raises an error flag
// and the kernel still runs to its end).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mprk.h"
#include "runtime_internal.hpp"

using namespace mprk;

namespace mprk {

constexpr int BND = 4;            // values per group reduction
constexpr long BAR_SPIN_LIMIT = 1L << 22;

struct BCtl {
  unsigned int bar_count;
  unsigned int bar_gen;
  int error;                     // a group barrier timed out
  int step_nonfinite;
  long long good_steps, bad_steps, life_iters, life_passes;
  int iters[MAXS], passes[MAXS], converged[MAXS], nonfinite[MAXS];
  double resid[MAXS];
};

struct BProb {
  Geo geo;
  Coef<double> K;                // FP64 operator
  double sigma;                  // dt * a_ii (single distinct diagonal)
  double dt;
  double *u, *rhs, *y, *res, *k; // FP64; k holds s vectors of stride N
  void *r, *z, *p0, *p1, *q, *x; // LP vectors
  void* dinv;                    // block-Jacobi inverses (LP)
  double* part;                  // 2 * BND * nwg partials
  BCtl* ctl;
  int wg0, nwg, chunk;           // workgroup range and rows per workgroup (multiple of 64)
};

struct BArgs {
  const BProb* probs;
  const int* wg2prob;
  int s;
  double A[MAXS][MAXS];          // full tableau (a_hi + a_lo)
  double b[MAXS];
  double rtol, atol, outer_tol;
  int maxit, max_passes, paper_mode, bs;
  int outer_stop;  // inner solves also stop at the outer target (as SolveCfg::outer_stop)
  // start values of the stage solves: y = rhs + sigma (ya[i] k_{i-1} + yb[i] k_{yj[i]}) for a
  // stage i > 0; the first stage y = rhs + sigma y0f f(u) when feval, f(u) also kept in the
  // last stage's slope slot until the second stage reads it when fkeep
  double ya[MAXS], yb[MAXS], y0f;
  int yj[MAXS];
  int feval, fkeep;
};

// Data one workgroup writes and another reads inside a stage launch (the stencil inputs y, p
// and z, and the reduction partials) are written with device-scope stores, which are coherent
// across the XCDs once complete.  A barrier therefore needs no L2 writeback: every wave waits
// for its own stores to complete before its workgroup arrives, and after the barrier every wave
// invalidates its non-coherent cached lines (agent-scope acquire) before reading other
// workgroups' rows.  Data a thread writes and only the same thread reads back (its own rows of
// r, x, q, res, rhs, k) stay plain stores.
template <typename T>
__device__ __forceinline__ void store_shared(T* p, T v) {
  if constexpr (sizeof(T) == 2) {
    unsigned short b;
    __builtin_memcpy(&b, &v, 2);
    __hip_atomic_store(reinterpret_cast<unsigned short*>(p), b, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  } else {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ __forceinline__ void wait_own_stores() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ unsigned int load_u32_dev(const unsigned int* p) {
  return __hip_atomic_load(const_cast<unsigned int*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier over the nwg workgroups of one problem (generation counter; bounded spin).
__device__ bool group_barrier(BCtl* c, int nwg) {
  if (nwg > 1) wait_own_stores();
  __syncthreads();
  if (nwg > 1) {
    if (threadIdx.x == 0) {
      // the generation is read (and the read completed) before this arrival is counted
      const unsigned gen = load_u32_dev(&c->bar_gen);
      wait_own_stores();
      const unsigned arrived = __hip_atomic_fetch_add(&c->bar_count, 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
      if (arrived == (unsigned)nwg - 1u) {
        __hip_atomic_store(&c->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wait_own_stores();  // the reset is visible before the next generation opens
        __hip_atomic_fetch_add(&c->bar_gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        long spins = 0;
        while (load_u32_dev(&c->bar_gen) == gen) {
          __builtin_amdgcn_s_sleep(2);
          if (++spins > BAR_SPIN_LIMIT) {
            __hip_atomic_store(&c->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
        }
      }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  return true;
}

// Group reduction of nd values; every workgroup of the group returns the same totals.  Each
// workgroup publishes its partials (device-scope stores), passes the group barrier, then sums
// all the group's partials itself in workgroup order (every thread a strided slice, fixed
// shuffle tree and wave order), so all workgroups take identical decisions without a second
// round trip.  Partials are double-buffered by `parity` (a fast workgroup may publish the next
// reduction's partials while a slow one still reads these).
template <int ND>
__device__ void group_reduce(const double (&v)[ND], int nd, const BProb& P, int wl, int& parity,
                             double (&out)[ND]) {
  __shared__ double wsum[NWAVE][BND];
  __shared__ double tot[BND];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    if (d < nd) {
      const double s = wave_sum(v[d]);
      if (lane == 0) wsum[wave][d] = s;
    }
  }
  __syncthreads();
  const int nwg = P.nwg;
  double* part = P.part + (size_t)parity * BND * nwg;
  if (threadIdx.x < nd) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) s += wsum[w][threadIdx.x];
    if (nwg > 1) store_dev(part + (size_t)threadIdx.x * nwg + wl, s);
    else tot[threadIdx.x] = s;
  }
  if (nwg > 1) {
    group_barrier(P.ctl, nwg);
    __shared__ double wt[NWAVE][BND];
#pragma unroll 1
    for (int d = 0; d < nd; ++d) {
      double s = 0.0;
#pragma unroll 1
      for (int w = threadIdx.x; w < nwg; w += TPB) s += load_dev(part + (size_t)d * nwg + w);
      s = wave_sum(s);
      if (lane == 0) wt[wave][d] = s;
    }
    __syncthreads();
    if (threadIdx.x < nd) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < NWAVE; ++w) s += wt[w][threadIdx.x];
      tot[threadIdx.x] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < ND; ++d) out[d] = d < nd ? tot[d] : 0.0;
  __syncthreads();
  parity ^= 1;
}

// one FP64 stencil row of K
__device__ __forceinline__ double k64_row(const Geo& geo, const Coef<double>& K,
                                          const double* __restrict__ y, int r, double& yc) {
  In1<double, double, 1> f{y};
  double c[1], o[1];
  stencil_group<double, 1>(geo, K, r, f, c, o);
  yc = c[0];
  return o[0];
}

// Rows it0 .. it0+RU-1 of this thread in [r0, r1) (nit rows per thread); a row past the end is
// replaced by r0 (a valid row) and flagged invalid.  RU rows are handled together by a thread
// in the CG phases, their loads issued together (RU = 1, 2 or 4, picked by the autotuner).
template <int RU>
__device__ __forceinline__ void rows_of(int r0, int r1, int nit, int it0, int (&row)[RU],
                                        bool (&val)[RU]) {
#pragma unroll
  for (int k = 0; k < RU; ++k) {
    const int rr = r0 + (it0 + k) * TPB + (int)threadIdx.x;
    val[k] = it0 + k < nit && rr < r1;
    row[k] = val[k] ? rr : r0;
  }
}

// Minimum waves per SIMD the compiler must allow (register budget) for each row unroll.
template <typename S, int RU>
constexpr int kb_min_waves() {
  return sizeof(S) == 8 ? (RU == 1 ? 4 : RU == 2 ? 3 : 2) : (RU == 1 ? 6 : RU == 2 ? 5 : 3);
}

template <typename S, typename C, int BS, int RU>
__global__ __launch_bounds__(TPB, (kb_min_waves<S, RU>())) void kb_stage(BArgs a, int stage) {
  const int pid = a.wg2prob[blockIdx.x];
  const BProb P = a.probs[pid];
  BCtl* ctl = P.ctl;
  const int wl = blockIdx.x - P.wg0;
  const int N = P.geo.N;
  const int r0 = wl * P.chunk;
  const int r1 = min(N, r0 + P.chunk);
  const int nit = (P.chunk + TPB - 1) / TPB;
  int parity = 0;
  const double sigma = P.sigma;
  const double sqrtN = sqrt((double)N);
  double* kout = P.k + (size_t)stage * N;
  const BJ<S> dinv{(const S*)P.dinv, nullptr, 0};
  S* r = (S*)P.r;
  S* z = BS > 0 ? (S*)P.z : (S*)P.r;
  S* q = (S*)P.q;
  S* x = (S*)P.x;
  const Coef<C> M = coef_cast<C>(coef_stage(P.K, sigma));

  if (stage == 0 && wl == 0 && threadIdx.x == 0)
    __hip_atomic_store(&ctl->step_nonfinite, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // ---- stage right-hand side: rhs = u + dt sum_{j<stage} a_ij k_j ; y = its start value ----
  for (int it = 0; it < nit; ++it) {
    const int row = r0 + it * TPB + threadIdx.x;
    if (row >= r1) break;
    double acc = P.u[row];
    for (int j = 0; j < stage; ++j) acc += P.dt * a.A[stage][j] * P.k[(size_t)j * N + row];
    P.rhs[row] = acc;
    double yv = acc;
    if (stage == 0 && a.feval) {
      double uc;
      const double fu = k64_row(P.geo, P.K, P.u, row, uc);
      yv += sigma * a.y0f * fu;
      if (a.fkeep) P.k[(size_t)(a.s - 1) * N + row] = fu;
    } else if (stage > 0) {
      yv += sigma * a.ya[stage] * P.k[(size_t)(stage - 1) * N + row];
      if (a.yb[stage] != 0.0) yv += sigma * a.yb[stage] * P.k[(size_t)a.yj[stage] * N + row];
    }
    store_shared(P.y + row, yv);
  }
  group_barrier(ctl, P.nwg);

  int passes = 0, total_iters = 0, converged = 0, nonfinite = 0;
  bool last_conv = false;  // the last LP solve stopped on its own tolerance
  double rel = 0.0;
  const int P_max = a.paper_mode ? 1 : a.max_passes;
  for (int pass = 0;; ++pass) {
    // ---- FP64 stage residual: k = K y ; res = rhs - y + sigma k ----
    double acc[BND] = {0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < nit; ++it) {
      const int row = r0 + it * TPB + threadIdx.x;
      if (row >= r1) break;
      double yc;
      const double ky = k64_row(P.geo, P.K, P.y, row, yc);
      const double b = P.rhs[row];
      const double rr = b - yc + sigma * ky;
      kout[row] = ky;
      P.res[row] = rr;
      acc[0] += rr * rr;
      acc[1] += b * b;
      acc[2] += (__builtin_isfinite(rr) && __builtin_isfinite(ky)) ? 0.0 : 1.0;
    }
    double t[BND];
    group_reduce<BND>(acc, 3, P, wl, parity, t);
    const double rn = sqrt(t[0]), bn = sqrt(t[1]);
    rel = bn > 0.0 ? rn / bn : rn;
    if (t[2] != 0.0 || !__builtin_isfinite(rn)) {
      nonfinite = 1;
      break;
    }
    converged = a.paper_mode ? (passes >= 1 && last_conv) : (rel <= a.outer_tol);
    if (converged || passes >= P_max || rn == 0.0) break;
    const double scale = rn / sqrtN;
    const double inv = 1.0 / scale;
    // ---- CG begin: r = LP(res / scale), z = BJ(r) ----
    double acc2[BND] = {0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < nit; ++it) {
      const int row = r0 + it * TPB + threadIdx.x;
      const bool valid = row < r1;
      C rv[1], zv[1];
      rv[0] = valid ? rnd<S, C>((C)(P.res[row] * inv)) : C(0);
      if constexpr (BS > 0) {
        bj_apply_lane<C, S, 1, BS>(dinv, row, valid, rv, zv);
        zv[0] = rnd<S, C>(zv[0]);
      } else {
        zv[0] = rv[0];
      }
      if (valid) {
        if constexpr (BS > 0) {
          r[row] = (S)rv[0];
          store_shared(z + row, (S)zv[0]);
        } else {
          store_shared(r + row, (S)rv[0]);  // z aliases r
        }
        acc2[0] += (double)(rv[0] * zv[0]);
        acc2[1] += (double)(rv[0] * rv[0]);
      }
    }
    group_reduce<BND>(acc2, 2, P, wl, parity, t);
    double rz = t[0];
    // (the outer target as for a single problem: the 2-norm of the LP residual, unit = scale)
    const double tol = fmax(fmax(a.rtol * sqrt(t[1]), a.atol / scale),
                            a.outer_stop ? 0.5 * a.outer_tol * bn / scale : 0.0);
    bool inner_done = sqrt(t[1]) <= tol;
    bool inner_conv = inner_done;
    double beta = 0.0;
    int its = 0;
    while (!inner_done && its < a.maxit) {
      // ---- C1: p_new = z + beta p_old ; q = M p_new ; (p, q) ----
      const S* pold = (its & 1) ? (const S*)P.p1 : (const S*)P.p0;
      S* pnew = (its & 1) ? (S*)P.p0 : (S*)P.p1;
      InAxpy<C, S, 1> f{z, pold, (C)beta, its > 0};
      double acc3[BND] = {0.0, 0.0, 0.0, 0.0};
      for (int it0 = 0; it0 < nit; it0 += RU) {
        int row[RU];
        bool val[RU];
        rows_of<RU>(r0, r1, nit, it0, row, val);
        C pc[RU][1], w[RU][1];
#pragma unroll
        for (int k = 0; k < RU; ++k) stencil_group<C, 1>(P.geo, M, row[k], f, pc[k], w[k]);
#pragma unroll
        for (int k = 0; k < RU; ++k) {
          if (val[k]) {
            w[k][0] = rnd<S, C>(w[k][0]);
            store_shared(pnew + row[k], (S)pc[k][0]);
            q[row[k]] = (S)w[k][0];
            acc3[0] += (double)(pc[k][0] * w[k][0]);
          }
        }
      }
      group_reduce<BND>(acc3, 1, P, wl, parity, t);
      const double pq = t[0];
      if (!(pq > 0.0) || !__builtin_isfinite(pq)) {
        inner_conv = false;
        break;
      }
      const C alpha = (C)(rz / pq);
      // ---- C2: x += alpha p ; r -= alpha q ; z = BJ(r) ; (r, z), (r, r) ----
      double acc4[BND] = {0.0, 0.0, 0.0, 0.0};
      for (int it0 = 0; it0 < nit; it0 += RU) {
        int row[RU];
        bool val[RU];
        rows_of<RU>(r0, r1, nit, it0, row, val);
        // every load of the RU rows first (x is read but unused in the first iteration)
        C pv[RU], xo[RU], ro[RU], qo[RU];
        BJRows<S, 1, BS == 0 ? 1 : BS> R[RU];
#pragma unroll
        for (int k = 0; k < RU; ++k) {
          pv[k] = (C)pnew[row[k]];
          xo[k] = (C)x[row[k]];
          ro[k] = (C)r[row[k]];
          qo[k] = (C)q[row[k]];
          if constexpr (BS > 0) bj_load<S, 1, BS>(dinv, row[k], val[k], R[k]);
        }
#pragma unroll
        for (int k = 0; k < RU; ++k) {
          C rv[1], zv[1];
          const C xv = its == 0 ? alpha * pv[k] : xo[k] + alpha * pv[k];
          rv[0] = val[k] ? rnd<S, C>(ro[k] - alpha * qo[k]) : C(0);
          if (val[k]) {
            x[row[k]] = (S)xv;
            if constexpr (BS > 0) r[row[k]] = (S)rv[0];
            else store_shared(r + row[k], (S)rv[0]);  // z aliases r
          }
          if constexpr (BS > 0) {
            bj_mul<C, S, 1, BS>(R[k], val[k], rv, zv);
            zv[0] = rnd<S, C>(zv[0]);
            if (val[k]) store_shared(z + row[k], (S)zv[0]);
          } else {
            zv[0] = rv[0];
          }
          if (val[k]) {
            acc4[0] += (double)(rv[0] * zv[0]);
            acc4[1] += (double)(rv[0] * rv[0]);
          }
        }
      }
      group_reduce<BND>(acc4, 2, P, wl, parity, t);
      ++its;
      const double rz_new = t[0];
      beta = rz_new / rz;
      rz = rz_new;
      inner_conv = __builtin_isfinite(t[1]) && sqrt(t[1]) <= tol;
      inner_done = !__builtin_isfinite(t[1]) || inner_conv;
    }
    last_conv = inner_conv;
    total_iters += its;
    // ---- promote: y += scale * x ----
    if (its > 0) {
      for (int it = 0; it < nit; ++it) {
        const int row = r0 + it * TPB + threadIdx.x;
        if (row >= r1) break;
        store_shared(P.y + row, P.y[row] + scale * (double)(C)x[row]);
      }
    }
    ++passes;
    group_barrier(ctl, P.nwg);
  }
  if (wl == 0 && threadIdx.x == 0) {
    ctl->iters[stage] = total_iters;
    ctl->passes[stage] = passes;
    ctl->resid[stage] = rel;
    ctl->converged[stage] = converged && !nonfinite;
    ctl->nonfinite[stage] = nonfinite;
    ctl->life_iters += total_iters;
    ctl->life_passes += passes;
    if (nonfinite) __hip_atomic_store(&ctl->step_nonfinite, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (stage == a.s - 1) {
    // ---- step combination u += dt sum_i b_i k_i (skipped after a non-finite residual) ----
    group_barrier(ctl, P.nwg);
    const int bad = __hip_atomic_load(&ctl->step_nonfinite, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!bad) {
      for (int it = 0; it < nit; ++it) {
        const int row = r0 + it * TPB + threadIdx.x;
        if (row >= r1) break;
        double acc = P.u[row];
        for (int i = 0; i < a.s; ++i) acc += P.dt * a.b[i] * P.k[(size_t)i * N + row];
        P.u[row] = acc;
      }
    }
    if (wl == 0 && threadIdx.x == 0) {
      if (bad) ctl->bad_steps += 1;
      else ctl->good_steps += 1;
    }
  }
}

}  // namespace mprk

// ------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------

struct mprk_batch {
  int count = 0;
  std::vector<mprk_problem> probs;
  mprk_tableau tab{};
  mprk_precisions prec{};
  hipStream_t stream = nullptr;
  int lp_bytes = 4;
  int bs = 0;
  std::vector<size_t> off_r, off_dinv, off_part, off_k, off_rhs;
  std::vector<int> N, nwg, chunk;
  size_t o_probs = 0, o_map = 0, o_ctl = 0, o_flag = 0, ws_bytes = 0;
  size_t lp_vec_bytes_total = 0;
  int G = 0;
  char* ws = nullptr;
  std::vector<double*> u;
  bool bound = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  long long good_base = 0;
  std::vector<long long> good_seen, bad_seen;
  std::vector<int> fixed_wg;  // caller-chosen workgroups per problem (empty: planned)
  double weight_exp = 0.5;    // exponent of the condition-number estimate in the work model
  // measured work model (autotuner): per problem, unknowns x (CG iterations + 1.6 x outer passes)
  // of the last step; used by plan_groups while use_measured is set
  std::vector<double> measured_w;
  bool use_measured = false;
  int ru = 2;                 // rows a thread handles together in the CG phases (1, 2, 4)
  int capacity = 0;           // co-resident workgroups of the device for the kernel in use
  int max_capacity = 0;       // largest capacity over the kernel variants (sizes the map)
  ~mprk_batch() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace mprk {
Coef<double> operator_coef(const mprk_grid& g, const mprk_operator& op);
}

template <typename S, typename C, int RU>
static const void* kb_kernel_ptr(int bs) {
  switch (bs) {
    case 0: return (const void*)kb_stage<S, C, 0, RU>;
    case 1: return (const void*)kb_stage<S, C, 1, RU>;
    case 2: return (const void*)kb_stage<S, C, 2, RU>;
    case 4: return (const void*)kb_stage<S, C, 4, RU>;
    default: return (const void*)kb_stage<S, C, 8, RU>;
  }
}

template <typename S, typename C>
static const void* kb_kernel_ru(int bs, int ru) {
  if (ru == 4) return kb_kernel_ptr<S, C, 4>(bs);
  if (ru == 2) return kb_kernel_ptr<S, C, 2>(bs);
  return kb_kernel_ptr<S, C, 1>(bs);
}

static const void* batch_kernel(int storage, int bs, int ru) {
  if (storage == MPRK_FP64) return kb_kernel_ru<double, double>(bs, ru);
  if (storage == MPRK_FP32) return kb_kernel_ru<float, float>(bs, ru);
  return kb_kernel_ru<half_t, float>(bs, ru);
}

// Weight of a problem's stage solve: unknowns x an estimate of CG iterations, which grow
// like a power e of the stage matrix's condition number 1 + sigma * 4 * diff * sum 1/h^2
// (e = 1/2 for unpreconditioned CG; the autotuner tries others).
static double work_weight(const mprk_problem& p, double a, double e) {
  const mprk_grid& g = p.grid;
  const double N = (double)g.nx * g.ny * g.nz;
  double s = 0.0;
  const int n[3] = {g.nx, g.ny, g.nz};
  for (int d = 0; d < 3; ++d) {
    const double h = g.bc == MPRK_BC_DIRICHLET0 ? 1.0 / (n[d] + 1) : 1.0 / n[d];
    s += 4.0 * p.op.diff / (h * h);
  }
  return N * std::pow(1.0 + p.dt * a * s, e);
}

extern "C" int32_t mprk_batch_create(int32_t count, const mprk_problem* problems,
                                     const mprk_tableau* tab, const mprk_precisions* prec,
                                     void* hip_stream, mprk_batch** out) {
  if (!out) return set_error(MPRK_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 1 || !problems || !tab || !prec) return set_error(MPRK_EINVAL, "bad batch arguments");
  if (prec->krylov != MPRK_CG) return set_error(MPRK_EUNSUPPORTED, "batched form implements CG only");
  if (prec->storage == MPRK_FP64 && prec->compute != MPRK_FP64)
    return set_error(MPRK_EUNSUPPORTED, "FP64 storage needs FP64 compute");
  if (prec->storage != MPRK_FP64 && prec->compute != MPRK_FP32)
    return set_error(MPRK_EUNSUPPORTED, "LP storage needs FP32 compute");
  if (prec->reorth) return set_error(MPRK_EUNSUPPORTED, "reorth is a GMRES option");
  if (prec->bj_adapt_tol > 0.0)
    return set_error(MPRK_EUNSUPPORTED, "batched form keeps block-Jacobi inverses in the storage type");
  if (prec->precond == MPRK_PRECOND_FDM)
    return set_error(MPRK_EUNSUPPORTED, "batched form implements block-Jacobi or no preconditioner");
  if (prec->stage_start < MPRK_START_AUTO || prec->stage_start > MPRK_START_EXTRAP)
    return set_error(MPRK_EINVAL, "stage_start must be one of the MPRK_START values");
  if (prec->inner_stop < MPRK_STOP_AUTO || prec->inner_stop > MPRK_STOP_RTOL)
    return set_error(MPRK_EINVAL, "inner_stop must be one of the MPRK_STOP values");
  // one distinct nonzero diagonal, no eps off-diagonals needing k^eps, all stages implicit
  double diag = 0.0;
  for (int i = 0; i < tab->s; ++i) {
    const double aii = tab->a_hi[i * tab->s + i] + tab->a_lo[i * tab->s + i];
    if (aii == 0.0) return set_error(MPRK_EUNSUPPORTED, "batched form needs every stage implicit");
    if (i == 0) diag = aii;
    else if (aii != diag) return set_error(MPRK_EUNSUPPORTED, "batched form needs a single diagonal value (SDIRK)");
    for (int j = 0; j < i; ++j)
      if (tab->a_lo[i * tab->s + j] != 0.0)
        return set_error(MPRK_EUNSUPPORTED, "batched form does not implement eps off-diagonals");
  }
  mprk_batch* b = new (std::nothrow) mprk_batch();
  if (!b) return set_error(MPRK_ENOMEM, "host allocation failed");
  b->count = count;
  b->probs.assign(problems, problems + count);
  b->tab = *tab;
  b->prec = *prec;
  b->stream = (hipStream_t)hip_stream;
  for (int p = 0; p < count; ++p) {
    const mprk_problem& q = problems[p];
    if (q.op.format != MPRK_FMT_STENCIL) {
      delete b;
      return set_error(MPRK_EUNSUPPORTED, "batched form uses the matrix-free stencil");
    }
    if (q.op.kind != MPRK_OP_HEAT && q.op.kind != MPRK_OP_ADVDIFF && q.op.kind != MPRK_OP_CENTRAL) {
      delete b;
      return set_error(MPRK_EINVAL, "bad operator kind");
    }
    if (q.op.kind != MPRK_OP_HEAT && (q.op.b[0] != 0.0 || q.op.b[1] != 0.0 || q.op.b[2] != 0.0)) {
      delete b;
      return set_error(MPRK_EINVAL, "CG needs a symmetric operator");
    }
    if (q.grid.nx < 1 || q.grid.ny < 1 || q.grid.nz < 1 || !(q.dt > 0.0) || !(q.op.diff >= 0.0)) {
      delete b;
      return set_error(MPRK_EINVAL, "bad problem in batch");
    }
  }
  b->lp_bytes = prec->storage == MPRK_FP64 ? 8 : (prec->storage == MPRK_FP32 ? 4 : 2);
  b->bs = prec->precond == MPRK_PRECOND_BJ ? prec->block : 0;
  if (b->bs && !(b->bs == 1 || b->bs == 2 || b->bs == 4 || b->bs == 8)) {
    delete b;
    return set_error(MPRK_EINVAL, "block size must be 1, 2, 4 or 8");
  }
  *out = b;
  return MPRK_OK;
}

// Workgroups per problem: proportional to the work estimate, at least one, at most one per
// 64 rows, in total at most the co-resident capacity of the device.
static int plan_groups(mprk_batch* b, int capacity) {
  const int s = b->tab.s;
  const double a = b->tab.a_hi[0] + b->tab.a_lo[0];
  std::vector<double> w(b->count);
  double W = 0.0;
  for (int p = 0; p < b->count; ++p) {
    w[p] = (b->use_measured && (int)b->measured_w.size() == b->count)
               ? b->measured_w[p]
               : work_weight(b->probs[p], a, b->weight_exp);
    W += w[p];
  }
  (void)s;
  b->nwg.assign(b->count, 1);
  b->chunk.assign(b->count, 0);
  b->N.assign(b->count, 0);
  int avail = capacity - b->count;
  if (avail < 0) return set_error(MPRK_EUNSUPPORTED, "more problems than co-resident workgroups");
  int fixed_total = 0;
  for (int p = 0; p < b->count; ++p) {
    const mprk_grid& g = b->probs[p].grid;
    const int N = g.nx * g.ny * g.nz;
    b->N[p] = N;
    const int maxwg = std::max(1, (N + 63) / 64);
    if (!b->fixed_wg.empty()) {
      b->nwg[p] = std::min(maxwg, std::max(1, b->fixed_wg[p]));
      fixed_total += b->nwg[p];
      continue;
    }
    int extra = (int)std::floor(avail * w[p] / W);
    b->nwg[p] = std::min(maxwg, 1 + extra);
  }
  if (fixed_total > capacity) return set_error(MPRK_EINVAL, "schedule exceeds co-resident workgroups");
  int G = 0;
  for (int p = 0; p < b->count; ++p) {
    const int N = b->N[p];
    int ch = (N + b->nwg[p] - 1) / b->nwg[p];
    ch = (ch + 63) / 64 * 64;  // block-Jacobi blocks (<= 8 rows) never straddle workgroups
    b->chunk[p] = ch;
    b->nwg[p] = (N + ch - 1) / ch;
    G += b->nwg[p];
  }
  b->G = G;
  return MPRK_OK;
}

static int batch_layout(mprk_batch* b) {
  const int s = b->tab.s;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  b->off_rhs.resize(b->count);
  b->off_k.resize(b->count);
  b->off_r.resize(b->count);
  b->off_dinv.resize(b->count);
  b->off_part.resize(b->count);
  for (int p = 0; p < b->count; ++p) {
    const size_t N = (size_t)b->N[p];
    b->off_rhs[p] = take(3 * N * 8);          // rhs, y, res
    b->off_k[p] = take((size_t)s * N * 8);
    const size_t vlp = (N * b->lp_bytes + 255) & ~(size_t)255;
    b->off_r[p] = take(6 * vlp);              // r, z, p0, p1, q, x
    b->off_dinv[p] = b->bs ? take(((N + b->bs - 1) / b->bs) * (size_t)b->bs * b->bs * b->lp_bytes) : 0;
    // partials for the largest group the problem can get (one workgroup per 64 rows), so that
    // the autotuner may change the schedule after binding
    b->off_part[p] = take(2 * BND * (size_t)std::max(1, (b->N[p] + 63) / 64) * 8);
  }
  b->o_probs = take(sizeof(BProb) * b->count);
  b->o_map = take(sizeof(int) * (size_t)std::max(b->G, b->max_capacity));
  b->o_ctl = take(sizeof(BCtl) * b->count);
  b->o_flag = take(256);
  b->ws_bytes = off;
  return MPRK_OK;
}

static int batch_capacity(mprk_batch* b, int ru, int* cap) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(MPRK_EDEVICE, "hipGetDevice failed");
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return set_error(MPRK_EDEVICE, "CU count query failed");
  const void* k = batch_kernel(b->prec.storage, b->bs, ru);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, TPB, 0) != hipSuccess)
    return set_error(MPRK_EDEVICE, "occupancy query failed");
  // stay one workgroup per CU below the occupancy bound
  *cap = std::max(1, cus * std::max(1, per - 1));
  return MPRK_OK;
}

extern "C" int32_t mprk_batch_set_schedule(mprk_batch* b, const int32_t* wg_per_problem) {
  if (!b) return set_error(MPRK_EINVAL, "NULL batch");
  if (b->ws_bytes) return set_error(MPRK_ESTATE, "schedule must be set before sizing/binding");
  if (!wg_per_problem) {
    b->fixed_wg.clear();
    return MPRK_OK;
  }
  b->fixed_wg.assign(wg_per_problem, wg_per_problem + b->count);
  return MPRK_OK;
}

extern "C" int32_t mprk_batch_get_schedule(mprk_batch* b, int32_t* wg_per_problem) {
  if (!b || !wg_per_problem) return set_error(MPRK_EINVAL, "NULL argument");
  if (mprk_batch_workspace_bytes(b) < 0) return MPRK_EINVAL;
  for (int p = 0; p < b->count; ++p) wg_per_problem[p] = b->nwg[p];
  return MPRK_OK;
}

extern "C" int64_t mprk_batch_workspace_bytes(const mprk_batch* cb) {
  if (!cb) return set_error(MPRK_EINVAL, "NULL batch");
  mprk_batch* b = const_cast<mprk_batch*>(cb);
  if (b->ws_bytes == 0) {
    int cap = 0, mx = 0;
    for (int ru : {1, 2, 4}) {
      int rc = batch_capacity(b, ru, &cap);
      if (rc) return rc;
      mx = std::max(mx, cap);
    }
    b->max_capacity = mx;
    int rc = batch_capacity(b, b->ru, &cap);
    if (rc) return rc;
    b->capacity = cap;
    rc = plan_groups(b, cap);
    if (rc) return rc;
    rc = batch_layout(b);
    if (rc) return rc;
  }
  return (int64_t)b->ws_bytes;
}

#define BHIP(x)                                                                        \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      return set_error(MPRK_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));  \
  } while (0)

static BArgs batch_args(mprk_batch* b) {
  BArgs a{};
  a.probs = (const BProb*)(b->ws + b->o_probs);
  a.wg2prob = (const int*)(b->ws + b->o_map);
  a.s = b->tab.s;
  for (int i = 0; i < a.s; ++i) {
    for (int j = 0; j < a.s; ++j) a.A[i][j] = b->tab.a_hi[i * a.s + j] + b->tab.a_lo[i * a.s + j];
    a.b[i] = b->tab.b[i];
  }
  a.rtol = b->prec.rtol;
  a.atol = b->prec.atol;
  a.outer_tol = b->prec.outer_tol;
  a.maxit = b->prec.maxit;
  a.max_passes = std::max(b->prec.refine_max, 1);
  a.paper_mode = b->prec.refine_max == 0;
  a.outer_stop = !a.paper_mode && (b->prec.inner_stop == MPRK_STOP_OUTER ||
                                   (b->prec.inner_stop == MPRK_STOP_AUTO &&
                                    b->prec.storage != MPRK_FP64));
  a.bs = b->bs;
  // start values (as for a single problem; every stage is implicit here): AUTO takes the
  // extrapolated slopes with the outer loop, rhs in the one-solve mode
  int mode = b->prec.stage_start;
  if (mode == MPRK_START_AUTO) mode = a.paper_mode ? MPRK_START_RHS : MPRK_START_EXTRAP;
  auto cst = [&](int r) {  // c_r; the step's start (r = -1) is c = 0
    double c = 0.0;
    for (int j = 0; j <= r; ++j) c += a.A[r][j];
    return c;
  };
  a.feval = mode == MPRK_START_SLOPE_EVAL || (mode == MPRK_START_EXTRAP && a.s > 1);
  a.fkeep = mode == MPRK_START_EXTRAP && a.s > 1;
  a.y0f = mode == MPRK_START_SLOPE_EVAL ? 1.0 : 0.0;
  for (int i = 1; i < a.s; ++i) {
    a.ya[i] = mode == MPRK_START_RHS ? 0.0 : 1.0;
    a.yb[i] = 0.0;
    a.yj[i] = 0;
    if (mode != MPRK_START_EXTRAP) continue;
    const double d1 = cst(i) - cst(i - 1), d0 = cst(i - 1) - cst(i - 2);
    if (std::fabs(d0) <= 1e-12) continue;
    const double th = d1 / d0;
    a.ya[i] = 1.0 + th;
    a.yb[i] = -th;
    a.yj[i] = i >= 2 ? i - 2 : a.s - 1;  // the slot holding f(u) before the second stage
  }
  return a;
}

// Device descriptors of every problem for the current schedule.
static void batch_problems(mprk_batch* b, std::vector<BProb>& hp, std::vector<int>& map) {
  const double a = b->tab.a_hi[0] + b->tab.a_lo[0];
  hp.assign(b->count, BProb{});
  map.assign(b->G, 0);
  int wg = 0;
  for (int p = 0; p < b->count; ++p) {
    const mprk_problem& q = b->probs[p];
    BProb& P = hp[p];
    const int N = b->N[p];
    P.geo = Geo{q.grid.nx, q.grid.ny, q.grid.nz, q.grid.bc, N, q.grid.nx * q.grid.ny};
    P.K = operator_coef(q.grid, q.op);
    P.sigma = q.dt * a;
    P.dt = q.dt;
    P.u = b->u[p];
    P.rhs = (double*)(b->ws + b->off_rhs[p]);
    P.y = P.rhs + N;
    P.res = P.y + N;
    P.k = (double*)(b->ws + b->off_k[p]);
    const size_t vlp = ((size_t)N * b->lp_bytes + 255) & ~(size_t)255;
    char* lp = b->ws + b->off_r[p];
    P.r = lp;
    P.z = lp + vlp;
    P.p0 = lp + 2 * vlp;
    P.p1 = lp + 3 * vlp;
    P.q = lp + 4 * vlp;
    P.x = lp + 5 * vlp;
    P.dinv = b->bs ? (void*)(b->ws + b->off_dinv[p]) : nullptr;
    P.part = (double*)(b->ws + b->off_part[p]);
    P.ctl = (BCtl*)(b->ws + b->o_ctl) + p;
    P.wg0 = wg;
    P.nwg = b->nwg[p];
    P.chunk = b->chunk[p];
    for (int i = 0; i < P.nwg; ++i) map[wg + i] = p;
    wg += P.nwg;
  }
}

// Upload the descriptors of the current schedule and capture one step (s stage launches) as a
// graph on a private non-blocking stream.
static int batch_upload_capture(mprk_batch* b, const std::vector<BProb>& hp, const std::vector<int>& map) {
  BHIP(hipMemcpyAsync(b->ws + b->o_probs, hp.data(), sizeof(BProb) * b->count, hipMemcpyHostToDevice, b->stream));
  BHIP(hipMemcpyAsync(b->ws + b->o_map, map.data(), sizeof(int) * b->G, hipMemcpyHostToDevice, b->stream));
  BHIP(hipStreamSynchronize(b->stream));  // host vectors may go out of scope
  if (b->gexec) {
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  const BArgs args = batch_args(b);
  const void* kern = batch_kernel(b->prec.storage, b->bs, b->ru);
  hipStream_t cs;
  BHIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    for (int st = 0; st < b->tab.s && e == hipSuccess; ++st) {
      void* kargs[] = {(void*)&args, (void*)&st};
      e = hipLaunchKernel(kern, dim3(b->G), dim3(TPB), kargs, 0, cs);
    }
    hipError_t e2 = hipStreamEndCapture(cs, &b->graph);
    if (e == hipSuccess) e = e2;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) return set_error(MPRK_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  return MPRK_OK;
}

extern "C" int32_t mprk_batch_bind(mprk_batch* b, double* const* u_dev, void* workspace_dev,
                                   int64_t bytes) {
  if (!b || !u_dev || !workspace_dev) return set_error(MPRK_EINVAL, "NULL argument");
  int64_t need = mprk_batch_workspace_bytes(b);
  if (need < 0) return (int32_t)need;
  if (bytes < need) return set_error(MPRK_ENOMEM, "workspace smaller than mprk_batch_workspace_bytes");
  if (((uintptr_t)workspace_dev & 255) != 0) return set_error(MPRK_EINVAL, "workspace must be 256-byte aligned");
  b->ws = (char*)workspace_dev;
  b->u.assign(u_dev, u_dev + b->count);
  for (int p = 0; p < b->count; ++p)
    if (!b->u[p]) return set_error(MPRK_EINVAL, "NULL state pointer");
  std::vector<BProb> hp;
  std::vector<int> map;
  batch_problems(b, hp, map);
  BHIP(hipMemsetAsync(b->ws + b->o_ctl, 0, sizeof(BCtl) * b->count, b->stream));
  BHIP(hipMemsetAsync(b->ws + b->o_flag, 0, 256, b->stream));
  // block-Jacobi inverses with the single-problem setup kernel
  int* fail = nullptr;
  if (b->bs) {
    Engine* eng = b->prec.storage == MPRK_FP64 ? make_engine_fp64()
                  : b->prec.storage == MPRK_FP32 ? make_engine_fp32() : make_engine_fp16();
    std::unique_ptr<Engine> guard(eng);
    fail = (int*)(b->ws + b->o_flag);
    for (int p = 0; p < b->count; ++p) {
      EngineCtx c{};
      c.stream = b->stream;
      c.geo = hp[p].geo;
      c.bs = b->bs;
      const int nblk = (c.geo.N + b->bs - 1) / b->bs;
      BHIP(eng->bj_setup_stencil(c, stage_coef(hp[p].K, hp[p].sigma), hp[p].dinv, fail, nblk, nullptr, 0));
    }
  }
  int hfail = 0;
  if (fail) {
    BHIP(hipMemcpyAsync(&hfail, fail, sizeof(int), hipMemcpyDeviceToHost, b->stream));
  }
  BHIP(hipStreamSynchronize(b->stream));
  if (hfail) return set_error(MPRK_EINVAL, "singular block-Jacobi block in batch");
  const int rc = batch_upload_capture(b, hp, map);
  if (rc) return rc;
  b->good_seen.assign(b->count, 0);
  b->bad_seen.assign(b->count, 0);
  b->bound = true;
  return MPRK_OK;
}

// Autotuner of the CTA-group schedule: for each exponent e of the work model (unknowns x
// condition-number estimate^e), plan the workgroups per problem, replay one step from the
// current state (after one untimed replay) and keep the fastest.  The problems' states and
// statistics are restored afterwards.  A schedule fixed with mprk_batch_set_schedule is kept.
extern "C" int32_t mprk_batch_autotune(mprk_batch* b, double* exponent_out, int32_t* rows_out) {
  if (!b) return set_error(MPRK_EINVAL, "NULL batch");
  if (!b->bound) return set_error(MPRK_ESTATE, "mprk_batch_autotune before mprk_batch_bind");
  if (!b->fixed_wg.empty()) return set_error(MPRK_ESTATE, "schedule fixed by mprk_batch_set_schedule");
  // save the states and the per-problem records on the host
  std::vector<std::vector<double>> saved(b->count);
  for (int p = 0; p < b->count; ++p) {
    saved[p].resize(b->N[p]);
    BHIP(hipMemcpyAsync(saved[p].data(), b->u[p], (size_t)b->N[p] * 8, hipMemcpyDeviceToHost, b->stream));
  }
  std::vector<BCtl> ctl(b->count);
  BHIP(hipMemcpyAsync(ctl.data(), b->ws + b->o_ctl, sizeof(BCtl) * b->count, hipMemcpyDeviceToHost, b->stream));
  BHIP(hipStreamSynchronize(b->stream));
  auto restore = [&]() -> int {
    for (int p = 0; p < b->count; ++p)
      BHIP(hipMemcpyAsync(b->u[p], saved[p].data(), (size_t)b->N[p] * 8, hipMemcpyHostToDevice, b->stream));
    BHIP(hipStreamSynchronize(b->stream));
    return MPRK_OK;
  };
  hipEvent_t e0, e1;
  BHIP(hipEventCreate(&e0));
  BHIP(hipEventCreate(&e1));
  // one trial: plan with the current (ru, weight_exp), replay one step twice from the saved
  // states, return the second replay's time
  auto trial = [&](float* ms) -> int {
    int r = batch_capacity(b, b->ru, &b->capacity);
    if (!r) r = plan_groups(b, b->capacity);
    std::vector<BProb> hp;
    std::vector<int> map;
    if (!r) {
      batch_problems(b, hp, map);
      r = batch_upload_capture(b, hp, map);
    }
    for (int rep = 0; rep < 2 && !r; ++rep) {
      r = restore();
      if (r) break;
      if (hipEventRecord(e0, b->stream) != hipSuccess || hipGraphLaunch(b->gexec, b->stream) != hipSuccess ||
          hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        r = set_error(MPRK_EDEVICE, "autotune replay failed");
    }
    if (!r && hipEventElapsedTime(ms, e0, e1) != hipSuccess) r = set_error(MPRK_EDEVICE, "autotune timing failed");
    return r;
  };
  int rc = MPRK_OK;
  // rows per thread per CG iteration (the work model fixed at its default), then the work model
  int best_ru = b->ru;
  float best_ms = 1e30f;
  for (int ru : {1, 2, 4}) {
    b->ru = ru;
    float ms = 0.f;
    rc = trial(&ms);
    if (rc) break;
    if (ms < best_ms) {
      best_ms = ms;
      best_ru = ru;
    }
  }
  b->ru = best_ru;
  double best_e = b->weight_exp;
  const double cands[] = {0.0, 0.25, 0.75, 1.0};
  for (double e : cands) {
    if (rc) break;
    const double keep = b->weight_exp;
    b->weight_exp = e;
    float ms = 0.f;
    rc = trial(&ms);
    if (rc) break;
    if (ms < best_ms) {
      best_ms = ms;
      best_e = e;
    }
    b->weight_exp = keep;
  }
  // the measured work of the last step (when one ran): unknowns x (CG iterations + 1.6 x outer
  // passes, an FP64 pass moving about 1.6 times a CG iteration's bytes), each problem's real
  // share instead of the condition-number estimate
  bool best_measured = false;
  {
    std::vector<double> mw(b->count);
    double tot = 0.0;
    for (int p = 0; p < b->count; ++p) {
      double it = 0.0, ps = 0.0;
      for (int i = 0; i < b->tab.s && i < MAXS; ++i) {
        it += ctl[p].iters[i];
        ps += ctl[p].passes[i];
      }
      mw[p] = (double)b->N[p] * (it + 1.6 * ps);
      tot += mw[p];
    }
    if (!rc && tot > 0.0) {
      b->measured_w = mw;
      b->use_measured = true;
      float ms = 0.f;
      rc = trial(&ms);
      if (!rc && ms < best_ms) {
        best_ms = ms;
        best_measured = true;
      }
      b->use_measured = best_measured;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->weight_exp = best_e;
  int rc2 = batch_capacity(b, b->ru, &b->capacity);
  if (!rc2) rc2 = plan_groups(b, b->capacity);
  if (!rc2) {
    std::vector<BProb> hp;
    std::vector<int> map;
    batch_problems(b, hp, map);
    rc2 = batch_upload_capture(b, hp, map);
  }
  if (!rc2) rc2 = restore();
  if (!rc2) {
    BHIP(hipMemcpyAsync(b->ws + b->o_ctl, ctl.data(), sizeof(BCtl) * b->count, hipMemcpyHostToDevice, b->stream));
    BHIP(hipStreamSynchronize(b->stream));
  }
  if (exponent_out) *exponent_out = best_measured ? -1.0 : best_e;
  if (rows_out) *rows_out = b->ru;
  return rc ? rc : rc2;
}

extern "C" int32_t mprk_batch_step(mprk_batch* b, int32_t nsteps) {
  if (!b) return set_error(MPRK_EINVAL, "NULL batch");
  if (!b->bound) return set_error(MPRK_ESTATE, "mprk_batch_step before mprk_batch_bind");
  if (nsteps < 0) return set_error(MPRK_EINVAL, "nsteps must be >= 0");
  for (int n = 0; n < nsteps; ++n) BHIP(hipGraphLaunch(b->gexec, b->stream));
  return MPRK_OK;
}

extern "C" int32_t mprk_batch_stats_sync(mprk_batch* b, int32_t idx, mprk_stats* out) {
  if (!b || !out) return set_error(MPRK_EINVAL, "NULL argument");
  if (!b->bound) return set_error(MPRK_ESTATE, "not bound");
  if (idx < 0 || idx >= b->count) return set_error(MPRK_EINVAL, "problem index out of range");
  BCtl c;
  BHIP(hipMemcpyAsync(&c, (BCtl*)(b->ws + b->o_ctl) + idx, sizeof(BCtl), hipMemcpyDeviceToHost, b->stream));
  BHIP(hipStreamSynchronize(b->stream));
  std::memset(out, 0, sizeof(*out));
  out->steps = c.good_steps;
  out->t = c.good_steps * b->probs[idx].dt;
  out->stages = b->tab.s;
  for (int i = 0; i < b->tab.s; ++i) {
    out->iters[i] = c.iters[i];
    out->passes[i] = c.passes[i];
    out->resid[i] = c.resid[i];
    out->converged[i] = c.converged[i];
  }
  out->total_iters = c.life_iters;
  out->total_passes = c.life_passes;
  out->nonfinite = c.bad_steps > 0;
  if (c.error) return set_error(MPRK_EDEVICE, "a batched group barrier timed out (workgroups not co-resident)");
  return MPRK_OK;
}

extern "C" void mprk_batch_destroy(mprk_batch* b) { delete b; }

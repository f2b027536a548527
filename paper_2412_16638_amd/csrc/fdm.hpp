// fdm.hpp -- fast-diagonalisation preconditioner kernels (gfx950).
//
// The preconditioner of Section "Problem setting and solver design", eq. preconbasic, with
// A = I - sigma Kx, B = -sigma Ky, C = -sigma Kz is the stage matrix itself for the heat
// operator; eq. Pinvform applies its inverse as
//   z = (Q_C (x) Q_B (x) Q_A) P_D^-1 (Q_C^-1 (x) Q_B^-1 (x) Q_A^-1) r,
// each Kronecker factor being the product of the three one-axis contractions of eq.
// TensorDecomp, (T_R x)_{ijk} = sum_q Q_{iq} x_{qjk} (along x), T_M along y, T_L along z.
// Here the 1-D eigenbases are real, orthogonal and symmetric (Q^-1 = Q): the sine basis for
// zero Dirichlet ends and the Hartley basis for periodic ones, so both halves use the same Q.
//
// Every contraction is a GEMM with K = n (the axis length): along x the rows of x are
// contiguous (out = X Q^T, "row" form); along y and z the contracted index is strided and the
// remaining index contiguous (out_b = Q X_b, "column" form).  One LDS-tiled kernel does both:
// 64 x 64 output tiles, K staged in LDS in chunks of 32 (FP32) or 16 (FP64), 256 threads with
// 4 x 4 outputs each, FP32 (FP64 for FP64 storage) accumulation.  The P_D^-1 scaling is fused
// into the third forward contraction.
#pragma once

#include <cmath>

#include "device.hpp"

namespace mprk {

constexpr int FT_M = 64;  // output tile rows
constexpr int FT_N = 64;  // output tile columns

// Contraction chunk staged in LDS per pass: both 64 x KC operand tiles are loaded with all their
// loads in flight, then KC rank-1 updates run from LDS (17 KB for either type, so that several
// blocks share a CU).
template <typename C>
constexpr int fdm_kc() {
  return sizeof(C) == 8 ? 16 : 32;
}
static_assert(fdm_kc<float>() % 4 == 0 && fdm_kc<double>() % 4 == 0, "k steps of 4");

// Geometry of one contraction.  ROW form (along x): out[r][a] = sum_q in[r][q] Q[a][q] for
// r < nr rows of length n.  COL form: out[b][a][c] = sum_q Q[a][q] in[b][q][c], c < nc
// contiguous, rows of `in` / `out` ld elements apart, batches bstride apart.
struct FdmGeo {
  int n;         // axis length (= contraction length)
  int nr;        // ROW form: number of rows
  int nc;        // COL form: contiguous extent
  int ld;        // COL form: elements between consecutive q (and a) rows
  long bstride;  // COL form: elements between batches
  int nb;        // COL form: batches
};

// Scaling by P_D^-1 (fused into a COL-form contraction along z): the output element with
// z-index a and contiguous index c = j nx + i is divided by 1 - sk (lx[i] + ly[j] + lz[a]).
struct FdmScale {
  const double* lx;
  const double* ly;
  const double* lz;
  double sk;  // sigma * kappa
  int nx;
  int on;
};

template <typename TI, typename TO, typename C, int ROW>
__global__ __launch_bounds__(256) void k_fdm_contract(FdmGeo g, const C* __restrict__ Q,
                                                      const TI* __restrict__ in, TO* __restrict__ out,
                                                      FdmScale sc, Ctl* ctl) {
  if (ctl->outer_done | ctl->inner_done) return;
  count_work(ctl, KC_FDM, g.n);
  constexpr int KC = fdm_kc<C>();
  // rows padded by 4 elements (4-wide vector reads stay aligned)
  __shared__ __align__(32) C As[KC][FT_M + 4];  // As[k][m]: the operand indexed by the output row
  __shared__ __align__(32) C Bs[KC][FT_N + 4];  // Bs[k][n]: the operand indexed by the output column
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  static_assert(FT_M * fdm_kc<C>() % 256 == 0 && FT_M == FT_N, "whole chunks per thread");
  const int m0 = blockIdx.x * FT_M;  // ROW: rows r; COL: a
  const int n0 = blockIdx.y * FT_N;  // ROW: a;      COL: c
  const int b = blockIdx.z;
  const int n = g.n;
  const TI* inb = ROW ? in : in + (size_t)b * g.bstride;
  C acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = C(0);
  // Each thread stages PER elements of each operand per chunk; the next chunk's elements are
  // loaded into registers while the current chunk is multiplied from LDS.
  constexpr int PER = FT_M * KC / 256;
  C ra[PER], rb[PER];
  auto load_chunk = [&](int q0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      // operands indexed (row, k) with k contiguous in memory: e -> row e / KC, k e % KC
      const int e = threadIdx.x + u * 256;
      const int lr = e / KC, kk = e % KC, q = q0 + kk;
      if constexpr (ROW) {
        const int r = m0 + lr, a = n0 + lr;
        ra[u] = (r < g.nr && q < n) ? (C)inb[(size_t)r * n + q] : C(0);
        rb[u] = (a < n && q < n) ? Q[(size_t)a * n + q] : C(0);
      } else {
        const int a = m0 + lr;
        ra[u] = (a < n && q < n) ? Q[(size_t)a * n + q] : C(0);
        // in[b][q][c], contiguous along c: e -> row e / 64, column e % 64
        const int kq = e / FT_N, lc = e % FT_N, qq = q0 + kq, c = n0 + lc;
        rb[u] = (qq < n && c < g.nc) ? (C)inb[(size_t)qq * g.ld + c] : C(0);
      }
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + u * 256;
      As[e % KC][e / KC] = ra[u];
      if constexpr (ROW) Bs[e % KC][e / KC] = rb[u];
      else Bs[e / FT_N][e % FT_N] = rb[u];
    }
  };
  load_chunk(0);
  for (int q0 = 0; q0 < n; q0 += KC) {
    store_chunk();
    __syncthreads();
    if (q0 + KC < n) load_chunk(q0 + KC);  // in flight during the multiply below
    // k in steps of 4 (the tiles are zero past n, and KC is a multiple of 4); each thread reads
    // its 4 rows and 4 columns of a k-slice as one 4-wide LDS vector each
    const int kend = min(KC, (n - q0 + 3) & ~3);
    for (int k0 = 0; k0 < kend; k0 += 4) {
      Vec<C, 4> av[4], bv[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        av[kk] = *reinterpret_cast<const Vec<C, 4>*>(&As[k0 + kk][ty * 4]);
        bv[kk] = *reinterpret_cast<const Vec<C, 4>*>(&Bs[k0 + kk][tx * 4]);
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] += av[kk].v[i] * bv[kk].v[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int mi = m0 + ty * 4 + i;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int nj = n0 + tx * 4 + j;
      if constexpr (ROW) {
        if (mi < g.nr && nj < n) out[(size_t)mi * n + nj] = (TO)acc[i][j];
      } else {
        if (mi < n && nj < g.nc) {
          C v = acc[i][j];
          if (sc.on) {
            const int ix = nj % sc.nx, jy = nj / sc.nx;
            v = (C)((double)v / (1.0 - sc.sk * (sc.lx[ix] + sc.ly[jy] + sc.lz[mi])));
          }
          out[(size_t)b * g.bstride + (size_t)mi * g.ld + nj] = (TO)v;
        }
      }
    }
  }
}

// Host-side description of one axis: orthogonal symmetric eigenbasis Q (n x n, row-major) and
// eigenvalues lam of the unscaled 1-D second difference divided by h^2 (so that the axis factor
// of sigma K is sigma kappa lam).
//   Dirichlet (h = 1/(n+1)): Q_{ik} = sqrt(2/(n+1)) sin(pi (i+1)(k+1)/(n+1)),
//     lam_k = -(4/h^2) sin^2(pi (k+1) h / 2);
//   periodic (h = 1/n): Q_{ik} = (cos(2 pi i k/n) + sin(2 pi i k/n)) / sqrt(n) (Hartley),
//     lam_k = -(4/h^2) sin^2(pi k / n).
inline void fdm_axis_basis(int n, int periodic, double* Q, double* lam) {
  const double pi = 3.14159265358979323846;
  if (!periodic) {
    const double h = 1.0 / (n + 1);
    const double s = std::sqrt(2.0 / (n + 1));
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) Q[(size_t)i * n + k] = s * std::sin(pi * (i + 1) * (k + 1) / (n + 1));
    for (int k = 0; k < n; ++k) {
      const double t = std::sin(pi * (k + 1) * h / 2.0);
      lam[k] = -(4.0 / (h * h)) * t * t;
    }
  } else {
    const double h = 1.0 / n;
    const double s = 1.0 / std::sqrt((double)n);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) {
        const double th = 2.0 * pi * (double)(((long)i * k) % n) / n;
        Q[(size_t)i * n + k] = s * (std::cos(th) + std::sin(th));
      }
    for (int k = 0; k < n; ++k) {
      const double t = std::sin(pi * k / n);
      lam[k] = -(4.0 / (h * h)) * t * t;
    }
  }
}


// ------------------------------------------------------------------------------------------
// CG with a preconditioner applied by separate launches (the contractions above): the
// residual update and the (r, z) product are split around the preconditioner.
// ------------------------------------------------------------------------------------------

// A3 for CG with an external preconditioner: r = LP(res / scale), (r, r); the tolerance and the
// inner decision are set here, (r, z) by k_cg_rz after z = P^-1 r.
template <typename S, typename C, int VEC>
__global__ __launch_bounds__(TPB) void k_cg_begin_ext(Launch ln, const double* __restrict__ res,
                                                      S* __restrict__ r, SolveCfg cfg, Ctl* ctl,
                                                      Red red) {
  if (ctl->outer_done) return;
  count_work(ctl, KC_CG_BEGIN);
  const double inv = 1.0 / ctl->scale;
  const int L = xcd_block(ln.G);
  double acc[1] = {0.0};
  for (int it = 0; it < ln.nit; ++it) {
    const int g = (L * ln.nit + it) * TPB + threadIdx.x;
    if (g >= ln.ng) break;
    double t[VEC];
    loadv<double, double, VEC>(res + g * VEC, t);
    C rv[VEC];
    C s = C(0);
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      rv[v] = rnd<S, C>((C)(t[v] * inv));
      s += rv[v] * rv[v];
    }
    storev<S, C, VEC>(r + g * VEC, rv);
    acc[0] += (double)s;
  }
  __shared__ double tot[1];
  if (!reduce_to_last<1>(acc, 1, red, L, ln.G, tot)) return;
  if (threadIdx.x == 0) {
    const double rr = tot[0];
    const double bn = sqrt(rr);
    ctl->rr = rr;
    ctl->beta = 0.0;
    ctl->iters = 0;
    ctl->tol = fmax(cfg.rtol * bn, cfg.atol / ctl->scale);
    ctl->inner_done = (bn <= ctl->tol) || cfg.maxit <= 0;
  }
}

// x += alpha p (x = alpha p first), r -= alpha q, (r, r); convergence test on ||r||.
template <typename S, typename C, int VEC>
__global__ __launch_bounds__(TPB) void k_cg_upd_ext(Launch ln, S* __restrict__ x,
                                                    const S* __restrict__ p, S* __restrict__ r,
                                                    const S* __restrict__ q, SolveCfg cfg, Ctl* ctl,
                                                    Red red) {
  if (ctl->outer_done | ctl->inner_done) return;
  count_work(ctl, KC_CG_UPD);
  const int first = ctl->iters == 0;
  const C alpha = (C)ctl->alpha;
  const int L = xcd_block(ln.G);
  double acc[1] = {0.0};
  for (int it = 0; it < ln.nit; ++it) {
    const int g = (L * ln.nit + it) * TPB + threadIdx.x;
    if (g >= ln.ng) break;
    const int e = g * VEC;
    C pv[VEC], qv[VEC], rv[VEC], xv[VEC];
    loadv<C, S, VEC>(p + e, pv);
    loadv<C, S, VEC>(q + e, qv);
    loadv<C, S, VEC>(r + e, rv);
    loadv<C, S, VEC>(x + e, xv);  // unused in the first iteration
    C s = C(0);
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      xv[v] = first ? alpha * pv[v] : xv[v] + alpha * pv[v];
      rv[v] = rnd<S, C>(rv[v] - alpha * qv[v]);
      s += rv[v] * rv[v];
    }
    storev<S, C, VEC>(x + e, xv);
    storev<S, C, VEC>(r + e, rv);
    acc[0] += (double)s;
  }
  __shared__ double tot[1];
  if (!reduce_to_last<1>(acc, 1, red, L, ln.G, tot)) return;
  if (threadIdx.x == 0) {
    const double rr = tot[0];
    const int its = ctl->iters + 1;
    ctl->iters = its;
    ctl->total_iters += 1;
    ctl->life_iters += 1;
    ctl->rr = rr;
    ctl->inner_done = !__builtin_isfinite(rr) || sqrt(rr) <= ctl->tol || its >= cfg.maxit;
  }
}

// (r, z) after z = P^-1 r.  BEGIN: the first product of a solve; else beta = (r,z)_new/(r,z)_old.
template <typename S, typename C, int VEC, int BEGIN>
__global__ __launch_bounds__(TPB) void k_cg_rz(Launch ln, const S* __restrict__ r,
                                               const S* __restrict__ z, Ctl* ctl, Red red) {
  if (ctl->outer_done | ctl->inner_done) return;
  count_work(ctl, KC_CG_RZ);
  const int L = xcd_block(ln.G);
  double acc[1] = {0.0};
  for (int it = 0; it < ln.nit; ++it) {
    const int g = (L * ln.nit + it) * TPB + threadIdx.x;
    if (g >= ln.ng) break;
    C rv[VEC], zv[VEC];
    loadv<C, S, VEC>(r + g * VEC, rv);
    loadv<C, S, VEC>(z + g * VEC, zv);
    C s = C(0);
#pragma unroll
    for (int v = 0; v < VEC; ++v) s += rv[v] * zv[v];
    acc[0] += (double)s;
  }
  __shared__ double tot[1];
  if (!reduce_to_last<1>(acc, 1, red, L, ln.G, tot)) return;
  if (threadIdx.x == 0) {
    const double rz = tot[0];
    if (!BEGIN) ctl->beta = rz / ctl->rz;
    ctl->rz = rz;
    if (!__builtin_isfinite(rz)) ctl->inner_done = 1;
  }
}

}  // namespace mprk

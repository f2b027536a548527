// fdm.hpp -- fast-diagonalisation preconditioner kernels (gfx950).
//
// The preconditioner of Section "Problem setting and solver design", eq. preconbasic, with
// A = I - sigma Kx, B = -sigma Ky, C = -sigma Kz is the stage matrix itself for every operator
// here (Kronecker sums); eq. Pinvform applies its inverse as
//   z = (Q_C (x) Q_B (x) Q_A) P_D^-1 (Q_C^-1 (x) Q_B^-1 (x) Q_A^-1) r,
// each Kronecker factor being the product of the three one-axis contractions of eq.
// TensorDecomp, (T_R x)_{ijk} = sum_q Q_{iq} x_{qjk} (along x), T_M along y, T_L along z.
// For the heat operator the 1-D eigenbases are real, orthogonal and symmetric (Q^-1 = Q): the
// sine basis for zero Dirichlet ends and the Hartley basis for periodic ones, so both halves
// use the same Q.  For the periodic advection operators the 1-D factors are circulant and the
// basis is the unitary DFT (complex; Q^-1 = conj(Q)), see k_fdm_contract_cx.
//
// Every contraction is a GEMM with K = n (the axis length): along x the rows of x are
// contiguous (out = X Q^T, "row" form); along y and z the contracted index is strided and the
// remaining index contiguous (out_b = Q X_b, "column" form).  One kernel does both on the
// matrix cores (FP32 MFMA, FP64 MFMA for FP64 storage): 64 x 64 output tiles, 4 waves of 2 x 2
// 16 x 16 products, K staged in LDS in chunks of 32 with the next chunk prefetched into
// registers.  (Tile heights 32/64 and chunks 32/64 measured alike at 128^3, within 5 %: a
// launch there is bound by its fixed latency, not by the matrix cores or HBM.)  The P_D^-1
// scaling is fused into the third forward contraction.
#pragma once

#include <cmath>

#include "device.hpp"

namespace mprk {

constexpr int FT_M = 64;  // output tile rows
constexpr int FT_N = 64;  // output tile columns
constexpr int FT_KC = 32; // contraction chunk staged in LDS per pass

// Row stride of a stored eigenbasis: n rounded up to 4 (zero padded), so that every 4-wide load
// of a basis row is aligned and in bounds.
inline int fdm_ldq(int n) { return (n + 3) & ~3; }

// Geometry of one contraction.  ROW form (along x): out[r][a] = sum_q in[r][q] Q[a][q] for
// r < nr rows of length n.  COL form: out[b][a][c] = sum_q Q[a][q] in[b][q][c], c < nc
// contiguous, rows of `in` / `out` ld elements apart, batches bstride apart.
struct FdmGeo {
  int n;         // axis length (= contraction length)
  int ldq;       // row stride of Q (fdm_ldq(n))
  int nr;        // ROW form: number of rows
  int nc;        // COL form: contiguous extent
  int ld;        // COL form: elements between consecutive q (and a) rows
  long bstride;  // COL form: elements between batches
  int nb;        // COL form: batches
  int tiles;     // output tiles (the grid is this rounded up to a multiple of 8)
  int skip_inner;  // 1: return once the inner solve is done (applies inside a Krylov loop)
  int rk = 0;    // complex ROW form: contraction extent = input row stride (0: n)
  int ro = 0;    // complex ROW form: outputs per row = output row stride (0: n)
  // complex COL form with folded batches (cfold > 0, nb = 1): contiguous index c stands for
  // batch c / cfold, element c % cfold, at (c / cfold) cstride + q ld + c % cfold
  int cfold = 0;
  long cstride = 0;
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

// One 16 x 16 x 4 matrix-core product-accumulate: D = A B + D, A 16 x 4, B 4 x 16.  Lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; its i-th accumulator (i < 4) holds
// D[row(l / 16, i)][l % 16], row = 4 (l / 16) + i for FP32 and 4 i + l / 16 for FP64.
template <typename C>
struct Mfma;
template <>
struct Mfma<float> {
  typedef float acc __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g4, int i) { return 4 * g4 + i; }
};
template <>
struct Mfma<double> {
  typedef double acc __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g4, int i) { return 4 * i + g4; }
};

// One contraction (either form) on the matrix cores.  A block computes a 64 x 64 output tile;
// each of its 4 waves a 32 x 32 quarter as 2 x 2 MFMA tiles.  K runs in chunks of FT_KC staged
// in LDS, the next chunk loaded into registers while the current one is multiplied.  Since the
// sum over q may visit q in any order common to both operands, lane group g of the j-th product
// of a 16-wide k block takes k = 4 g + j: each lane then reads its 4 k values of an operand
// whose k is contiguous as one 4-wide LDS vector.  Tiles are zero past the problem edges, so
// padded rows and k values add nothing.  V4: the data operand is loaded 4 elements at a time
// (its contiguous extent is a multiple of 4), else element by element.
template <typename TI, typename TO, typename C, int ROW, int V4, int BM, int KC>
__global__ __launch_bounds__(256) void k_fdm_contract(FdmGeo g, const C* __restrict__ Q,
                                                      const TI* __restrict__ in, TO* __restrict__ out,
                                                      FdmScale sc, Ctl* ctl) {
  static_assert((BM == 32 || BM == 64) && (KC == 32 || KC == 64), "tile shapes");
  if (ctl->outer_done | (g.skip_inner & ctl->inner_done)) return;
  count_work(ctl, KC_FDM, g.n);
  constexpr int PK = KC + 4, PN = FT_N + 4;
  constexpr int MI = BM / 32;              // 16-row MFMA tiles per wave (waves 2 x 2)
  constexpr int KV = KC / 4;               // 4-wide vectors per k-contiguous row of a chunk
  constexpr int NA = BM * KV / 256;        // staged vectors per thread: A operand
  constexpr int NB = FT_N * KV / 256;      //                            B operand
  typedef typename Mfma<C>::acc Acc;
  // As[m][k]: the operand indexed by the output row.  ROW: Bs[n][k] (basis rows, k contiguous);
  // COL: Bs[k][n] (data rows, n contiguous).  Row strides of KC + 4 and 68 elements keep the
  // 16-lane groups of an MFMA operand read on distinct banks.
  __shared__ __align__(32) C As[BM][PK];
  __shared__ __align__(32) C Bs[ROW ? FT_N : KC][ROW ? PK : PN];
  const int n = g.n;
  const int T = xcd_block((g.tiles + 7) & ~7);
  if (T >= g.tiles) return;
  // tiles that read the same data rows are consecutive (same XCD, same L2)
  int mt, nt, b = 0;
  if constexpr (ROW) {
    const int NT = (n + FT_N - 1) / FT_N;
    nt = T % NT;
    mt = T / NT;
  } else {
    const int MT = (n + BM - 1) / BM, NT = (g.nc + FT_N - 1) / FT_N;
    mt = T % MT;
    nt = (T / MT) % NT;
    b = T / (MT * NT);
  }
  const int m0 = mt * BM;    // ROW: rows r; COL: a
  const int n0 = nt * FT_N;  // ROW: a;      COL: c
  const TI* inb = ROW ? in : in + (size_t)b * g.bstride;
  const int tid = threadIdx.x;
  // staging: vector e of a k-contiguous operand covers row e / KV, k 4 (e % KV) .. + 3; vector e
  // of the COL data covers k e / 16, n 4 (e % 16) .. + 3
  Vec<C, 4> ra[NA], rb[NB];
  auto zero4 = [](Vec<C, 4>& v) {
#pragma unroll
    for (int j = 0; j < 4; ++j) v.v[j] = C(0);
  };
  auto load_q = [&](Vec<C, 4>& v, int a, int q) {  // Q[a][q .. q + 3]
    if (a < n && q < g.ldq) v = *reinterpret_cast<const Vec<C, 4>*>(Q + (size_t)a * g.ldq + q);
    else zero4(v);
  };
  // data rows with k contiguous (ROW form): in[r][q .. q + 3]
  auto load_row = [&](Vec<C, 4>& v, int r, int q) {
    const TI* src = inb + (size_t)r * n + q;
    if constexpr (V4) {
      if (r < g.nr && q < n) {
        const Vec<TI, 4> t = *reinterpret_cast<const Vec<TI, 4>*>(src);
#pragma unroll
        for (int j = 0; j < 4; ++j) v.v[j] = (C)t.v[j];
      } else {
        zero4(v);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) v.v[j] = (r < g.nr && q + j < n) ? (C)src[j] : C(0);
    }
  };
  // data rows with n contiguous (COL form): in[b][qq][c .. c + 3]
  auto load_col = [&](Vec<C, 4>& v, int qq, int c) {
    const TI* src = inb + (size_t)qq * g.ld + c;
    if constexpr (V4) {
      if (qq < n && c < g.nc) {
        const Vec<TI, 4> t = *reinterpret_cast<const Vec<TI, 4>*>(src);
#pragma unroll
        for (int j = 0; j < 4; ++j) v.v[j] = (C)t.v[j];
      } else {
        zero4(v);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) v.v[j] = (qq < n && c + j < g.nc) ? (C)src[j] : C(0);
    }
  };
  auto load_chunk = [&](int q0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = tid + u * 256, row = e / KV, q = q0 + (e % KV) * 4;
      if constexpr (ROW) load_row(ra[u], m0 + row, q);
      else load_q(ra[u], m0 + row, q);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + u * 256;
      if constexpr (ROW) load_q(rb[u], n0 + e / KV, q0 + (e % KV) * 4);
      else load_col(rb[u], q0 + e / 16, n0 + (e % 16) * 4);
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = tid + u * 256;
      *reinterpret_cast<Vec<C, 4>*>(&As[e / KV][(e % KV) * 4]) = ra[u];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + u * 256;
      if constexpr (ROW) *reinterpret_cast<Vec<C, 4>*>(&Bs[e / KV][(e % KV) * 4]) = rb[u];
      else *reinterpret_cast<Vec<C, 4>*>(&Bs[e / 16][(e % 16) * 4]) = rb[u];
    }
  };
  const int lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, g4 = lane >> 4;
  const int wm = (w >> 1) * (BM / 2), wn = (w & 1) * 32;
  constexpr int NKB = KC / 16;  // 16-wide k blocks per chunk
  Acc acc[MI][2];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = Acc{};
  auto products = [&](const Vec<C, 4> (&av)[MI], const Vec<C, 4> (&bv)[2]) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = Mfma<C>::op(av[mi].v[j], bv[ni].v[j], acc[mi][ni]);
  };
  // Pipeline per chunk: read all of its operands from LDS into registers, barrier, then the
  // products of the first k block, the LDS store of the next chunk (loaded one chunk earlier)
  // and the global loads of the one after, and the remaining products, so that matrix-core
  // work overlaps the memory traffic.  Tiles are zero past n, so every k block is multiplied.
  load_chunk(0);
  store_chunk();
  __syncthreads();
  if (KC < n) load_chunk(KC);
  for (int q0 = 0; q0 < n; q0 += KC) {
    Vec<C, 4> av[NKB][MI], bv[NKB][2];
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      const int k = kb * 16 + 4 * g4;
#pragma unroll
      for (int i = 0; i < MI; ++i) av[kb][i] = *reinterpret_cast<const Vec<C, 4>*>(&As[wm + 16 * i + l16][k]);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if constexpr (ROW) {
          bv[kb][i] = *reinterpret_cast<const Vec<C, 4>*>(&Bs[wn + 16 * i + l16][k]);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) bv[kb][i].v[j] = Bs[k + j][wn + 16 * i + l16];
        }
      }
    }
    __syncthreads();  // every wave holds this chunk: the LDS tiles may be overwritten
    products(av[0], bv[0]);
    if (q0 + KC < n) {
      store_chunk();
      if (q0 + 2 * KC < n) load_chunk(q0 + 2 * KC);
    }
#pragma unroll
    for (int kb = 1; kb < NKB; ++kb) products(av[kb], bv[kb]);
    __syncthreads();  // the next chunk is in LDS
  }
  // P_D^-1 factors of this lane's rows and columns, loaded together (indices clamped in range)
  double sxy[2] = {0.0, 0.0}, sz[MI][4] = {};
  if constexpr (!ROW) {
    if (sc.on) {
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) {
        const int col = min(n0 + wn + 16 * ni + l16, g.nc - 1);
        sxy[ni] = sc.lx[col % sc.nx] + sc.ly[col / sc.nx];
      }
#pragma unroll
      for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int i = 0; i < 4; ++i) sz[mi][i] = sc.lz[min(m0 + wm + 16 * mi + Mfma<C>::row(g4, i), n - 1)];
    }
  }
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = m0 + wm + 16 * mi + Mfma<C>::row(g4, i);
        const int col = n0 + wn + 16 * ni + l16;
        C v = acc[mi][ni][i];
        if constexpr (ROW) {
          if (m < g.nr && col < n) out[(size_t)m * n + col] = (TO)v;
        } else {
          if (sc.on) v = (C)((double)v / (1.0 - sc.sk * (sxy[ni] + sz[mi][i])));
          if (m < n && col < g.nc) out[(size_t)b * g.bstride + (size_t)m * g.ld + col] = (TO)v;
        }
      }
}

// Complex eigenbases (the periodic advection operators: circulant 1-D factors, diagonalised by
// the unitary DFT Q_{aq} = e^{-2 pi i a q / n} / sqrt(n), inverse conj(Q)).  Planar storage: a
// complex array is a real and an imaginary array of the compute type.
struct FdmCx {
  const void* qr;   // Re Q (n x ldq)
  const void* qi;   // Im Q
  double qsign;     // +1: Q (forward), -1: conj(Q) (backward)
  const double* lxi;  // imaginary parts of the axis eigenvalues (real parts in FdmScale)
  const double* lyi;
  const double* lzi;
};

// One contraction with the complex basis on the matrix cores: the tile layout, staging and
// k-order of k_fdm_contract, with a real and an imaginary tile per operand and three real
// products per complex one by Gauss's rearrangement (two when the data operand is real, INR, or
// only the real part of the result is kept, OUTR).  The epilogue of the forward z contraction divides by the complex
// P_D = 1 - sk (lx + ly + lz).
template <typename TI, typename TO, typename C, int ROW, int V4, int INR, int OUTR>
__global__ __launch_bounds__(256) void k_fdm_contract_cx(FdmGeo g, FdmCx cx,
                                                         const TI* __restrict__ in_r,
                                                         const TI* __restrict__ in_i,
                                                         TO* __restrict__ out_r,
                                                         TO* __restrict__ out_i, FdmScale sc,
                                                         Ctl* ctl) {
  static_assert(!(INR && OUTR), "a contraction of the chain has a complex side");
  if (ctl->outer_done | (g.skip_inner & ctl->inner_done)) return;
  count_work(ctl, KC_FDM, g.n);
  constexpr int BM = 64, KC = FT_KC, PK = KC + 4, PN = FT_N + 4, KV = KC / 4;
  typedef typename Mfma<C>::acc Acc;
  const C* Qr = (const C*)cx.qr;
  const C* Qi = (const C*)cx.qi;
  const C qs = (C)cx.qsign;
  // As: the operand indexed by the output row ([m][k]); Bs: ROW [n][k], COL [k][n]
  __shared__ __align__(32) C Ar_s[BM][PK];
  __shared__ __align__(32) C Ai_s[BM][PK];
  __shared__ __align__(32) C Br_s[ROW ? FT_N : KC][ROW ? PK : PN];
  __shared__ __align__(32) C Bi_s[ROW ? FT_N : KC][ROW ? PK : PN];
  const int n = g.n;
  // ROW form: contraction extent (input row stride) and outputs per row (output row stride);
  // below n for the half spectrum of real data
  const int RK = (ROW && g.rk) ? g.rk : n, RO = (ROW && g.ro) ? g.ro : n;
  const int KN = ROW ? RK : n;
  const int T = xcd_block((g.tiles + 7) & ~7);
  if (T >= g.tiles) return;
  int mt, nt, b = 0;
  if constexpr (ROW) {
    const int NT = (RO + FT_N - 1) / FT_N;
    nt = T % NT;
    mt = T / NT;
  } else {
    const int MT = (n + BM - 1) / BM, NT = (g.nc + FT_N - 1) / FT_N;
    mt = T % MT;
    nt = (T / MT) % NT;
    b = T / (MT * NT);
  }
  const int m0 = mt * BM, n0 = nt * FT_N;
  const size_t boff = ROW ? 0 : (size_t)b * g.bstride;
  // COL form: offset of row q, contiguous index c (folded batches when g.cfold > 0; c and the
  // three after it share a batch, as cfold is a multiple of 4)
  auto coff = [&](int q, int c) -> size_t {
    if (g.cfold > 0) return (size_t)(c / g.cfold) * g.cstride + (size_t)q * g.ld + (c % g.cfold);
    return boff + (size_t)q * g.ld + c;
  };
  const int tid = threadIdx.x;
  auto zero4 = [](Vec<C, 4>& v) {
#pragma unroll
    for (int j = 0; j < 4; ++j) v.v[j] = C(0);
  };
  auto load_q = [&](Vec<C, 4>& vr, Vec<C, 4>& vi, int a, int q) {
    if (a < n && q < g.ldq) {
      vr = *reinterpret_cast<const Vec<C, 4>*>(Qr + (size_t)a * g.ldq + q);
      vi = *reinterpret_cast<const Vec<C, 4>*>(Qi + (size_t)a * g.ldq + q);
#pragma unroll
      for (int j = 0; j < 4; ++j) vi.v[j] *= qs;
    } else {
      zero4(vr);
      zero4(vi);
    }
  };
  // 4 consecutive data elements at src (row-contiguous), masked by `ok` / per element by lim
  auto load_data = [&](Vec<C, 4>& v, const TI* src, bool ok, int lim) {
    if constexpr (V4) {
      if (ok) {
        const Vec<TI, 4> t = *reinterpret_cast<const Vec<TI, 4>*>(src);
#pragma unroll
        for (int j = 0; j < 4; ++j) v.v[j] = (C)t.v[j];
      } else {
        zero4(v);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) v.v[j] = (ok && j < lim) ? (C)src[j] : C(0);
    }
  };
  Vec<C, 4> rar[2], rai[2], rbr[2], rbi[2];
  auto load_chunk = [&](int q0) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = tid + u * 256;
      const int row = e / KV, q = q0 + (e % KV) * 4;
      if constexpr (ROW) {
        const int r = m0 + row;
        const size_t off = (size_t)r * RK + q;
        load_data(rar[u], in_r + off, r < g.nr && q < RK, RK - q);
        if constexpr (!INR) load_data(rai[u], in_i + off, r < g.nr && q < RK, RK - q);
        load_q(rbr[u], rbi[u], n0 + row, q);
      } else {
        load_q(rar[u], rai[u], m0 + row, q);
        const int kk = e >> 4, c = n0 + (e & 15) * 4, qq = q0 + kk;
        const size_t off = (qq < n && c < g.nc) ? coff(qq, c) : 0;
        load_data(rbr[u], in_r + off, qq < n && c < g.nc, g.nc - c);
        if constexpr (!INR) load_data(rbi[u], in_i + off, qq < n && c < g.nc, g.nc - c);
      }
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = tid + u * 256;
      const int row = e / KV, kq = (e % KV) * 4;
      *reinterpret_cast<Vec<C, 4>*>(&Ar_s[row][kq]) = rar[u];
      if constexpr (!(ROW && INR)) *reinterpret_cast<Vec<C, 4>*>(&Ai_s[row][kq]) = rai[u];
      if constexpr (ROW) {
        *reinterpret_cast<Vec<C, 4>*>(&Br_s[row][kq]) = rbr[u];
        *reinterpret_cast<Vec<C, 4>*>(&Bi_s[row][kq]) = rbi[u];
      } else {
        *reinterpret_cast<Vec<C, 4>*>(&Br_s[e >> 4][(e & 15) * 4]) = rbr[u];
        if constexpr (!INR) *reinterpret_cast<Vec<C, 4>*>(&Bi_s[e >> 4][(e & 15) * 4]) = rbi[u];
      }
    }
  };
  const int lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, g4 = lane >> 4;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  // the data operand's imaginary part is zero (INR): A for ROW, B for COL
  constexpr bool AR = ROW && INR, BR = !ROW && INR;
  // both operands complex and the full result kept: three real products per complex one
  // (P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi); re = P1 - P2, im = P3 - P1 - P2)
  constexpr bool G3 = !AR && !BR && !OUTR;
  // 16 x 16 product tiles of this wave with no output in range (a partial last tile, e.g. the
  // H = nx/2 + 1 frequencies of the half spectrum) skip their products; wave-uniform
  bool live[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
      live[mi][ni] = ROW ? (m0 + wm + 16 * mi < g.nr && n0 + wn + 16 * ni < RO)
                         : (m0 + wm + 16 * mi < n && n0 + wn + 16 * ni < g.nc);
  Acc accr[2][2], acci[2][2], accq[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accr[i][j] = Acc{};
      acci[i][j] = Acc{};
      accq[i][j] = Acc{};
    }
  load_chunk(0);
  for (int q0 = 0; q0 < KN; q0 += KC) {
    store_chunk();
    __syncthreads();
    if (q0 + KC < KN) load_chunk(q0 + KC);
#pragma unroll
    for (int kb = 0; kb < KC; kb += 16) {
      const int k = kb + 4 * g4;
      Vec<C, 4> avr[2], avi[2], bvr[2], bvi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        avr[i] = *reinterpret_cast<const Vec<C, 4>*>(&Ar_s[wm + 16 * i + l16][k]);
        if constexpr (!AR) avi[i] = *reinterpret_cast<const Vec<C, 4>*>(&Ai_s[wm + 16 * i + l16][k]);
        if constexpr (ROW) {
          bvr[i] = *reinterpret_cast<const Vec<C, 4>*>(&Br_s[wn + 16 * i + l16][k]);
          bvi[i] = *reinterpret_cast<const Vec<C, 4>*>(&Bi_s[wn + 16 * i + l16][k]);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            bvr[i].v[j] = Br_s[k + j][wn + 16 * i + l16];
            if constexpr (!BR) bvi[i].v[j] = Bi_s[k + j][wn + 16 * i + l16];
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if constexpr (G3) {
          C as[2], bs[2];
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            as[i] = avr[i].v[j] + avi[i].v[j];
            bs[i] = bvr[i].v[j] + bvi[i].v[j];
          }
#pragma unroll
          for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int ni = 0; ni < 2; ++ni) {
              if (!live[mi][ni]) continue;
              accr[mi][ni] = Mfma<C>::op(avr[mi].v[j], bvr[ni].v[j], accr[mi][ni]);
              accq[mi][ni] = Mfma<C>::op(avi[mi].v[j], bvi[ni].v[j], accq[mi][ni]);
              acci[mi][ni] = Mfma<C>::op(as[mi], bs[ni], acci[mi][ni]);
            }
          continue;
        }
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
          for (int ni = 0; ni < 2; ++ni) {
            if (!live[mi][ni]) continue;
            // re += Ar Br - Ai Bi ; im += Ar Bi + Ai Br
            accr[mi][ni] = Mfma<C>::op(avr[mi].v[j], bvr[ni].v[j], accr[mi][ni]);
            if constexpr (!AR && !BR) accr[mi][ni] = Mfma<C>::op(-avi[mi].v[j], bvi[ni].v[j], accr[mi][ni]);
            if constexpr (!OUTR) {
              if constexpr (!BR) acci[mi][ni] = Mfma<C>::op(avr[mi].v[j], bvi[ni].v[j], acci[mi][ni]);
              if constexpr (!AR) acci[mi][ni] = Mfma<C>::op(avi[mi].v[j], bvr[ni].v[j], acci[mi][ni]);
            }
          }
      }
    }
    __syncthreads();
  }
  if constexpr (G3) {
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) {
        const Acc p1 = accr[mi][ni], p2 = accq[mi][ni], p3 = acci[mi][ni];
        accr[mi][ni] = p1 - p2;
        acci[mi][ni] = p3 - p1 - p2;
      }
  }
  // complex P_D factors of this lane's rows and columns (indices clamped in range)
  double sxr[2] = {0.0, 0.0}, sxi[2] = {0.0, 0.0}, szr[2][4] = {}, szi[2][4] = {};
  if constexpr (!ROW) {
    if (sc.on) {
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) {
        const int col = min(n0 + wn + 16 * ni + l16, g.nc - 1);
        const int ix = col % sc.nx, jy = col / sc.nx;
        sxr[ni] = sc.lx[ix] + sc.ly[jy];
        sxi[ni] = cx.lxi[ix] + cx.lyi[jy];
      }
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = min(m0 + wm + 16 * mi + Mfma<C>::row(g4, i), n - 1);
          szr[mi][i] = sc.lz[m];
          szi[mi][i] = cx.lzi[m];
        }
    }
  }
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = m0 + wm + 16 * mi + Mfma<C>::row(g4, i);
        const int col = n0 + wn + 16 * ni + l16;
        C vr = accr[mi][ni][i], vi = OUTR ? C(0) : acci[mi][ni][i];
        if constexpr (!ROW) {
          if (sc.on) {  // (vr + i vi) / (dr + i di)
            const double dr = 1.0 - sc.sk * (sxr[ni] + szr[mi][i]);
            const double di = -sc.sk * (sxi[ni] + szi[mi][i]);
            const double den = dr * dr + di * di;
            const double xr = ((double)vr * dr + (double)vi * di) / den;
            const double xi = ((double)vi * dr - (double)vr * di) / den;
            vr = (C)xr;
            vi = (C)xi;
          }
        }
        size_t off;
        bool ok;
        if constexpr (ROW) {
          ok = m < g.nr && col < RO;
          off = (size_t)m * RO + col;
        } else {
          ok = m < n && col < g.nc;
          off = ok ? coff(m, col) : 0;
        }
        if (ok) {
          out_r[off] = (TO)vr;
          if constexpr (!OUTR) out_i[off] = (TO)vi;
        }
      }
}

// Host-side description of one axis: orthogonal symmetric eigenbasis Q (n x n, row-major) and
// eigenvalues lam of the unscaled 1-D second difference divided by h^2 (the caller multiplies
// them by kappa, so that the axis factor of sigma K is sigma lam).
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

// Periodic advection axis (h = 1/n): the 1-D factor nu D2 / h^2 - b D1 / h is circulant, so the
// unitary DFT Q_{aq} = e^{-2 pi i a q / n} / sqrt(n) diagonalises it, with eigenvalue (theta =
// 2 pi k / n) nu (2 cos theta - 2) / h^2 - |b| (1 - cos theta) / h - i b sin theta / h for the
// upwind difference (backward for b >= 0, forward for b < 0) and the same without the |b| term
// for the central difference.
inline void fdm_axis_dft(int n, bool central, double nu, double b, double* Qr, double* Qi,
                         double* lr, double* li) {
  const double pi = 3.14159265358979323846;
  const double h = 1.0 / n, s = 1.0 / std::sqrt((double)n);
  for (int a = 0; a < n; ++a)
    for (int q = 0; q < n; ++q) {
      const double th = 2.0 * pi * (double)(((long)a * q) % n) / n;
      Qr[(size_t)a * n + q] = s * std::cos(th);
      Qi[(size_t)a * n + q] = -s * std::sin(th);
    }
  for (int k = 0; k < n; ++k) {
    const double th = 2.0 * pi * k / n;
    lr[k] = nu * (2.0 * std::cos(th) - 2.0) / (h * h) - (central ? 0.0 : std::fabs(b) * (1.0 - std::cos(th)) / h);
    li[k] = -b * std::sin(th) / h;
  }
}

// ------------------------------------------------------------------------------------------
// CG with a preconditioner applied by separate launches (the contractions above): the
// residual update and the (r, z) product are split around the preconditioner.
// ------------------------------------------------------------------------------------------

// Start of a CG pass with an external preconditioner: r = LP(res / scale), (r, r); the tolerance and the
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
    ctl->tol = fmax(fmax(cfg.rtol * bn, cfg.atol / ctl->scale),
                    outer_target(cfg, ctl, ctl->scale));
    ctl->inner_conv = bn <= ctl->tol;
    ctl->inner_done = ctl->inner_conv || cfg.maxit <= 0;
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
    ctl->inner_conv = __builtin_isfinite(rr) && sqrt(rr) <= ctl->tol;
    ctl->inner_done = !__builtin_isfinite(rr) || ctl->inner_conv || its >= cfg.maxit;
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
    if (!__builtin_isfinite(rz)) {
      ctl->inner_done = 1;
      ctl->inner_conv = 0;
    }
  }
}

// ------------------------------------------------------------------------------------------
// GMRES with a preconditioner applied by separate launches: the Arnoldi kernels run without
// the fused block-Jacobi (the matrix-vector product reads z = P^-1 v_j of the stored vector j,
// applied between the launches), and the end of a cycle is split into the combination
// t = sum_i y_i v_i, z = P^-1 t, y += scale z.
// ------------------------------------------------------------------------------------------

// Least-squares solution of the cycle (back substitution of the rotated Hessenberg system)
// and t = sum_i ys_i vscale_i v_i in the compute type; counts the pass.
template <typename S, typename C, int VEC, int NDM>
__global__ __launch_bounds__(TPB) void k_gm_combine_ext(Launch ln, C* __restrict__ t,
                                                        const S* __restrict__ V, size_t vstride,
                                                        Ctl* ctl) {
  if (ctl->outer_done) return;
  const int J = ctl->J;
  count_work(ctl, KC_GM_FINISH, J);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (ctl->passes < MAXPASS) ctl->pass_iters[ctl->passes] = ctl->iters;
    ctl->passes += 1;
    ctl->life_passes += 1;
  }
  if (J == 0) return;
  if (J > NDM) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctl->nonfinite = 1;
      ctl->step_nonfinite = 1;
    }
    return;
  }
  __shared__ double ys[MAXM];
  if (threadIdx.x == 0) {
    for (int i = J - 1; i >= 0; --i) {
      double acc = ctl->g[i];
      for (int k = i + 1; k < J; ++k) acc -= ctl->H[k * (MAXM + 1) + i] * ys[k];
      const double d = ctl->H[i * (MAXM + 1) + i];
      ys[i] = (d != 0.0 && __builtin_isfinite(acc)) ? acc / d : 0.0;
    }
  }
  __syncthreads();
  C cf[NDM];
#pragma unroll
  for (int i = 0; i < NDM; ++i) cf[i] = i < J ? (C)(ys[i] * ctl->vscale[i]) : C(0);
  const int L = xcd_block(ln.G);
  for (int it = 0; it < ln.nit; ++it) {
    const int g = (L * ln.nit + it) * TPB + threadIdx.x;
    if (g >= ln.ng) break;
    const int e = g * VEC;
    C acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = C(0);
#pragma unroll
    for (int i = 0; i < NDM; ++i) {
      if (i < J) {
        C vv[VEC];
        loadv<C, S, VEC>(V + (size_t)i * vstride + e, vv);
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] += cf[i] * vv[v];
      }
    }
    storev<C, C, VEC>(t + e, acc);
  }
}

// y += scale z (z = P^-1 t in the compute type) when the cycle produced a correction.
template <typename C, int VEC>
__global__ __launch_bounds__(TPB) void k_gm_update_ext(Launch ln, double* __restrict__ y,
                                                       const C* __restrict__ z, Ctl* ctl) {
  if (ctl->outer_done || ctl->J == 0 || ctl->nonfinite) return;  // no correction, or J beyond the bound
  count_work(ctl, KC_PROMOTE);
  const double sc = ctl->scale;
  const int L = xcd_block(ln.G);
  for (int it = 0; it < ln.nit; ++it) {
    const int g = (L * ln.nit + it) * TPB + threadIdx.x;
    if (g >= ln.ng) break;
    double yv[VEC];
    C zv[VEC];
    loadv<double, double, VEC>(y + g * VEC, yv);
    loadv<C, C, VEC>(z + g * VEC, zv);
#pragma unroll
    for (int v = 0; v < VEC; ++v) yv[v] += sc * (double)zv[v];
    storev<double, double, VEC>(y + g * VEC, yv);
  }
}

}  // namespace mprk

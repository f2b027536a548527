// engine.hpp -- host-side launchers of the LP (low-precision) solve kernels, one instance per
// (storage type S, compute type C): (double, double), (float, float), (half, float).
// Each instance lives in its own translation unit so the three precisions compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "kernels.hpp"
#include "fdm.hpp"

namespace mprk {

// Optional per-launch event timing (bench/profiling).  Events are recorded on the launch
// stream immediately before and after each kernel of a class.
struct Profiler {
  hipStream_t stream = nullptr;
  std::vector<hipEvent_t> pool;
  struct Rec {
    int kc, e0, e1, n;  // n: launches between the two events
  };
  std::vector<Rec> recs;
  size_t used = 0;
  int cur_kc = -1, cur_e0 = -1, cur_n = 1;
  bool failed = false;
  int next() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        failed = true;
        return -1;
      }
      pool.push_back(e);
    }
    return (int)used++;
  }
  // n > 1: one event pair around n back-to-back launches of one class (event overhead would
  // otherwise dominate launches of a few microseconds)
  void before(int kc, int n = 1) {
    cur_kc = kc;
    cur_n = n;
    cur_e0 = next();
    if (cur_e0 >= 0 && hipEventRecord(pool[cur_e0], stream) != hipSuccess) failed = true;
  }
  void after() {
    const int e1 = next();
    if (e1 >= 0 && hipEventRecord(pool[e1], stream) != hipSuccess) failed = true;
    if (cur_e0 >= 0 && e1 >= 0) recs.push_back(Rec{cur_kc, cur_e0, e1, cur_n});
  }
  void reset() {
    recs.clear();
    used = 0;
    failed = false;
  }
  ~Profiler() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// What the engine needs to know about the problem and the workspace.
struct EngineCtx {
  Profiler* prof = nullptr;
  hipStream_t stream;
  Geo geo;
  int fmt;            // 0 stencil, 1 CSR
  int vec;            // values per group of the LP kernels: 8 (FP16, nx % 8 == 0), 4 or 1
  Launch ln_vec;      // groups of `vec` elements (streaming kernels)
  Launch ln_row;      // CSR rows (VEC = 1)
  Launch ln_mv;       // launch of the SpMV kernels (= ln_vec for stencil, ln_row for CSR)
  Launch ln_red;      // groups of `vec` elements, kernels with a grid reduction
  Launch ln_mv_red;   // SpMV kernels with a grid reduction
  int bs;             // block-Jacobi block size (0 = no preconditioner)
  Csr csr;
  const void* mval;   // LP CSR values of K / kscale (S)
  double kscale;
  Ctl* ctl;
  Red red;            // grid-reduction workspace
  // fast-diagonalisation preconditioner (fdm_on): per-axis eigenbasis (compute type, n x n),
  // eigenvalues of the axis second difference / h^2 (FP64), two compute-type scratch vectors
  int fdm_on;
  const void* fdm_Q[3];
  const double* fdm_lam[3];
  void* fdm_t[2];
  double kappa;
  double fdm_sigma;  // sigma of the solve in progress (the end-of-cycle preconditioner apply)
  // complex eigenbases (periodic advection operators): imaginary parts of the bases and
  // eigenvalues, imaginary halves of the two scratch vectors
  int fdm_cx;
  const void* fdm_Qi[3];
  const double* fdm_lami[3];
  void* fdm_ti[2];
  // half spectrum along x (real data): fdm_half = frequencies kept (a multiple of 4, at most
  // nx; 0: full spectrum) and the x basis weighted for the real inverse (real, imaginary)
  int fdm_half;
  const void* fdm_Qw[2];
  // LP vectors (S*)
  void *r, *z, *p0, *p1, *q, *x;
  void* V;
  size_t vstride;     // elements between GMRES basis vectors
  void* Zb;           // GMRES with block-Jacobi, gather form: the stored preconditioned directions
                      // BJ(V_j), vstride apart (the cycle's end then combines them without the
                      // inverse); null: one direction buffer z
  int reorth;         // GMRES: second classical Gram-Schmidt pass (CGS2)
  // GMRES Arnoldi step form: 0 gather kernels, 1 product on z-marching tiles + update kernel,
  // 2 folded onto z-marching tiles (stencil, block-Jacobi or none); the tile launch, its LDS
  // bytes, the two product buffers of the folded form
  int gform;
  ZLaunch zl;
  size_t zlds;
  void* zw[2];
  double* res;        // FP64 residual
  double* y;          // FP64 stage solution
};

class Engine {
 public:
  virtual ~Engine() {}
  // setup
  // invert nslot diagonal blocks (block reps[i] into slot i; reps == nullptr: every block)
  // lay: row layout of a per-block table (0 row-major, else interleaved for lanes of lay rows);
  // atag/aoff (non-null): the adaptive-precision layout with per-chunk types and offsets
  virtual hipError_t bj_setup_stencil(const EngineCtx& c, const Coef<double>& Mc, void* dinv,
                                      int* fail, int nslot, const int* reps, int lay,
                                      const int* atag = nullptr, const long long* aoff = nullptr) = 0;
  virtual hipError_t bj_setup_csr(const EngineCtx& c, const double* kval, double sigma, void* dinv,
                                  int* fail, int nslot, const int* reps, int lay,
                                  const int* atag = nullptr, const long long* aoff = nullptr) = 0;
  virtual hipError_t csr_values(const EngineCtx& c, long nnz, const double* kval, void* out) = 0;
  // CG
  virtual hipError_t cg_begin(const EngineCtx& c, const SolveCfg& cfg, const BJDesc& dinv) = 0;
  virtual hipError_t cg_iter(const EngineCtx& c, const SolveCfg& cfg, const Coef<double>& Mc,
                             const BJDesc& dinv, int it) = 0;
  virtual hipError_t cg_finish(const EngineCtx& c) = 0;
  // z = P^-1 r with the fast-diagonalisation preconditioner for stage shift sigma (S storage)
  virtual hipError_t fdm_apply(const EngineCtx& c, double sigma, const void* r, void* z) = 0;
  // GMRES
  virtual hipError_t gm_begin(const EngineCtx& c, const SolveCfg& cfg, const BJDesc& dinv) = 0;
  // Arnoldi step k of the cycle (k = the device's j for every step that does work)
  virtual hipError_t gm_iter(const EngineCtx& c, const SolveCfg& cfg, const Coef<double>& Mc,
                             const BJDesc& dinv, int k) = 0;
  // nsteps: Arnoldi steps enqueued in this cycle (an upper bound on the device's J)
  virtual hipError_t gm_finish(const EngineCtx& c, const SolveCfg& cfg, const BJDesc& dinv,
                               int nsteps) = 0;
  // verification access
  virtual hipError_t apply_m(const EngineCtx& c, const Coef<double>& Mc, double sigma,
                             const void* x, void* y) = 0;
  virtual hipError_t apply_bj(const EngineCtx& c, const BJDesc& dinv, const void* x, void* y) = 0;
  virtual int elem_bytes() const = 0;
};

Engine* make_engine_fp64();
Engine* make_engine_fp32();
Engine* make_engine_fp16();
Engine* make_engine_cb16();  // FP16 storage, FP64 arithmetic
Engine* make_engine_cb32();  // FP32 storage, FP64 arithmetic

template <typename C>
inline Coef<C> cast_coef(const Coef<double>& a) {
  return Coef<C>{(C)a.c, (C)a.xm, (C)a.xp, (C)a.ym, (C)a.yp, (C)a.zm, (C)a.zp};
}

#define MPRK_LAUNCH_KC(c, kc, kern, ln, ...)                                            \
  do {                                                                                   \
    if ((c).prof) (c).prof->before(kc);                                                  \
    hipLaunchKernelGGL((kern), dim3((ln).G), dim3(TPB), 0, (c).stream, __VA_ARGS__);      \
    if ((c).prof) (c).prof->after();                                                     \
  } while (0)

// the same with `lds` bytes of dynamic shared memory and G workgroups
#define MPRK_LAUNCH_KC_LDS(c, kc, kern, G, lds, ...)                                    \
  do {                                                                                   \
    if ((c).prof) (c).prof->before(kc);                                                  \
    hipLaunchKernelGGL((kern), dim3(G), dim3(TPB), (lds), (c).stream, __VA_ARGS__);       \
    if ((c).prof) (c).prof->after();                                                     \
  } while (0)

template <typename S, typename C>
class EngineT final : public Engine {
  // 16-byte groups for 2-byte storage; wider types never use an 8-wide group
  static constexpr int V8 = sizeof(S) == 2 ? 8 : 4;
  // the block-Jacobi kernels' instantiation for the adaptive-precision layout (mode 4)
  template <int BS, typename F>
  static void with_ad(const BJDesc& d, F&& f) {
    if constexpr (BS > 0) {
      if (d.mode == 4) {
        f(IC<1>{});
        return;
      }
    }
    f(IC<0>{});
  }

 public:
  int elem_bytes() const override { return (int)sizeof(S); }

  hipError_t bj_setup_stencil(const EngineCtx& c, const Coef<double>& Mc, void* dinv, int* fail,
                              int nslot, const int* reps, int lay, const int* atag,
                              const long long* aoff) override {
    hipLaunchKernelGGL(k_bj_setup_stencil<S>, dim3((nslot + 127) / 128), dim3(128), 0, c.stream,
                       nslot, c.bs, c.geo, Mc, (S*)dinv, fail, reps, lay, atag, aoff);
    return hipGetLastError();
  }
  hipError_t bj_setup_csr(const EngineCtx& c, const double* kval, double sigma, void* dinv, int* fail,
                          int nslot, const int* reps, int lay, const int* atag,
                          const long long* aoff) override {
    hipLaunchKernelGGL(k_bj_setup_csr<S>, dim3((nslot + 127) / 128), dim3(128), 0, c.stream, nslot,
                       c.bs, c.geo.N, c.csr, kval, sigma, (S*)dinv, fail, reps, lay, atag, aoff);
    return hipGetLastError();
  }
  hipError_t csr_values(const EngineCtx& c, long nnz, const double* kval, void* out) override {
    const long nb = (nnz + 255) / 256;
    hipLaunchKernelGGL(k_csr_lp_values<S>, dim3((unsigned)nb), dim3(256), 0, c.stream, nnz, kval,
                       1.0 / c.kscale, (S*)out);
    return hipGetLastError();
  }

  // ---------------- CG ----------------
  template <int VEC, int BS>
  void cg_begin_t(const EngineCtx& c, const SolveCfg& cfg, const BJDesc& dinv) {
    S* z = BS > 0 ? (S*)c.z : (S*)c.r;
    with_ad<BS>(dinv, [&](auto ad) {
      constexpr int AD = decltype(ad)::value;
      MPRK_LAUNCH_KC(c, KC_CG_BEGIN, (k_cg_begin<S, C, VEC, BS, AD>), c.ln_red, c.ln_red, c.res, (S*)c.r, z,
                    bj_typed<S>(dinv), cfg, c.ctl, c.red);
    });
  }
  hipError_t cg_begin(const EngineCtx& c, const SolveCfg& cfg, const BJDesc& dinv) override {
    if (c.fdm_on) {
      dispatch_vec(c, [&](auto vec) {
        constexpr int VEC = decltype(vec)::value;
        MPRK_LAUNCH_KC(c, KC_CG_BEGIN, (k_cg_begin_ext<S, C, VEC>), c.ln_red, c.ln_red, c.res, (S*)c.r,
                       cfg, c.ctl, c.red);
      });
      fdm_apply(c, cfg.sigma, c.r, c.z);
      cg_rz_t<1>(c);
      return hipGetLastError();
    }
    dispatch_vec_bs(c, [&](auto vec, auto bs) { cg_begin_t<decltype(vec)::value, decltype(bs)::value>(c, cfg, dinv); });
    return hipGetLastError();
  }
  template <int BEGIN>
  void cg_rz_t(const EngineCtx& c) {
    dispatch_vec(c, [&](auto vec) {
      constexpr int VEC = decltype(vec)::value;
      MPRK_LAUNCH_KC(c, KC_CG_RZ, (k_cg_rz<S, C, VEC, BEGIN>), c.ln_red, c.ln_red, (const S*)c.r,
                     (const S*)c.z, c.ctl, c.red);
    });
  }

  template <int VEC, int FMT>
  void cg_dir_t(const EngineCtx& c, const SolveCfg& cfg, const Coef<double>& Mc, const S* z,
                const S* pold, S* pnew) {
    const Coef<C> M = cast_coef<C>(Mc);
    const C msig = (C)(cfg.sigma * c.kscale);
    MPRK_LAUNCH_KC(c, KC_CG_DIR, (k_cg_dir<S, C, VEC, FMT>), c.ln_mv_red, c.ln_mv_red, c.geo, M, c.csr,
                (const S*)c.mval, msig, z, pold, pnew, (S*)c.q, c.ctl, c.red);
  }
  template <int VEC, int BS>
  void cg_upd_t(const EngineCtx& c, const SolveCfg& cfg, const S* p, const BJDesc& dinv) {
    S* z = BS > 0 ? (S*)c.z : (S*)c.r;
    with_ad<BS>(dinv, [&](auto ad) {
      constexpr int AD = decltype(ad)::value;
      MPRK_LAUNCH_KC(c, KC_CG_UPD, (k_cg_upd<S, C, VEC, BS, AD>), c.ln_red, c.ln_red, (S*)c.x, p, (S*)c.r,
                    (const S*)c.q, z, bj_typed<S>(dinv), cfg, c.ctl, c.red);
    });
  }
  hipError_t cg_iter(const EngineCtx& c, const SolveCfg& cfg, const Coef<double>& Mc,
                     const BJDesc& dinv, int it) override {
    if (c.fdm_on && it > 0) {
      // z = P^-1 r and r.z of the previous update, issued at the start of the iteration that
      // reads them, so the last iteration enqueued in a pass leaves no apply behind it
      fdm_apply(c, cfg.sigma, c.r, c.z);
      cg_rz_t<0>(c);
    }
    const S* z = (c.bs > 0 || c.fdm_on) ? (const S*)c.z : (const S*)c.r;
    const S* pold = (it & 1) ? (const S*)c.p1 : (const S*)c.p0;
    S* pnew = (it & 1) ? (S*)c.p0 : (S*)c.p1;
    if (c.fmt == 1) cg_dir_t<1, 1>(c, cfg, Mc, z, pold, pnew);
    else if (c.vec == 8) cg_dir_t<V8, 0>(c, cfg, Mc, z, pold, pnew);
    else if (c.vec == 4) cg_dir_t<4, 0>(c, cfg, Mc, z, pold, pnew);
    else cg_dir_t<1, 0>(c, cfg, Mc, z, pold, pnew);
    if (c.fdm_on) {
      dispatch_vec(c, [&](auto vec) {
        constexpr int VEC = decltype(vec)::value;
        MPRK_LAUNCH_KC(c, KC_CG_UPD, (k_cg_upd_ext<S, C, VEC>), c.ln_red, c.ln_red, (S*)c.x,
                       (const S*)pnew, (S*)c.r, (const S*)c.q, cfg, c.ctl, c.red);
      });
      return hipGetLastError();
    }
    dispatch_vec_bs(c, [&](auto vec, auto bs) {
      cg_upd_t<decltype(vec)::value, decltype(bs)::value>(c, cfg, pnew, dinv);
    });
    return hipGetLastError();
  }

  // ---------------- fast-diagonalisation preconditioner ----------------
  template <typename TI, typename TO, int V4, int BM, int KC>
  void fdm_launch(const EngineCtx& c, FdmGeo g, int row, const void* Q, const TI* in, TO* out,
                  const FdmScale& sc) {
    const int n = g.n;
    g.tiles = row ? ((g.nr + BM - 1) / BM) * ((n + FT_N - 1) / FT_N)
                  : ((n + BM - 1) / BM) * ((g.nc + FT_N - 1) / FT_N) * g.nb;
    const dim3 grid((unsigned)((g.tiles + 7) & ~7));
    if (row)
      hipLaunchKernelGGL((k_fdm_contract<TI, TO, C, 1, V4, BM, KC>), grid, dim3(256), 0, c.stream, g,
                         (const C*)Q, in, out, sc, c.ctl);
    else
      hipLaunchKernelGGL((k_fdm_contract<TI, TO, C, 0, V4, BM, KC>), grid, dim3(256), 0, c.stream, g,
                         (const C*)Q, in, out, sc, c.ctl);
  }
  // the data operand is read 4 elements at a time when its rows have a multiple of 4 elements
  template <typename TI, typename TO>
  void fdm_go(const EngineCtx& c, const FdmGeo& g, int row, const void* Q, const TI* in, TO* out,
              const FdmScale& sc) {
    if (c.geo.nx % 4 == 0) fdm_launch<TI, TO, 1, 64, FT_KC>(c, g, row, Q, in, out, sc);
    else fdm_launch<TI, TO, 0, 64, FT_KC>(c, g, row, Q, in, out, sc);
  }
  template <typename TI, typename TO>
  void fdm_row(const EngineCtx& c, int n, int nr, const void* Q, const TI* in, TO* out, int skip = 1) {
    const FdmGeo g{n, fdm_ldq(n), nr, 0, 0, 0, 1, 0, skip};
    const FdmScale none{nullptr, nullptr, nullptr, 0.0, 1, 0};
    fdm_go<TI, TO>(c, g, 1, Q, in, out, none);
  }
  void fdm_col(const EngineCtx& c, int n, int nc, int ld, long bstride, int nb, const void* Q,
               const C* in, C* out, const FdmScale& sc, int skip = 1) {
    const FdmGeo g{n, fdm_ldq(n), 0, nc, ld, bstride, nb, 0, skip};
    fdm_go<C, C>(c, g, 0, Q, in, out, sc);
  }
  // complex-basis contractions: V4 dispatch as for the real ones
  template <typename TI, typename TO, int INR, int OUTR, int V4>
  void fdm_launch_cx(const EngineCtx& c, FdmGeo g, int row, const FdmCx& cx, const TI* in_r,
                     const TI* in_i, TO* out_r, TO* out_i, const FdmScale& sc) {
    const int n = g.n;
    const int ro = g.ro ? g.ro : n;
    g.tiles = row ? ((g.nr + 63) / 64) * ((ro + FT_N - 1) / FT_N)
                  : ((n + 63) / 64) * ((g.nc + FT_N - 1) / FT_N) * g.nb;
    const dim3 grid((unsigned)((g.tiles + 7) & ~7));
    if (row)
      hipLaunchKernelGGL((k_fdm_contract_cx<TI, TO, C, 1, V4, INR, OUTR>), grid, dim3(256), 0,
                         c.stream, g, cx, in_r, in_i, out_r, out_i, sc, c.ctl);
    else
      hipLaunchKernelGGL((k_fdm_contract_cx<TI, TO, C, 0, V4, INR, OUTR>), grid, dim3(256), 0,
                         c.stream, g, cx, in_r, in_i, out_r, out_i, sc, c.ctl);
  }
  template <typename TI, typename TO, int INR, int OUTR>
  void fdm_go_cx(const EngineCtx& c, const FdmGeo& g, int row, const FdmCx& cx, const TI* in_r,
                 const TI* in_i, TO* out_r, TO* out_i, const FdmScale& sc) {
    if (c.geo.nx % 4 == 0) fdm_launch_cx<TI, TO, INR, OUTR, 1>(c, g, row, cx, in_r, in_i, out_r, out_i, sc);
    else fdm_launch_cx<TI, TO, INR, OUTR, 0>(c, g, row, cx, in_r, in_i, out_r, out_i, sc);
  }
  // z = Re(conj(U) P_D^-1 U r), U the 3-D unitary DFT (axis by axis), for the circulant factors
  // of the periodic advection operators; planar complex scratch (t0, t0i), (t1, t1i).  The data
  // are real and the symbol is conjugate-symmetric, so the x frequencies k and nx - k carry
  // conjugate values throughout: only k < H = fdm_half pass through the y and z contractions,
  // and the last one sums them with weight 2 for 0 < k < nx / 2 (1 for k = 0 and k = nx / 2,
  // 0 from nx / 2 + 1 on; the weights are in fdm_Qw).
  template <typename TI, typename TO>
  void fdm_chain_cx(const EngineCtx& c, double sigma, const TI* in, TO* out, int skip) {
    if (c.fdm_half) {
      fdm_chain_cx_half<TI, TO>(c, sigma, in, out, skip);
      return;
    }
    const int nx = c.geo.nx, ny = c.geo.ny, nz = c.geo.nz;
    C* t0 = (C*)c.fdm_t[0];
    C* t1 = (C*)c.fdm_t[1];
    C* t0i = (C*)c.fdm_ti[0];
    C* t1i = (C*)c.fdm_ti[1];
    const FdmScale none{nullptr, nullptr, nullptr, 0.0, nx, 0};
    const FdmScale sc{c.fdm_lam[0], c.fdm_lam[1], c.fdm_lam[2], sigma, nx, 1};
    auto cxd = [&](int d, double sign) {
      return FdmCx{c.fdm_Q[d], c.fdm_Qi[d], sign, c.fdm_lami[0], c.fdm_lami[1], c.fdm_lami[2]};
    };
    const FdmGeo gx{nx, fdm_ldq(nx), ny * nz, 0, 0, 0, 1, 0, skip};
    const FdmGeo gy{ny, fdm_ldq(ny), 0, nx, nx, (long)nx * ny, nz, 0, skip};
    const FdmGeo gz{nz, fdm_ldq(nz), 0, nx * ny, nx * ny, 0, 1, 0, skip};
    if (c.prof) c.prof->before(KC_FDM, 6);
    fdm_go_cx<TI, C, 1, 0>(c, gx, 1, cxd(0, 1.0), in, nullptr, t0, t0i, none);
    fdm_go_cx<C, C, 0, 0>(c, gy, 0, cxd(1, 1.0), t0, t0i, t1, t1i, none);
    fdm_go_cx<C, C, 0, 0>(c, gz, 0, cxd(2, 1.0), t1, t1i, t0, t0i, sc);
    fdm_go_cx<C, C, 0, 0>(c, gz, 0, cxd(2, -1.0), t0, t0i, t1, t1i, none);
    fdm_go_cx<C, C, 0, 0>(c, gy, 0, cxd(1, -1.0), t1, t1i, t0, t0i, none);
    fdm_go_cx<C, TO, 0, 1>(c, gx, 1, cxd(0, -1.0), t0, t0i, out, nullptr, none);
    if (c.prof) c.prof->after();
  }
  template <typename TI, typename TO>
  void fdm_chain_cx_half(const EngineCtx& c, double sigma, const TI* in, TO* out, int skip) {
    const int nx = c.geo.nx, ny = c.geo.ny, nz = c.geo.nz, H = c.fdm_half;
    C* t0 = (C*)c.fdm_t[0];
    C* t1 = (C*)c.fdm_t[1];
    C* t0i = (C*)c.fdm_ti[0];
    C* t1i = (C*)c.fdm_ti[1];
    const FdmScale none{nullptr, nullptr, nullptr, 0.0, H, 0};
    const FdmScale sc{c.fdm_lam[0], c.fdm_lam[1], c.fdm_lam[2], sigma, H, 1};
    auto cxd = [&](int d, double sign) {
      return FdmCx{c.fdm_Q[d], c.fdm_Qi[d], sign, c.fdm_lami[0], c.fdm_lami[1], c.fdm_lami[2]};
    };
    const FdmCx xw{c.fdm_Qw[0], c.fdm_Qw[1], -1.0, c.fdm_lami[0], c.fdm_lami[1], c.fdm_lami[2]};
    FdmGeo gxf{nx, fdm_ldq(nx), ny * nz, 0, 0, 0, 1, 0, skip};
    gxf.rk = nx;
    gxf.ro = H;
    FdmGeo gxb{nx, fdm_ldq(nx), ny * nz, 0, 0, 0, 1, 0, skip};
    gxb.rk = H;
    gxb.ro = nx;
    // y: the nz batches of H columns folded into one contiguous index of H nz columns, so the
    // 64-wide column tiles do not each end a batch half empty
    FdmGeo gy{ny, fdm_ldq(ny), 0, H * nz, H, 0, 1, 0, skip};
    gy.cfold = H;
    gy.cstride = (long)H * ny;
    const FdmGeo gz{nz, fdm_ldq(nz), 0, H * ny, H * ny, 0, 1, 0, skip};
    if (c.prof) c.prof->before(KC_FDM, 6);
    fdm_go_cx<TI, C, 1, 0>(c, gxf, 1, cxd(0, 1.0), in, nullptr, t0, t0i, none);
    fdm_go_cx<C, C, 0, 0>(c, gy, 0, cxd(1, 1.0), t0, t0i, t1, t1i, none);
    fdm_go_cx<C, C, 0, 0>(c, gz, 0, cxd(2, 1.0), t1, t1i, t0, t0i, sc);
    fdm_go_cx<C, C, 0, 0>(c, gz, 0, cxd(2, -1.0), t0, t0i, t1, t1i, none);
    fdm_go_cx<C, C, 0, 0>(c, gy, 0, cxd(1, -1.0), t1, t1i, t0, t0i, none);
    fdm_go_cx<C, TO, 0, 1>(c, gxb, 1, xw, t0, t0i, out, nullptr, none);
    if (c.prof) c.prof->after();
  }
  // z = P^-1 r: T_R, T_M, T_L with the basis (its own inverse), P_D^-1, then back.  in and out
  // may be t1 (the chain never reads and writes one buffer in the same launch).  skip: the
  // launches return once the inner solve is done (inside a Krylov loop).
  template <typename TI, typename TO>
  void fdm_chain(const EngineCtx& c, double sigma, const TI* in, TO* out, int skip) {
    if (c.fdm_cx) {
      fdm_chain_cx<TI, TO>(c, sigma, in, out, skip);
      return;
    }
    const int nx = c.geo.nx, ny = c.geo.ny, nz = c.geo.nz;
    C* t0 = (C*)c.fdm_t[0];
    C* t1 = (C*)c.fdm_t[1];
    const FdmScale none{nullptr, nullptr, nullptr, 0.0, nx, 0};
    const FdmScale sc{c.fdm_lam[0], c.fdm_lam[1], c.fdm_lam[2], sigma, nx, 1};
    if (c.prof) c.prof->before(KC_FDM, 6);
    fdm_row<TI, C>(c, nx, ny * nz, c.fdm_Q[0], in, t0, skip);
    fdm_col(c, ny, nx, nx, (long)nx * ny, nz, c.fdm_Q[1], t0, t1, none, skip);
    fdm_col(c, nz, nx * ny, nx * ny, 0, 1, c.fdm_Q[2], t1, t0, sc, skip);
    fdm_col(c, nz, nx * ny, nx * ny, 0, 1, c.fdm_Q[2], t0, t1, none, skip);
    fdm_col(c, ny, nx, nx, (long)nx * ny, nz, c.fdm_Q[1], t1, t0, none, skip);
    fdm_row<C, TO>(c, nx, ny * nz, c.fdm_Q[0], t0, out, skip);
    if (c.prof) c.prof->after();
  }
  hipError_t fdm_apply(const EngineCtx& c, double sigma, const void* r, void* z) override {
    fdm_chain<S, S>(c, sigma, (const S*)r, (S*)z, 1);
    return hipGetLastError();
  }
  hipError_t cg_finish(const EngineCtx& c) override {
    if (c.vec == 8)
      MPRK_LAUNCH_KC(c, KC_PROMOTE, (k_promote<S, C, V8>), c.ln_vec, c.ln_vec, c.y, (const S*)c.x, c.ctl);
    else if (c.vec == 4)
      MPRK_LAUNCH_KC(c, KC_PROMOTE, (k_promote<S, C, 4>), c.ln_vec, c.ln_vec, c.y, (const S*)c.x, c.ctl);
    else
      MPRK_LAUNCH_KC(c, KC_PROMOTE, (k_promote<S, C, 1>), c.ln_vec, c.ln_vec, c.y, (const S*)c.x, c.ctl);
    return hipGetLastError();
  }

  // ---------------- GMRES ----------------
  template <int VEC, int BS>
  void gm_begin_t(const EngineCtx& c, const SolveCfg& cfg, const BJDesc& dinv) {
    with_ad<BS>(dinv, [&](auto ad) {
      constexpr int AD = decltype(ad)::value;
      MPRK_LAUNCH_KC(c, KC_GM_BEGIN, (k_gm_begin<S, C, VEC, BS, AD>), c.ln_red, c.ln_red, c.res, (S*)c.V,
                       (S*)(c.Zb ? c.Zb : c.z), bj_typed<S>(dinv), cfg, c.ctl, c.red);
    });
  }
  hipError_t gm_begin(const EngineCtx& c, const SolveCfg& cfg, const BJDesc& dinv) override {
    dispatch_vec_bs(c, [&](auto vec, auto bs) { gm_begin_t<decltype(vec)::value, decltype(bs)::value>(c, cfg, dinv); });
    if (c.fdm_on) fdm_chain<S, S>(c, cfg.sigma, (const S*)c.V, (S*)c.z, 1);  // z = P^-1 v_0
    return hipGetLastError();
  }
  template <int VEC, int FMT, int PREC, int NDM>
  void gm_matvec_t(const EngineCtx& c, const SolveCfg& cfg, const Coef<double>& Mc) {
    const Coef<C> M = cast_coef<C>(Mc);
    const C msig = (C)(cfg.sigma * c.kscale);
    MPRK_LAUNCH_KC(c, KC_GM_MATVEC, (k_gm_matvec<S, C, VEC, FMT, PREC, NDM>), c.ln_mv_red, c.ln_mv_red, c.geo, M, c.csr,
                (const S*)c.mval, msig, (const S*)(c.Zb ? c.Zb : c.z), c.Zb ? c.vstride : (size_t)0,
                (S*)c.V, c.vstride, cfg, c.ctl, c.red);
  }
  template <int VEC, int BS, int NDM>
  void gm_orth_t(const EngineCtx& c, const SolveCfg& cfg, const BJDesc& dinv) {
    with_ad<BS>(dinv, [&](auto ad) {
      constexpr int AD = decltype(ad)::value;
      MPRK_LAUNCH_KC(c, KC_GM_ORTH, (k_gm_orth<S, C, VEC, BS, NDM, AD>), c.ln_red, c.ln_red, (S*)c.V, c.vstride,
                       (S*)(c.Zb ? c.Zb : c.z), c.Zb ? c.vstride : (size_t)0, bj_typed<S>(dinv), cfg,
                       c.ctl, c.red);
    });
  }
  // folded steps on z-marching tiles (c.vec is 4 or 8 there)
  template <int VEC>
  void gm_zfirst_t(const EngineCtx& c, const SolveCfg& cfg, const Coef<double>& Mc) {
    const Coef<C> M = cast_coef<C>(Mc);
    const S* zin = c.bs > 0 ? (const S*)c.z : (const S*)c.V;
    MPRK_LAUNCH_KC_LDS(c, KC_GM_MATVEC, (k_gm_zfirst<S, C, VEC>), c.zl.G, c.zlds, c.zl, c.geo, M, zin,
                       (const S*)c.V, (S*)c.zw[0], cfg, c.ctl, c.red);
  }
  template <int VEC, int BS, int NDM>
  void gm_zstep_t(const EngineCtx& c, const SolveCfg& cfg, const Coef<double>& Mc, const BJDesc& dinv,
                  int k) {
    const Coef<C> M = cast_coef<C>(Mc);
    with_ad<BS>(dinv, [&](auto ad) {
      constexpr int AD = decltype(ad)::value;
      MPRK_LAUNCH_KC_LDS(c, KC_GM_STEP, (k_gm_zstep<S, C, VEC, BS, NDM, AD>), c.zl.G, c.zlds, c.zl, c.geo, M,
                           (S*)c.V, c.vstride, (const S*)c.zw[(k - 1) & 1], (S*)c.zw[k & 1],
                           bj_typed<S>(dinv), cfg, c.ctl, c.red);
    });
  }
  template <int NDM>
  void gm_zstep_n(const EngineCtx& c, const SolveCfg& cfg, const Coef<double>& Mc, const BJDesc& dinv,
                  int k) {
    dispatch_vec_bs(c, [&](auto vec, auto bs) {
      constexpr int V = decltype(vec)::value;
      if constexpr (V > 1) gm_zstep_t<V, decltype(bs)::value, NDM>(c, cfg, Mc, dinv, k);
    });
  }
  void gm_ziter(const EngineCtx& c, const SolveCfg& cfg, const Coef<double>& Mc, const BJDesc& dinv,
                int k) {
    if (k == 0) {
      dispatch_vec(c, [&](auto vec) {
        constexpr int V = decltype(vec)::value;
        if constexpr (V > 1) gm_zfirst_t<V>(c, cfg, Mc);
      });
    } else if (k < 4) {
      gm_zstep_n<4>(c, cfg, Mc, dinv, k);
    } else if (k < 8) {
      gm_zstep_n<8>(c, cfg, Mc, dinv, k);
    } else if (k < 16) {
      gm_zstep_n<16>(c, cfg, Mc, dinv, k);
    } else {
      gm_zstep_n<MAXD>(c, cfg, Mc, dinv, k);
    }
  }
  template <int NDM>
  void gm_zclose_n(const EngineCtx& c, const SolveCfg& cfg, int nsteps) {
    dispatch_vec(c, [&](auto vec) {
      constexpr int V = decltype(vec)::value;
      MPRK_LAUNCH_KC(c, KC_GM_CLOSE, (k_gm_zclose<S, C, V, NDM>), c.ln_red, c.ln_red, (const S*)c.V,
                     c.vstride, (const S*)c.zw[(nsteps - 1) & 1], cfg, c.ctl, c.red);
    });
  }
  template <int NDM>
  void gm_iter_t(const EngineCtx& c, const SolveCfg& cfg, const Coef<double>& Mc, const BJDesc& dinv) {
    const bool prec = c.bs > 0 || c.fdm_on;  // the product reads z = P^-1 v_j
    if (c.gform == 1) {
      const Coef<C> M = cast_coef<C>(Mc);
      dispatch_vec(c, [&](auto vec) {
        constexpr int V = decltype(vec)::value;
        if constexpr (V > 1) {
          if (prec)
            MPRK_LAUNCH_KC_LDS(c, KC_GM_MATVEC, (k_gm_zmatvec<S, C, V, 1, NDM>), c.zl.G, c.zlds, c.zl,
                               c.geo, M, (const S*)c.z, (S*)c.V, c.vstride, cfg, c.ctl, c.red);
          else
            MPRK_LAUNCH_KC_LDS(c, KC_GM_MATVEC, (k_gm_zmatvec<S, C, V, 0, NDM>), c.zl.G, c.zlds, c.zl,
                               c.geo, M, (const S*)c.z, (S*)c.V, c.vstride, cfg, c.ctl, c.red);
        }
      });
    } else if (c.fmt == 1) {
      if (prec) gm_matvec_t<1, 1, 1, NDM>(c, cfg, Mc); else gm_matvec_t<1, 1, 0, NDM>(c, cfg, Mc);
    } else if (c.vec == 8) {
      if (prec) gm_matvec_t<V8, 0, 1, NDM>(c, cfg, Mc); else gm_matvec_t<V8, 0, 0, NDM>(c, cfg, Mc);
    } else if (c.vec == 4) {
      if (prec) gm_matvec_t<4, 0, 1, NDM>(c, cfg, Mc); else gm_matvec_t<4, 0, 0, NDM>(c, cfg, Mc);
    } else {
      if (prec) gm_matvec_t<1, 0, 1, NDM>(c, cfg, Mc); else gm_matvec_t<1, 0, 0, NDM>(c, cfg, Mc);
    }
    if (c.reorth) {
      dispatch_vec(c, [&](auto vec) {
        constexpr int V = decltype(vec)::value;
        MPRK_LAUNCH_KC(c, KC_GM_REORTH, (k_gm_reorth<S, C, V, NDM>), c.ln_red, c.ln_red, (S*)c.V,
                       c.vstride, cfg, c.ctl, c.red);
      });
    }
    dispatch_vec_bs(c, [&](auto vec, auto bs) {
      gm_orth_t<decltype(vec)::value, decltype(bs)::value, NDM>(c, cfg, dinv);
    });
  }
  hipError_t gm_iter(const EngineCtx& c, const SolveCfg& cfg, const Coef<double>& Mc,
                     const BJDesc& dinv, int k) override {
    // z = P^-1 v_k, issued at the start of the step that reads it (v_0's comes with the
    // begin), so the last step enqueued in a pass leaves no apply behind it; the launches
    // return once the cycle has ended
    if (c.gform == 2) {
      gm_ziter(c, cfg, Mc, dinv, k);
      return hipGetLastError();
    }
    if (c.fdm_on && k > 0 && k <= cfg.m)
      fdm_chain<S, S>(c, cfg.sigma, (const S*)c.V + (size_t)k * c.vstride, (S*)c.z, 1);
    // smallest compiled bound on the basis size that covers step k
    if (k < 4) gm_iter_t<4>(c, cfg, Mc, dinv);
    else if (k < 8) gm_iter_t<8>(c, cfg, Mc, dinv);
    else if (k < 16) gm_iter_t<16>(c, cfg, Mc, dinv);
    else gm_iter_t<MAXD>(c, cfg, Mc, dinv);
    return hipGetLastError();
  }
  template <int VEC, int BS, int NDM>
  void gm_finish_t(const EngineCtx& c, const BJDesc& dinv) {
    with_ad<BS>(dinv, [&](auto ad) {
      constexpr int AD = decltype(ad)::value;
      MPRK_LAUNCH_KC(c, KC_GM_FINISH, (k_gm_finish<S, C, VEC, BS, NDM, AD>), c.ln_vec, c.ln_vec, c.y, (const S*)c.V,
                    c.vstride, bj_typed<S>(dinv), c.ctl);
    });
  }
  template <int NDM>
  void gm_finish_n(const EngineCtx& c, const BJDesc& dinv) {
    if (c.fdm_on) {
      // t = sum_i y_i v_i -> t1; z = P^-1 t (also after the cycle's end) -> t1; y += scale z
      C* t1 = (C*)c.fdm_t[1];
      dispatch_vec(c, [&](auto vec) {
        constexpr int V = decltype(vec)::value;
        MPRK_LAUNCH_KC(c, KC_GM_FINISH, (k_gm_combine_ext<S, C, V, NDM>), c.ln_vec, c.ln_vec, t1,
                       (const S*)c.V, c.vstride, c.ctl);
      });
      fdm_chain<C, C>(c, c.fdm_sigma, t1, t1, 0);
      dispatch_vec(c, [&](auto vec) {
        constexpr int V = decltype(vec)::value;
        MPRK_LAUNCH_KC(c, KC_PROMOTE, (k_gm_update_ext<C, V>), c.ln_vec, c.ln_vec, c.y, t1, c.ctl);
      });
      return;
    }
    if (c.Zb) {
      // y += scale * sum_i ysol_i vscale_i BJ(V_i): the stored directions, no inverse read
      dispatch_vec(c, [&](auto vec) {
        constexpr int V = decltype(vec)::value;
        MPRK_LAUNCH_KC(c, KC_GM_FINISH, (k_gm_finish<S, C, V, 0, NDM, 0>), c.ln_vec, c.ln_vec, c.y,
                       (const S*)c.Zb, c.vstride, BJ<S>{}, c.ctl);
      });
      return;
    }
    dispatch_vec_bs(c, [&](auto vec, auto bs) {
      gm_finish_t<decltype(vec)::value, decltype(bs)::value, NDM>(c, dinv);
    });
  }
  hipError_t gm_finish(const EngineCtx& c, const SolveCfg& cfg, const BJDesc& dinv,
                       int nsteps) override {
    if (c.gform == 2 && nsteps > 0) {  // the cycle's last column
      if (nsteps <= 4) gm_zclose_n<4>(c, cfg, nsteps);
      else if (nsteps <= 8) gm_zclose_n<8>(c, cfg, nsteps);
      else if (nsteps <= 16) gm_zclose_n<16>(c, cfg, nsteps);
      else gm_zclose_n<MAXD>(c, cfg, nsteps);
    }
    if (nsteps <= 4) gm_finish_n<4>(c, dinv);
    else if (nsteps <= 8) gm_finish_n<8>(c, dinv);
    else if (nsteps <= 16) gm_finish_n<16>(c, dinv);
    else gm_finish_n<MAXM>(c, dinv);
    return hipGetLastError();
  }

  // ---------------- verification ----------------
  template <int VEC, int FMT>
  void apply_m_t(const EngineCtx& c, const Coef<double>& Mc, double sigma, const void* x, void* y) {
    const Coef<C> M = cast_coef<C>(Mc);
    const C msig = (C)(sigma * c.kscale);
    MPRK_LAUNCH_KC(c, KC_APPLY64, (k_apply_lp<S, C, VEC, FMT>), c.ln_mv, c.ln_mv, c.geo, M, c.csr,
                (const S*)c.mval, msig, (const S*)x, (S*)y);
  }
  hipError_t apply_m(const EngineCtx& c, const Coef<double>& Mc, double sigma, const void* x,
                     void* y) override {
    if (c.fmt == 1) apply_m_t<1, 1>(c, Mc, sigma, x, y);
    else if (c.vec == 8) apply_m_t<V8, 0>(c, Mc, sigma, x, y);
    else if (c.vec == 4) apply_m_t<4, 0>(c, Mc, sigma, x, y);
    else apply_m_t<1, 0>(c, Mc, sigma, x, y);
    return hipGetLastError();
  }
  template <int VEC, int BS>
  void apply_bj_t(const EngineCtx& c, const BJDesc& dinv, const void* x, void* y) {
    if constexpr (BS > 0) {
      with_ad<BS>(dinv, [&](auto ad) {
        constexpr int AD = decltype(ad)::value;
        MPRK_LAUNCH_KC(c, KC_APPLY64, (k_bj_apply<S, C, VEC, BS, AD>), c.ln_vec, c.ln_vec, (const S*)x,
                       (S*)y, bj_typed<S>(dinv));
      });
    }
  }
  hipError_t apply_bj(const EngineCtx& c, const BJDesc& dinv, const void* x, void* y) override {
    if (c.bs == 0) return hipErrorInvalidValue;
    dispatch_vec_bs(c, [&](auto vec, auto bs) { apply_bj_t<decltype(vec)::value, decltype(bs)::value>(c, dinv, x, y); });
    return hipGetLastError();
  }

 private:
  template <int V>
  struct IC {
    static constexpr int value = V;
  };
  template <typename F>
  static void dispatch_vec(const EngineCtx& c, F&& f) {
    if (c.vec == 8) f(IC<V8>{});
    else if (c.vec == 4) f(IC<4>{});
    else f(IC<1>{});
  }
  template <typename F>
  static void dispatch_vec_bs(const EngineCtx& c, F&& f) {
    if (c.vec == 8) {
      switch (c.bs) {
        case 0: f(IC<V8>{}, IC<0>{}); break;
        case 1: f(IC<V8>{}, IC<1>{}); break;
        case 2: f(IC<V8>{}, IC<2>{}); break;
        case 4: f(IC<V8>{}, IC<4>{}); break;
        default: f(IC<V8>{}, IC<8>{}); break;
      }
    } else if (c.vec == 4) {
      switch (c.bs) {
        case 0: f(IC<4>{}, IC<0>{}); break;
        case 1: f(IC<4>{}, IC<1>{}); break;
        case 2: f(IC<4>{}, IC<2>{}); break;
        case 4: f(IC<4>{}, IC<4>{}); break;
        default: f(IC<4>{}, IC<8>{}); break;
      }
    } else {
      switch (c.bs) {
        case 0: f(IC<1>{}, IC<0>{}); break;
        case 1: f(IC<1>{}, IC<1>{}); break;
        case 2: f(IC<1>{}, IC<2>{}); break;
        case 4: f(IC<1>{}, IC<4>{}); break;
        default: f(IC<1>{}, IC<8>{}); break;
      }
    }
  }
};

}  // namespace mprk

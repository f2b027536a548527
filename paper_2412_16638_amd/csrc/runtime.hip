// runtime.hip -- the C ABI of include/mprk.h: problem set-up, workspace layout, operator
// assembly, and the host driver that enqueues one time step and steers the Krylov loops by
// polling the 64-byte device control head.
//
// The DIRK step (eq. RKstep) is organised as in the paper's implementation: explicit
// operations and stage vectors in FP64, implicit stage systems (eq. corelinear) solved in the
// low precision after converting the right-hand side, result converted back (Section
// "Implementation of the Mixed-precision Runge--Kutta methods").  Here the conversion is of
// the FP64 stage residual, and the stage is repeated until the FP64 residual meets
// outer_tol (refine_max = 0 keeps the paper's single conversion).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/mprk.h"
#include "engine.hpp"
#include "runtime_internal.hpp"

using namespace mprk;

// launch with optional per-kernel event timing (member functions of mprk_handle)
#define PLAUNCH(kc, ...)                   \
  do {                                     \
    if (prof_on) prof.before(kc);          \
    hipLaunchKernelGGL(__VA_ARGS__);       \
    if (prof_on) prof.after();             \
  } while (0)

#define HIPCHK(x)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      return set_error(MPRK_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));   \
  } while (0)

namespace mprk {
static_assert((int)KC_COUNT == (int)MPRK_KC_COUNT, "kernel classes of the C ABI and the device");

thread_local std::string g_err;

int set_error(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

Launch make_launch_nit(long ng, int nit) {
  long G = (ng + (long)nit * TPB - 1) / ((long)nit * TPB);
  G = std::max(8L, (G + 7) / 8 * 8);
  return Launch{(int)ng, nit, (int)G};
}

Launch make_launch(long ng) {
  const long target_blocks = 2048;  // 8 resident 256-thread blocks on each of 256 CUs
  long nit = (ng + (long)TPB * target_blocks - 1) / ((long)TPB * target_blocks);
  nit = std::max(1L, std::min(nit, 8L));
  long G = (ng + nit * TPB - 1) / (nit * TPB);
  G = std::max(8L, (G + 7) / 8 * 8);
  return Launch{(int)ng, (int)nit, (int)G};
}

// 7-point coefficients of K (FP64): K u = kc u + sum_d (km_d u[-e_d] + kp_d u[+e_d]).
Coef<double> operator_coef(const mprk_grid& g, const mprk_operator& op) {
  const int n[3] = {g.nx, g.ny, g.nz};
  double km[3], kp[3], kc = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double h = g.bc == MPRK_BC_DIRICHLET0 ? 1.0 / (n[d] + 1) : 1.0 / n[d];
    const double b = op.kind == MPRK_OP_HEAT ? 0.0 : op.b[d];
    const double dif = op.diff / (h * h);
    if (op.kind == MPRK_OP_CENTRAL) {  // - b (u_{i+1} - u_{i-1}) / (2h)
      km[d] = dif + b / (2.0 * h);
      kp[d] = dif - b / (2.0 * h);
      kc -= 2.0 * dif;
    } else {                           // upwind: backward for b >= 0, forward for b < 0
      km[d] = dif + (b >= 0.0 ? b / h : 0.0);
      kp[d] = dif + (b < 0.0 ? -b / h : 0.0);
      kc -= 2.0 * dif + std::fabs(b) / h;
    }
  }
  return Coef<double>{kc, km[0], kp[0], km[1], kp[1], km[2], kp[2]};
}

// M = I - sigma K
Coef<double> stage_coef(const Coef<double>& K, double sigma) {
  return Coef<double>{1.0 - sigma * K.c, -sigma * K.xm, -sigma * K.xp, -sigma * K.ym,
                      -sigma * K.yp,     -sigma * K.zm, -sigma * K.zp};
}

// Entries of row r of K from the stencil: sorted columns, duplicates merged (periodic axes
// with fewer than 3 points), exact zeros dropped.  Returns the count (<= 7).
static int csr_row_entries(const Geo& geo, const Coef<double>& K, int r, int* col, double* val) {
  const bool per = geo.bc == MPRK_BC_PERIODIC;
  const int x = r % geo.nx, t = r / geo.nx, y = t % geo.ny, z = t / geo.ny;
  int ne = 0;
  auto add = [&](int c, double v) {
    for (int i = 0; i < ne; ++i)
      if (col[i] == c) {
        val[i] += v;
        return;
      }
    col[ne] = c;
    val[ne] = v;
    ++ne;
  };
  add(r, K.c);
  if (x > 0) add(r - 1, K.xm); else if (per) add(r + geo.nx - 1, K.xm);
  if (x < geo.nx - 1) add(r + 1, K.xp); else if (per) add(r - geo.nx + 1, K.xp);
  if (y > 0) add(r - geo.nx, K.ym); else if (per) add(r + (geo.ny - 1) * geo.nx, K.ym);
  if (y < geo.ny - 1) add(r + geo.nx, K.yp); else if (per) add(r - (geo.ny - 1) * geo.nx, K.yp);
  if (z > 0) add(r - geo.plane, K.zm); else if (per) add(r + (geo.nz - 1) * geo.plane, K.zm);
  if (z < geo.nz - 1) add(r + geo.plane, K.zp); else if (per) add(r - (geo.nz - 1) * geo.plane, K.zp);
  for (int i = 1; i < ne; ++i) {  // insertion sort by column
    const int c = col[i];
    const double v = val[i];
    int k = i - 1;
    while (k >= 0 && col[k] > c) {
      col[k + 1] = col[k];
      val[k + 1] = val[k];
      --k;
    }
    col[k + 1] = c;
    val[k + 1] = v;
  }
  int m = 0;
  for (int i = 0; i < ne; ++i)
    if (val[i] != 0.0) {
      col[m] = col[i];
      val[m] = val[i];
      ++m;
    }
  return m;
}

// Number of stored entries and max |K_ij| of the CSR form of K.
long csr_count(const Geo& geo, const Coef<double>& K, double* maxabs) {
  long nnz = 0;
  double mx = 0.0;
  int c[7];
  double v[7];
  for (int r = 0; r < geo.N; ++r) {
    const int m = csr_row_entries(geo, K, r, c, v);
    nnz += m;
    for (int i = 0; i < m; ++i) mx = std::max(mx, std::fabs(v[i]));
  }
  if (maxabs) *maxabs = mx;
  return nnz;
}

// Host CSR assembly of K from the stencil.
void assemble_csr(const Geo& geo, const Coef<double>& K, std::vector<int>& rowptr,
                  std::vector<int>& col, std::vector<double>& val) {
  const int N = geo.N;
  rowptr.assign((size_t)N + 1, 0);
  const long nnz = csr_count(geo, K, nullptr);
  col.resize((size_t)nnz);
  val.resize((size_t)nnz);
  long pos = 0;
  for (int r = 0; r < N; ++r) {
    const int m = csr_row_entries(geo, K, r, col.data() + pos, val.data() + pos);
    pos += m;
    rowptr[(size_t)r + 1] = (int)pos;
  }
}

// Distinct diagonal blocks of M = I - sigma K (block size bs, lexicographic blocks).  reps[i] is
// the first block with the i-th distinct value set; idx[b] the distinct slot of block b.  The key
// is the exact FP64 block, so equal keys give equal inverses.
static void bj_dedup(const Geo& geo, const Coef<double>& K, double sigma, int bs,
                     std::vector<int>& reps, std::vector<int>& idx) {
  const int N = geo.N;
  const int nblk = (N + bs - 1) / bs;
  reps.clear();
  idx.assign((size_t)nblk, 0);
  std::unordered_map<std::string, int> seen;
  std::string key, last_key;
  int last = -1;
  int c[7];
  double v[7];
  for (int b = 0; b < nblk; ++b) {
    const int r0 = b * bs, n = std::min(bs, N - r0);
    double D[BJ_MAX * BJ_MAX] = {};
    for (int i = 0; i < n; ++i) {
      D[i * BJ_MAX + i] += 1.0;
      const int m = csr_row_entries(geo, K, r0 + i, c, v);
      for (int e = 0; e < m; ++e)
        if (c[e] >= r0 && c[e] < r0 + n) D[i * BJ_MAX + (c[e] - r0)] -= sigma * v[e];
    }
    key.assign((const char*)D, sizeof(D));
    key.push_back((char)n);
    if (last >= 0 && key == last_key) {
      idx[(size_t)b] = last;
      continue;
    }
    auto it = seen.find(key);
    int slot;
    if (it == seen.end()) {
      slot = (int)reps.size();
      reps.push_back(b);
      seen.emplace(key, slot);
    } else {
      slot = it->second;
    }
    idx[(size_t)b] = slot;
    last = slot;
    last_key = key;
  }
}

// Adaptive-precision block-Jacobi layout (Ginkgo's adaptive block-Jacobi, cited in the
// Introduction: each diagonal block's inverse stored in the lowest precision its conditioning
// allows).  A block may be stored in a type of unit roundoff u when u * cond_1(D_b) <= tol
// (the rounding of the stored inverse then perturbs the preconditioned block by at most about
// tol) and its inverse's entries are within that type's range; FP8, FP16, FP32, FP64 in that
// order.
// The type is chosen per chunk of 64 lane groups of vec rows (the unit a wave reads), as the
// widest its blocks need.  Fills tag (per chunk) and aoff (per chunk byte offsets, plus the
// total at the end); the distinct blocks are found as for the shared-inverse table.
static void bj_adaptive_layout(const Geo& geo, const Coef<double>& K, double sigma, int bs, int vec,
                               double tol, std::vector<int>& tag, std::vector<long long>& aoff) {
  std::vector<int> reps, idx;
  bj_dedup(geo, K, sigma, bs, reps, idx);
  const int N = geo.N;
  std::vector<int> rtag(reps.size());
  int c[7];
  double v[7];
  for (size_t s = 0; s < reps.size(); ++s) {
    const int r0 = reps[s] * bs, n = std::min(bs, N - r0);
    double a[BJ_MAX][BJ_MAX] = {}, inv[BJ_MAX][BJ_MAX];
    for (int i = 0; i < n; ++i) {
      a[i][i] += 1.0;
      const int m = csr_row_entries(geo, K, r0 + i, c, v);
      for (int e = 0; e < m; ++e)
        if (c[e] >= r0 && c[e] < r0 + n) a[i][c[e] - r0] -= sigma * v[e];
    }
    double n1 = 0.0;
    for (int k = 0; k < n; ++k) {
      double cs = 0.0;
      for (int i = 0; i < n; ++i) cs += std::fabs(a[i][k]);
      n1 = std::max(n1, cs);
    }
    double a2[BJ_MAX][BJ_MAX];
    std::memcpy(a2, a, sizeof(a));
    int t = 3;
    if (!gj_invert(a2, inv, n)) {
      double ni = 0.0, mx = 0.0;
      for (int k = 0; k < n; ++k) {
        double cs = 0.0;
        for (int i = 0; i < n; ++i) {
          cs += std::fabs(inv[i][k]);
          mx = std::max(mx, std::fabs(inv[i][k]));
        }
        ni = std::max(ni, cs);
      }
      const double kappa = n1 * ni;
      // FP8 (E4M3: unit roundoff 2^-4, largest finite 448, spacing 2^-9 below its smallest
      // normal 2^-6): an entry's error is at most max(2^-4 |x|, 2^-10), so the inverse's
      // relative 1-norm error adds n 2^-10 / ||D^-1||_1, i.e. n 2^-10 ||D||_1 to u kappa
      if (std::ldexp(1.0, -4) * kappa + std::ldexp(1.0, -10) * n * n1 <= tol && mx <= 448.0) t = 0;
      else if (std::ldexp(1.0, -11) * kappa <= tol && mx < 6.0e4) t = 1;
      else if (std::ldexp(1.0, -24) * kappa <= tol && mx < 1.0e38) t = 2;
    }
    rtag[s] = t;
  }
  const long rows = (long)bj_chunks((long)((N + bs - 1) / bs) * bs, vec);
  const int nch = (int)(rows / (64L * vec));
  const int nblk = (N + bs - 1) / bs;
  tag.assign((size_t)nch, 0);
  for (int b = 0; b < nblk; ++b) {
    const int ch = (int)(((long)b * bs / vec) >> 6);
    tag[(size_t)ch] = std::max(tag[(size_t)ch], rtag[(size_t)idx[(size_t)b]]);
  }
  aoff.assign((size_t)nch + 1, 0);
  const long long per = 64LL * vec * bs;  // entries per chunk
  for (int ch = 0; ch < nch; ++ch) {
    const long long bytes = per * (1LL << tag[(size_t)ch]);  // 1, 2, 4, 8 bytes per entry
    aoff[(size_t)ch + 1] = aoff[(size_t)ch] + ((bytes + 255) & ~255LL);
  }
}

}  // namespace mprk

// ------------------------------------------------------------------------------------------
// tableaus and defaults
// ------------------------------------------------------------------------------------------

extern "C" int32_t mprk_tableau_builtin(int32_t id, int32_t param, mprk_tableau* out) {
  if (!out) return set_error(MPRK_EINVAL, "mprk_tableau_builtin: out is NULL");
  std::memset(out, 0, sizeof(*out));
  auto HI = [&](int i, int j, double v) { out->a_hi[i * out->s + j] = v; };
  auto LO = [&](int i, int j, double v) { out->a_lo[i * out->s + j] = v; };
  switch (id) {
    case MPRK_TAB_SDIRK2: {  // Alexander's L-stable two-stage SDIRK, gamma = 1 - 1/sqrt(2)
      out->s = 2;
      const double g = 1.0 - 1.0 / std::sqrt(2.0);
      LO(0, 0, g);
      HI(1, 0, 1.0 - g);
      LO(1, 1, g);
      out->b[0] = 1.0 - g;
      out->b[1] = g;
      return MPRK_OK;
    }
    case MPRK_TAB_SDIRK3: {  // Alexander's L-stable three-stage SDIRK of order 3
      out->s = 3;
      const double g = 0.43586652150845899941601945;
      const double b1 = -1.5 * g * g + 4.0 * g - 0.25;
      const double b2 = 1.5 * g * g - 5.0 * g + 1.25;
      LO(0, 0, g);
      HI(1, 0, 0.5 * (1.0 - g));
      LO(1, 1, g);
      HI(2, 0, b1);
      HI(2, 1, b2);
      LO(2, 2, g);
      out->b[0] = b1;
      out->b[1] = b2;
      out->b[2] = g;
      return MPRK_OK;
    }
    case MPRK_TAB_MID: {  // implicit midpoint + `param` FP64 corrector steps (Appendix A)
      if (param < 0 || param > MPRK_MAX_STAGES - 1)
        return set_error(MPRK_EINVAL, "MID: corrector count must be in [0, 7]");
      out->s = param + 1;
      LO(0, 0, 0.5);
      for (int i = 1; i <= param; ++i) HI(i, i - 1, 0.5);
      out->b[param] = 1.0;
      return MPRK_OK;
    }
    case MPRK_TAB_4S3PA: {  // Table ButchertabA
      out->s = 4;
      LO(0, 0, 0.788675134594813);
      HI(1, 0, 0.211324865405187);
      HI(2, 0, 0.709495523817170);
      LO(2, 0, 0.051944240459852);
      HI(2, 1, -0.86531425061942);
      LO(2, 2, 0.788675134594813);
      HI(3, 0, 0.705123240545107);
      HI(3, 1, 0.943370088535775);
      HI(3, 2, -0.859818194486069);
      out->b[1] = 0.5;
      out->b[3] = 0.5;
      return MPRK_OK;
    }
    case MPRK_TAB_4S3PB: {  // Table ButchertabB, a42^(eps) = -3/2 - a42
      out->s = 4;
      for (int i = 0; i < 4; ++i) LO(i, i, 0.5);
      HI(1, 0, 2.543016042796356);
      LO(1, 0, -2.376349376129689);
      HI(2, 0, 2.451484396921318);
      LO(2, 0, -2.951484396921318);
      HI(2, 1, 0.024108961241221);
      LO(2, 1, 0.475891038758779);
      HI(3, 0, 2.073861819468268);
      LO(3, 0, -0.573861819468268);
      HI(3, 1, 2.367724727682735);
      LO(3, 1, -1.5 - 2.367724727682735);
      HI(3, 2, 1.711868223075524);
      LO(3, 2, -1.211868223075524);
      out->b[0] = 1.5;
      out->b[1] = -1.5;
      out->b[2] = 0.5;
      out->b[3] = 0.5;
      return MPRK_OK;
    }
    case MPRK_TAB_4S3PC: {  // Table ButchertabC
      out->s = 4;
      LO(0, 0, 0.511243008730995);
      LO(1, 0, -1.999347282862640);
      HI(1, 0, -0.050470366527530);
      LO(1, 1, 1.957161067302390);
      LO(2, 0, 0.443312893511937);
      HI(2, 0, 0.368613367355336);
      LO(2, 1, -0.573131033672219);
      HI(2, 1, 0.273504374252976);
      LO(2, 2, 0.128283796414019);
      LO(3, 0, -2.0);
      HI(3, 0, 1.803794668975043);
      LO(3, 1, -0.160330320741428);
      HI(3, 1, 0.097485042980759);
      LO(3, 2, 0.579597314161362);
      HI(3, 2, -1.895660952342050);
      LO(3, 3, 1.484688928981990);
      out->b[0] = 0.002837446974069;
      out->b[1] = 0.336264433650450;
      out->b[2] = 0.806376720267787;
      out->b[3] = -0.145478600892306;
      return MPRK_OK;
    }
    default:
      return set_error(MPRK_EINVAL, "unknown tableau id");
  }
}

extern "C" int32_t mprk_precisions_default(int32_t storage, int32_t krylov, mprk_precisions* out) {
  if (!out) return set_error(MPRK_EINVAL, "mprk_precisions_default: out is NULL");
  if (storage < MPRK_FP64 || storage > MPRK_FP16 || krylov < MPRK_CG || krylov > MPRK_GMRES)
    return set_error(MPRK_EINVAL, "mprk_precisions_default: bad storage or krylov");
  std::memset(out, 0, sizeof(*out));
  out->storage = storage;
  out->compute = storage == MPRK_FP64 ? MPRK_FP64 : MPRK_FP32;
  out->krylov = krylov;
  out->restart = 30;
  out->precond = MPRK_PRECOND_BJ;
  out->block = 8;
  out->atol = 0.0;
  out->strict = 0;
  out->reorth = 0;
  out->gm_form = MPRK_GMFORM_AUTO;
  if (storage == MPRK_FP64) {
    out->rtol = 1e-12;
    out->outer_tol = 1e-11;
    out->refine_max = krylov == MPRK_CG ? 4 : 20;
  } else if (storage == MPRK_FP32) {
    out->rtol = krylov == MPRK_CG ? 1e-5 : 1e-4;
    out->outer_tol = 1e-10;
    out->refine_max = krylov == MPRK_CG ? 8 : 20;
  } else {
    out->rtol = 1e-2;
    out->outer_tol = 1e-6;
    out->refine_max = 20;
  }
  out->maxit = krylov == MPRK_CG ? 1000 : 30;
  return MPRK_OK;
}

// ------------------------------------------------------------------------------------------
// create / layout
// ------------------------------------------------------------------------------------------

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static int validate(const mprk_grid* g, const mprk_operator* op, const mprk_tableau* tab,
                    const mprk_precisions* p, double dt) {
  if (!g || !op || !tab || !p) return set_error(MPRK_EINVAL, "NULL argument");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return set_error(MPRK_EINVAL, "grid extents must be >= 1");
  if (g->bc != MPRK_BC_DIRICHLET0 && g->bc != MPRK_BC_PERIODIC) return set_error(MPRK_EINVAL, "bad bc");
  const double N = (double)g->nx * g->ny * g->nz;
  if (N * 7.0 >= 2147483647.0) return set_error(MPRK_EINVAL, "grid too large for int32 indexing");
  if (op->kind != MPRK_OP_HEAT && op->kind != MPRK_OP_ADVDIFF && op->kind != MPRK_OP_CENTRAL)
    return set_error(MPRK_EINVAL, "bad operator kind");
  if (op->format != MPRK_FMT_STENCIL && op->format != MPRK_FMT_CSR) return set_error(MPRK_EINVAL, "bad format");
  if (!(op->diff >= 0.0) || !std::isfinite(op->diff)) return set_error(MPRK_EINVAL, "diffusion must be finite and >= 0");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(op->b[d])) return set_error(MPRK_EINVAL, "velocity must be finite");
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(MPRK_EINVAL, "dt must be > 0");
  if (tab->s < 1 || tab->s > MPRK_MAX_STAGES) return set_error(MPRK_EINVAL, "tableau stages must be in [1, 8]");
  for (int i = 0; i < tab->s; ++i) {
    for (int j = 0; j < tab->s; ++j) {
      const double a = tab->a_hi[i * tab->s + j] + tab->a_lo[i * tab->s + j];
      if (!std::isfinite(a)) return set_error(MPRK_EINVAL, "tableau entries must be finite");
      if (j > i && a != 0.0) return set_error(MPRK_EINVAL, "tableau must be lower triangular (DIRK)");
    }
    if (!std::isfinite(tab->b[i])) return set_error(MPRK_EINVAL, "tableau weights must be finite");
  }
  if (p->storage < MPRK_FP64 || p->storage > MPRK_FP16) return set_error(MPRK_EINVAL, "bad storage");
  if (p->compute != MPRK_FP64 && p->compute != MPRK_FP32) return set_error(MPRK_EINVAL, "bad compute");
  if (p->storage == MPRK_FP64 && p->compute != MPRK_FP64)
    return set_error(MPRK_EUNSUPPORTED, "FP64 storage needs FP64 compute");
  if (p->krylov != MPRK_CG && p->krylov != MPRK_GMRES) return set_error(MPRK_EINVAL, "bad krylov");
  if (p->krylov == MPRK_GMRES && (p->restart < 1 || p->restart > MPRK_MAX_RESTART))
    return set_error(MPRK_EINVAL, "GMRES restart must be in [1, 32]");
  if (p->precond != MPRK_PRECOND_NONE && p->precond != MPRK_PRECOND_BJ && p->precond != MPRK_PRECOND_FDM)
    return set_error(MPRK_EINVAL, "bad precond");
  if (p->precond == MPRK_PRECOND_FDM) {
    // implemented cases: the heat operator (real symmetric eigenbases) and the periodic
    // advection operators (circulant factors, the complex DFT basis), with CG or GMRES
    if (op->kind != MPRK_OP_HEAT && g->bc != MPRK_BC_PERIODIC)
      return set_error(MPRK_EUNSUPPORTED,
                       "fast-diagonalisation preconditioner for advection needs periodic boundaries");
  }
  if (p->precond == MPRK_PRECOND_BJ && !(p->block == 1 || p->block == 2 || p->block == 4 || p->block == 8))
    return set_error(MPRK_EINVAL, "block size must be 1, 2, 4 or 8");
  if (!(p->rtol >= 0.0) || !(p->atol >= 0.0) || !(p->outer_tol >= 0.0))
    return set_error(MPRK_EINVAL, "tolerances must be >= 0");
  if (p->maxit < 0 || p->refine_max < 0) return set_error(MPRK_EINVAL, "maxit and refine_max must be >= 0");
  if (p->krylov == MPRK_CG && op->kind != MPRK_OP_HEAT &&
      (op->b[0] != 0.0 || op->b[1] != 0.0 || op->b[2] != 0.0))
    return set_error(MPRK_EINVAL, "CG needs a symmetric operator; use GMRES for advection");
  if (p->reorth != 0 && p->reorth != 1) return set_error(MPRK_EINVAL, "reorth must be 0 or 1");
  if (p->gm_form < MPRK_GMFORM_AUTO || p->gm_form > MPRK_GMFORM_FOLDED)
    return set_error(MPRK_EINVAL, "gm_form must be one of the MPRK_GMFORM values");
  if (!(p->bj_adapt_tol >= 0.0)) return set_error(MPRK_EINVAL, "bj_adapt_tol must be >= 0");
  if (p->stage_start < MPRK_START_AUTO || p->stage_start > MPRK_START_EXTRAP)
    return set_error(MPRK_EINVAL, "stage_start must be one of the MPRK_START values");
  if (p->inner_stop < MPRK_STOP_AUTO || p->inner_stop > MPRK_STOP_RTOL)
    return set_error(MPRK_EINVAL, "inner_stop must be one of the MPRK_STOP values");
  if (p->bj_adapt_tol > 0.0 && p->bj_shared)
    return set_error(MPRK_EINVAL, "adaptive-precision block-Jacobi stores one inverse per block "
                                  "(bj_shared must be 0)");
  return MPRK_OK;
}

extern "C" int32_t mprk_create(const mprk_grid* grid, const mprk_operator* op,
                               const mprk_tableau* tab, const mprk_precisions* prec, double dt,
                               void* hip_stream, mprk_handle** out) {
  if (!out) return set_error(MPRK_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(grid, op, tab, prec, dt);
  if (rc) return rc;
  mprk_handle* h = new (std::nothrow) mprk_handle();
  if (!h) return set_error(MPRK_ENOMEM, "host allocation failed");
  rc = h->init(*grid, *op, *tab, *prec, dt, (hipStream_t)hip_stream);
  if (rc) {
    delete h;
    return rc;
  }
  if (prec->gm_form != MPRK_GMFORM_AUTO && prec->krylov == MPRK_GMRES &&
      !(h->gform_ok & (1 << (prec->gm_form - 1)))) {
    delete h;
    return set_error(MPRK_EUNSUPPORTED, "this GMRES step form needs the stencil format, whole groups "
                                        "per x-row (folded: also CGS1 and block-Jacobi or none)");
  }
  // pinned status records and events are made here when a device is present (a handle made
  // without one, e.g. to validate a problem, makes them at its first mprk_bind), so that
  // mprk_bind_static allocates nothing
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
    rc = h->make_device_resources();
    if (rc) {
      delete h;
      return rc;
    }
  } else {
    (void)hipGetLastError();
  }
  *out = h;
  return MPRK_OK;
}

int mprk_handle::init(const mprk_grid& g, const mprk_operator& o, const mprk_tableau& t,
                      const mprk_precisions& p, double dt_, hipStream_t s) {
  grid = g;
  op = o;
  tab = t;
  prec = p;
  dt = dt_;
  stream = s;
  geo = Geo{g.nx, g.ny, g.nz, g.bc, g.nx * g.ny * g.nz, g.nx * g.ny};
  N = geo.N;
  vec = (g.nx % 4 == 0) ? 4 : 1;
  vec_lp = (p.storage == MPRK_FP16 && g.nx % 8 == 0) ? 8 : vec;
  Kc = operator_coef(g, o);
  // FP64 arithmetic over FP32 / FP16 storage: the compressed-basis variants
  const bool cb = p.compute == MPRK_FP64 && p.storage != MPRK_FP64;
  switch (p.storage) {
    case MPRK_FP64: eng.reset(make_engine_fp64()); break;
    case MPRK_FP32: eng.reset(cb ? make_engine_cb32() : make_engine_fp32()); break;
    default: eng.reset(cb ? make_engine_cb16() : make_engine_fp16()); break;
  }
  lp_bytes = eng->elem_bytes();
  nstages = t.s;
  need_keps = false;
  sigmas.clear();
  for (int i = 0; i < t.s; ++i) {
    const double aii = t.a_hi[i * t.s + i] + t.a_lo[i * t.s + i];
    implicit_[i] = aii != 0.0;
    sig_idx[i] = -1;
    if (implicit_[i]) {
      const double sg = dt * aii;
      int k = -1;
      for (size_t q = 0; q < sigmas.size(); ++q)
        if (sigmas[q] == sg) k = (int)q;
      if (k < 0) {
        sigmas.push_back(sg);
        k = (int)sigmas.size() - 1;
      }
      sig_idx[i] = k;
    }
    for (int j = 0; j < i; ++j)
      if (t.a_lo[i * t.s + j] != 0.0 && (t.a_hi[j * t.s + j] + t.a_lo[j * t.s + j]) != 0.0)
        need_keps = true;
  }
  // launches
  ln_vec = make_launch(N / vec);
  ln_row = make_launch(N);
  // kernels with a grid reduction: one group per thread by default (the two-level reduction
  // keeps its cost independent of the number of blocks)
  ln_vec_red = make_launch_nit(N / vec, 1);
  ln_row_red = make_launch_nit(N, 1);
  ln_lp = make_launch(N / vec_lp);
  ln_lp_red = make_launch_nit(N / vec_lp, 1);
  // z-marching residual: about four workgroups per CU (planes per tile a power of two in
  // [ZM_LZ_MIN, 32]); the autotuner may switch to another tile depth or the gather kernel
  long zm_g_max = 0;
  if (o.format == MPRK_FMT_STENCIL && zmarch_fits(geo, vec)) {
    const ZLaunch z1 = make_zlaunch(geo, vec, 1);
    const long want = (long)z1.nty * geo.nz / 1024;
    int lz = ZM_LZ_MIN;
    while (lz < 32 && lz < want) lz *= 2;
    zm_lz = lz;
    zl_res = make_zlaunch(geo, vec, zm_lz);
    zm_g_max = make_zlaunch(geo, vec, ZM_LZ_MIN).G;
  }
  // GMRES Arnoldi step forms on z-marching tiles of the LP vectors
  bs = p.precond == MPRK_PRECOND_BJ ? p.block : 0;
  gform_ok = 1;  // the gather kernels always
  if (p.krylov == MPRK_GMRES && o.format == MPRK_FMT_STENCIL && zmarch_fits(geo, vec_lp)) {
    const ZLaunch z1 = make_zlaunch(geo, vec_lp, 1);
    const long want = (long)z1.nty * geo.nz / 1024;
    int lz = ZM_LZ_MIN;
    while (lz < 32 && lz < want) lz *= 2;
    zl_lp = make_zlaunch(geo, vec_lp, lz);
    zm_g_max = std::max(zm_g_max, (long)make_zlaunch(geo, vec_lp, ZM_LZ_MIN).G);
    gform_ok |= 2;
    const bool blocks_ok = bs == 0 || (g.nx % bs == 0 && (bs <= vec_lp || z1.gx % (bs / vec_lp) == 0));
    if (p.precond != MPRK_PRECOND_FDM && !p.reorth && blocks_ok) gform_ok |= 4;
  }
  // the library's choice: the gather kernels (measured fastest for the 256^3 FP16 step); the
  // autotuner times the tiled forms where they apply
  gform = p.gm_form == MPRK_GMFORM_AUTO ? 0 : p.gm_form - 1;
  // partials cover every reducing launch shape the autotuner may pick (nit >= 1)
  pstride = std::max({(long)ln_vec_red.G, (long)ln_row_red.G, (long)ln_lp_red.G, zm_g_max});
  pstride2 = (pstride + RGRP - 1) / RGRP;
  nblk = bs ? (N + bs - 1) / bs : 0;
  // CSR size (assembled at bind)
  nnz = 0;
  if (o.format == MPRK_FMT_CSR) {
    double mx = 0.0;
    nnz = csr_count(geo, Kc, &mx);
    kscale = mx > 0.0 ? std::ldexp(1.0, (int)std::ceil(std::log2(mx))) : 1.0;
  } else {
    kscale = 1.0;
  }
  // layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o2 = off;
    off += align256(bytes);
    return o2;
  };
  const size_t v64 = (size_t)N * 8;
  const size_t vlp = align256((size_t)N * lp_bytes);
  o_rhs = take(v64);
  o_y = take(v64);
  o_res = take(v64);
  o_k = take(v64 * nstages);
  o_keps = need_keps ? take(v64 * nstages) : 0;
  o_scr = take(v64);  // scratch FP64 vector (solve output of k, verification)
  fdm = p.precond == MPRK_PRECOND_FDM;
  // the fast-diagonalisation inverse is exact for the operators it accepts: one Krylov iteration
  // per pass, so no predicted iteration beyond the last solve's count
  predict_margin = fdm ? 0 : 1;
  // the start value of the stage solves (the automatic choice follows what saved outer passes):
  // with GMRES the previous stage's slope, and under the FDM preconditioner, whose passes reduce
  // the residual furthest, also the first stage from f(u); with CG (symmetric, diffusion
  // operators) the slopes extrapolated linearly in c, which the previous slope alone did not
  // make close enough; the FDM-preconditioned CG already needs one pass, and the one-solve
  // mode's result would depend on the start value
  start_mode = p.stage_start;
  if (start_mode == MPRK_START_AUTO) {
    start_mode = MPRK_START_RHS;
    if (p.refine_max > 0 && p.krylov == MPRK_GMRES)
      start_mode = fdm ? MPRK_START_SLOPE_EVAL : MPRK_START_SLOPE;
    else if (p.refine_max > 0 && !fdm)
      start_mode = MPRK_START_EXTRAP;
  }
  start_slope = start_mode >= MPRK_START_SLOPE;
  start_eval = start_mode == MPRK_START_SLOPE_EVAL || start_mode == MPRK_START_EXTRAP;
  start_first_eval = start_mode == MPRK_START_SLOPE_EVAL;
  start_extrap = start_mode == MPRK_START_EXTRAP;
  if (p.krylov == MPRK_CG) {
    o_r = take(vlp);
    o_z = (bs || fdm) ? take(vlp) : o_r;
    o_p0 = take(vlp);
    o_p1 = take(vlp);
    o_q = take(vlp);
    o_x = take(vlp);
    o_V = 0;
  } else {
    o_V = take(vlp * (size_t)(p.restart + 1));
    o_z = (bs || fdm) ? take(vlp) : 0;
    // the stored preconditioned directions BJ(V_0) .. BJ(V_m) of the gather form
    o_Zb = (bs && !fdm) ? take(vlp * (size_t)(p.restart + 1)) : 0;
    o_r = o_p0 = o_p1 = o_q = o_x = 0;
    if (gform_ok & 4) {  // folded form: products alternate between W0 and W1 (W1 reuses BJ(V_0)'s)
      o_w0 = take(vlp);
      o_w1 = bs ? o_z : take(vlp);
    }
  }
  vstride = vlp / lp_bytes;
  bjsets.assign(bs ? sigmas.size() : 0, BJSet());
  for (size_t q = 0; q < bjsets.size(); ++q) {
    BJSet& B = bjsets[q];
    if (p.bj_shared) {
      bj_dedup(geo, Kc, sigmas[q], bs, B.reps, B.idx);
      B.nslot = (int)B.reps.size();
      B.mode = B.nslot == 1 ? 2 : 1;
      if (B.mode == 2) B.idx.clear();
    } else {
      B.nslot = nblk;
      B.mode = p.bj_adapt_tol > 0.0 ? 4 : 3;  // rows interleaved for lanes of vec_lp rows
    }
    if (B.mode == 4) {
      bj_adaptive_layout(geo, Kc, sigmas[q], bs, vec_lp, p.bj_adapt_tol, B.tag, B.aoff);
      B.o_inv = take((size_t)B.aoff.back());
      B.aoff.pop_back();
      B.o_tag = take(B.tag.size() * 4);
      B.o_aoff = take(B.aoff.size() * 8);
      continue;
    }
    const size_t rows = B.mode == 3 ? std::max((size_t)nblk * bs, bj_chunks((long)nblk * bs, vec_lp))
                                    : (size_t)B.nslot * bs;
    B.o_inv = take(rows * bs * lp_bytes);
    if (B.table()) B.o_reps = take((size_t)B.nslot * 4);
    if (B.mode == 1) B.o_idx = take((size_t)nblk * 4);
  }
  if (o.format == MPRK_FMT_CSR) {
    o_rowptr = take((size_t)(N + 1) * 4);
    o_col = take((size_t)nnz * 4);
    o_kval = take((size_t)nnz * 8);
    o_mval = take((size_t)nnz * lp_bytes);
  }
  fdm_cx = fdm && o.kind != MPRK_OP_HEAT;
  if (fdm) {
    const size_t cb = p.compute == MPRK_FP64 ? 8 : 4;
    const int n3[3] = {g.nx, g.ny, g.nz};
    for (int d = 0; d < 3; ++d) {
      o_fdm_Q[d] = take((size_t)n3[d] * fdm_ldq(n3[d]) * cb);  // rows padded to fdm_ldq
      o_fdm_lam[d] = take((size_t)n3[d] * 8);
      if (fdm_cx) {
        o_fdm_Qi[d] = take((size_t)n3[d] * fdm_ldq(n3[d]) * cb);
        o_fdm_lami[d] = take((size_t)n3[d] * 8);
      }
    }
    for (int k = 0; k < 2; ++k) {
      o_fdm_t[k] = take((size_t)N * cb);
      if (fdm_cx) o_fdm_ti[k] = take((size_t)N * cb);
    }
    // real data: x frequencies 0 .. nx/2 suffice (rounded up to 4 for aligned rows; needs nx >= 4)
    const int H = (g.nx / 2 + 1 + 3) & ~3;
    fdm_half = fdm_cx && H <= g.nx ? H : 0;
    if (fdm_half)
      for (int k = 0; k < 2; ++k) o_fdm_Qw[k] = take((size_t)g.nx * fdm_ldq(g.nx) * cb);
  }
  o_ctl = take(sizeof(Ctl));
  o_flag = take(256);
  o_part = take((size_t)MAXRED * pstride * 8);
  o_part2 = take((size_t)MAXRED * pstride2 * 8);
  o_tick = take(red_ticks(pstride) * 4);
  ws_bytes = off;
  // per-sigma solve configurations
  cfgs.clear();
  for (double sg : sigmas) {
    SolveCfg c{};
    c.sigma = sg;
    c.outer_tol = p.outer_tol;
    c.max_passes = std::max(p.refine_max, 1);
    c.paper_mode = p.refine_max == 0;
    c.outer_stop = !c.paper_mode && (p.inner_stop == MPRK_STOP_OUTER ||
                                     (p.inner_stop == MPRK_STOP_AUTO && p.storage != MPRK_FP64));
    c.strict = p.strict != 0;
    c.rtol = p.rtol;
    c.atol = p.atol;
    c.m = p.krylov == MPRK_GMRES ? p.restart : 0;
    c.maxit = p.krylov == MPRK_GMRES ? std::min(p.maxit, p.restart) : p.maxit;
    c.sqrtN = std::sqrt((double)N);
    c.invN = 1.0 / (double)N;
    cfgs.push_back(c);
  }
  return MPRK_OK;
}

// Pinned poll slots and events: made on the first bind (the first call that needs a device).
int mprk_handle::make_device_resources() {
  if (events_made) return MPRK_OK;
  if (!slots) {
    HIPCHK(hipHostMalloc((void**)&slots, sizeof(CtlHead) * (NSLOT + MPRK_MAX_STAGES + 1)));
    std::memset(slots, 0, sizeof(CtlHead) * (NSLOT + MPRK_MAX_STAGES + 1));
  }
  for (int i = 0; i < NSLOT; ++i) HIPCHK(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
  HIPCHK(hipHostMalloc((void**)&rec_iters, sizeof(int) * MAXPASS * (MPRK_MAX_STAGES + 1)));
  for (int i = 0; i <= MPRK_MAX_STAGES; ++i)
    HIPCHK(hipEventCreateWithFlags(&rec_ev[i], hipEventDisableTiming));
  prof.stream = stream;
  events_made = true;
  return MPRK_OK;
}

mprk_handle::~mprk_handle() {
  if (events_made) {
    for (int i = 0; i < NSLOT; ++i) (void)hipEventDestroy(ev[i]);
    for (int i = 0; i <= MPRK_MAX_STAGES; ++i) (void)hipEventDestroy(rec_ev[i]);
  }
  if (slots) (void)hipHostFree(slots);
  if (rec_iters) (void)hipHostFree(rec_iters);
  graph_drop();
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
}

extern "C" int64_t mprk_workspace_bytes(const mprk_handle* h) {
  if (!h) return set_error(MPRK_EINVAL, "NULL handle");
  return (int64_t)h->ws_bytes;
}


EngineCtx mprk_handle::ctx() const {
  EngineCtx c{};
  c.prof = prof_on ? const_cast<Profiler*>(&prof) : nullptr;
  c.stream = stream;
  c.geo = geo;
  c.fmt = op.format;
  c.vec = vec_lp;
  c.ln_vec = ln_lp;
  c.ln_row = ln_row;
  c.ln_mv = op.format == MPRK_FMT_CSR ? ln_row : ln_lp;
  c.ln_red = ln_lp_red;
  c.ln_mv_red = op.format == MPRK_FMT_CSR ? ln_row_red : ln_lp_red;
  c.bs = bs;
  c.csr = Csr{(const int*)(ws + o_rowptr), (const int*)(ws + o_col)};
  c.mval = ws + o_mval;
  c.kscale = kscale;
  c.ctl = (Ctl*)(ws + o_ctl);
  c.red = red();
  c.fdm_on = fdm ? 1 : 0;
  for (int d = 0; d < 3; ++d) {
    c.fdm_Q[d] = fdm ? ws + o_fdm_Q[d] : nullptr;
    c.fdm_lam[d] = fdm ? (const double*)(ws + o_fdm_lam[d]) : nullptr;
  }
  c.fdm_t[0] = fdm ? ws + o_fdm_t[0] : nullptr;
  c.fdm_t[1] = fdm ? ws + o_fdm_t[1] : nullptr;
  c.fdm_cx = fdm_cx ? 1 : 0;
  for (int d = 0; d < 3; ++d) {
    c.fdm_Qi[d] = fdm_cx ? ws + o_fdm_Qi[d] : nullptr;
    c.fdm_lami[d] = fdm_cx ? (const double*)(ws + o_fdm_lami[d]) : nullptr;
  }
  for (int k = 0; k < 2; ++k) c.fdm_ti[k] = fdm_cx ? ws + o_fdm_ti[k] : nullptr;
  c.fdm_half = fdm_half;
  for (int k = 0; k < 2; ++k) c.fdm_Qw[k] = fdm_half ? ws + o_fdm_Qw[k] : nullptr;
  c.kappa = op.diff;
  c.r = ws + o_r;
  c.z = ws + o_z;
  c.p0 = ws + o_p0;
  c.p1 = ws + o_p1;
  c.q = ws + o_q;
  c.x = ws + o_x;
  c.V = ws + o_V;
  c.vstride = vstride;
  c.Zb = (o_Zb && gform == 0) ? ws + o_Zb : nullptr;
  c.reorth = prec.krylov == MPRK_GMRES && prec.reorth;
  c.gform = gform;
  c.zl = zl_lp;
  c.zlds = gform ? zmarch_lds(geo, zl_lp, prec.compute == MPRK_FP64 ? 8 : 4) : 0;
  c.zw[0] = (gform_ok & 4) ? ws + o_w0 : nullptr;
  c.zw[1] = (gform_ok & 4) ? ws + o_w1 : nullptr;
  c.res = (double*)(ws + o_res);
  c.y = (double*)(ws + o_y);
  return c;
}

// Attach u and a workspace and run the setup kernels.  Allocates no device or pinned memory
// itself (the pinned records exist once make_device_resources has run).
static int bind_impl(mprk_handle* h, double* u_dev, void* workspace_dev) {
  h->graph_epoch += 1;  // new state and workspace addresses
  h->u = u_dev;
  h->ws = (char*)workspace_dev;
  h->bound = false;
  HIPCHK(hipMemsetAsync(h->ws + h->o_ctl, 0, sizeof(Ctl), h->stream));
  HIPCHK(hipMemsetAsync(h->ws + h->o_flag, 0, 256, h->stream));
  HIPCHK(hipMemsetAsync(h->ws + h->o_tick, 0, red_ticks(h->pstride) * 4, h->stream));
  // the device counters restart from zero with the control record
  h->good_base = 0;
  h->bad_base = 0;
  h->missed_base = 0;
  h->held_base = 0;
  EngineCtx c = h->ctx();
  if (h->op.format == MPRK_FMT_CSR) {
    std::vector<int> rp, cl;
    std::vector<double> vl;
    assemble_csr(h->geo, h->Kc, rp, cl, vl);
    if ((long)cl.size() != h->nnz) return set_error(MPRK_EINVAL, "CSR size mismatch");
    HIPCHK(hipMemcpyAsync(h->ws + h->o_rowptr, rp.data(), rp.size() * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->ws + h->o_col, cl.data(), cl.size() * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->ws + h->o_kval, vl.data(), vl.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h->eng->csr_values(c, h->nnz, (const double*)(h->ws + h->o_kval), h->ws + h->o_mval));
    HIPCHK(hipStreamSynchronize(h->stream));  // host vectors go out of scope
  }
  int* fail = (int*)(h->ws + h->o_flag);
  for (size_t q = 0; q < h->bjsets.size(); ++q) {
    const mprk_handle::BJSet& B = h->bjsets[q];
    void* dinv = h->ws + B.o_inv;
    const int* reps = nullptr;
    if (B.table()) {
      HIPCHK(hipMemcpyAsync(h->ws + B.o_reps, B.reps.data(), B.reps.size() * 4, hipMemcpyHostToDevice, h->stream));
      reps = (const int*)(h->ws + B.o_reps);
    }
    if (B.mode == 1)
      HIPCHK(hipMemcpyAsync(h->ws + B.o_idx, B.idx.data(), B.idx.size() * 4, hipMemcpyHostToDevice, h->stream));
    const int* atag = nullptr;
    const long long* aoff = nullptr;
    if (B.mode == 4) {
      HIPCHK(hipMemcpyAsync(h->ws + B.o_tag, B.tag.data(), B.tag.size() * 4, hipMemcpyHostToDevice, h->stream));
      HIPCHK(hipMemcpyAsync(h->ws + B.o_aoff, B.aoff.data(), B.aoff.size() * 8, hipMemcpyHostToDevice,
                            h->stream));
      atag = (const int*)(h->ws + B.o_tag);
      aoff = (const long long*)(h->ws + B.o_aoff);
    }
    const int lay = (B.mode == 3 || B.mode == 4) ? h->vec_lp : 0;
    if (h->op.format == MPRK_FMT_CSR)
      HIPCHK(h->eng->bj_setup_csr(c, (const double*)(h->ws + h->o_kval), h->sigmas[q], dinv, fail,
                                  B.nslot, reps, lay, atag, aoff));
    else
      HIPCHK(h->eng->bj_setup_stencil(c, stage_coef(h->Kc, h->sigmas[q]), dinv, fail, B.nslot, reps,
                                      lay, atag, aoff));
  }
  if (h->fdm) {
    // fast-diagonalisation: per-axis eigenbasis (compute type, rows padded with zeros to
    // fdm_ldq) and eigenvalues (FP64); complex for the periodic advection operators
    const int n3[3] = {h->grid.nx, h->grid.ny, h->grid.nz};
    const bool f64 = h->prec.compute == MPRK_FP64;
    auto upload = [&](size_t off, const std::vector<double>& Q, int n) -> int {
      const int ldq = fdm_ldq(n);
      std::vector<double> Qp((size_t)n * ldq, 0.0);
      for (int a = 0; a < n; ++a)
        for (int q = 0; q < n; ++q) Qp[(size_t)a * ldq + q] = Q[(size_t)a * n + q];
      if (f64) {
        HIPCHK(hipMemcpyAsync(h->ws + off, Qp.data(), Qp.size() * 8, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
      } else {
        std::vector<float> Qf(Qp.begin(), Qp.end());
        HIPCHK(hipMemcpyAsync(h->ws + off, Qf.data(), Qf.size() * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));  // Qf goes out of scope
      }
      return MPRK_OK;
    };
    for (int d = 0; d < 3; ++d) {
      const int n = n3[d];
      std::vector<double> Q((size_t)n * n), lam(n);
      if (!h->fdm_cx) {
        fdm_axis_basis(n, h->grid.bc == MPRK_BC_PERIODIC, Q.data(), lam.data());
        for (auto& l : lam) l *= h->op.diff;  // the axis factor of sigma K is sigma lam
        int rc = upload(h->o_fdm_Q[d], Q, n);
        if (rc) return rc;
      } else {
        std::vector<double> Qi((size_t)n * n), lami(n);
        fdm_axis_dft(n, h->op.kind == MPRK_OP_CENTRAL, h->op.diff, h->op.b[d], Q.data(), Qi.data(),
                     lam.data(), lami.data());
        int rc = upload(h->o_fdm_Q[d], Q, n);
        if (!rc) rc = upload(h->o_fdm_Qi[d], Qi, n);
        if (rc) return rc;
        if (d == 0 && h->fdm_half) {
          // weights of the real inverse over frequencies 0 .. n/2: 2 where k and n - k are
          // distinct, 1 at k = 0 and (n even) k = n/2, 0 above n/2
          std::vector<double> Wr((size_t)n * n, 0.0), Wi((size_t)n * n, 0.0);
          for (int a = 0; a < n; ++a)
            for (int q = 0; q <= n / 2; ++q) {
              const double w = (q == 0 || 2 * q == n) ? 1.0 : 2.0;
              Wr[(size_t)a * n + q] = w * Q[(size_t)a * n + q];
              Wi[(size_t)a * n + q] = w * Qi[(size_t)a * n + q];
            }
          rc = upload(h->o_fdm_Qw[0], Wr, n);
          if (!rc) rc = upload(h->o_fdm_Qw[1], Wi, n);
          if (rc) return rc;
        }
        HIPCHK(hipMemcpyAsync(h->ws + h->o_fdm_lami[d], lami.data(), lami.size() * 8, hipMemcpyHostToDevice, h->stream));
      }
      HIPCHK(hipMemcpyAsync(h->ws + h->o_fdm_lam[d], lam.data(), lam.size() * 8, hipMemcpyHostToDevice, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
    }
  }
  int hfail = 0;
  HIPCHK(hipMemcpyAsync(&hfail, fail, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (hfail) return set_error(MPRK_EINVAL, "singular block-Jacobi block");
  h->bound = true;
  return MPRK_OK;
}

extern "C" int32_t mprk_bind(mprk_handle* h, double* u_dev, void* workspace_dev, int64_t bytes) {
  if (!h || !u_dev || !workspace_dev) return set_error(MPRK_EINVAL, "NULL argument");
  if (bytes < (int64_t)h->ws_bytes) return set_error(MPRK_ENOMEM, "workspace smaller than mprk_workspace_bytes");
  if (((uintptr_t)workspace_dev & 255) != 0) return set_error(MPRK_EINVAL, "workspace must be 256-byte aligned");
  if (((uintptr_t)u_dev & 31) != 0) return set_error(MPRK_EINVAL, "u must be 32-byte aligned");
  int rc0 = h->make_device_resources();
  if (rc0) return rc0;
  h->static_dev = -1;
  return bind_impl(h, u_dev, workspace_dev);
}

// ------------------------------------------------------------------------------------------
// the library's static device scratch (for callers that cannot allocate)
// ------------------------------------------------------------------------------------------

// One copy per device, held from the library's load on that device until the process ends.
static __device__ __align__(256) char scratch[MPRK_STATIC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
struct ScratchSlot {
  char* ptr = nullptr;          // this device's copy of `scratch` (from hipGetSymbolAddress)
  unsigned long long gen = 0;   // static binds on this device so far
};
std::map<int, ScratchSlot> g_scratch;  // device ordinal -> slot
}  // namespace

// A handle bound to the static scratch stays valid until another handle binds it on the same
// device; later calls on the older handle then fail instead of reading the newer one's data.
int mprk_handle::check_ws() const {
  if (static_dev < 0) return MPRK_OK;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(static_dev);
  if (it == g_scratch.end() || it->second.gen != static_gen)
    return set_error(MPRK_ESTATE, "the static scratch of this device was bound by another handle "
                                  "since this handle's mprk_bind_static");
  return MPRK_OK;
}

extern "C" int32_t mprk_bind_static(mprk_handle* h, double* u_dev) {
  if (!h || !u_dev) return set_error(MPRK_EINVAL, "NULL argument");
  if (((uintptr_t)u_dev & 31) != 0) return set_error(MPRK_EINVAL, "u must be 32-byte aligned");
  if (h->ws_bytes > (size_t)MPRK_STATIC_SCRATCH_BYTES)
    return set_error(MPRK_ENOMEM, "workspace of " + std::to_string(h->ws_bytes) +
                                      " bytes exceeds the static scratch of " +
                                      std::to_string((long long)MPRK_STATIC_SCRATCH_BYTES) + " bytes");
  if (!h->events_made)
    return set_error(MPRK_ESTATE, "handle created without a device: mprk_bind_static cannot make "
                                  "its pinned status records");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  char* ptr = nullptr;
  unsigned long long gen = 0;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ScratchSlot& sl = g_scratch[dev];
    if (!sl.ptr) {
      // first use on this device, with it current: the address of this device's copy; the
      // symbol's own name is a host-side stand-in and is never passed to a kernel or a copy
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return set_error(MPRK_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      sl.ptr = (char*)p;
    }
    ptr = sl.ptr;
    gen = ++sl.gen;
  }
  h->static_dev = dev;
  h->static_gen = gen;
  return bind_impl(h, u_dev, ptr);
}

// ------------------------------------------------------------------------------------------
// polling
// ------------------------------------------------------------------------------------------

int mprk_handle::poll_enqueue(int* slot) {
  const int s = slot_next;
  slot_next = (slot_next + 1) % NSLOT;
  // the slot's previous copy must have landed before it is overwritten
  if (slot_used[s]) HIPCHK(hipEventSynchronize(ev[s]));
  HIPCHK(hipMemcpyAsync(&slots[s], ws + o_ctl, sizeof(CtlHead), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipEventRecord(ev[s], stream));
  slot_used[s] = true;
  *slot = s;
  return MPRK_OK;
}

int mprk_handle::poll_wait(int s, CtlHead* out) {
  HIPCHK(hipEventSynchronize(ev[s]));
  std::atomic_thread_fence(std::memory_order_acquire);
  std::memcpy(out, (const void*)&slots[s], sizeof(*out));
  return MPRK_OK;
}

int mprk_handle::stage_record(int slot) {
  Ctl* ctl = (Ctl*)(ws + o_ctl);
  HIPCHK(hipMemcpyAsync(&slots[NSLOT + slot], ctl, sizeof(CtlHead), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(rec_iters + slot * MAXPASS, ctl->pass_iters, sizeof(int) * MAXPASS,
                        hipMemcpyDeviceToHost, stream));
  HIPCHK(hipEventRecord(rec_ev[slot], stream));
  rec_pending[slot] = true;
  return MPRK_OK;
}

// Fold the last record of `slot` into its history (waits for the record's copy, which has
// normally landed long before).
int mprk_handle::update_hist(int slot) {
  if (!rec_pending[slot]) return MPRK_OK;
  HIPCHK(hipEventSynchronize(rec_ev[slot]));
  std::atomic_thread_fence(std::memory_order_acquire);
  rec_pending[slot] = false;
  CtlHead hd;
  std::memcpy(&hd, (const void*)&slots[NSLOT + slot], sizeof(hd));
  StageHist& H = hist[slot];
  if (hd.nonfinite || !hd.converged || hd.passes <= 0 || hd.passes > MAXPASS) {
    H.valid = false;
    return MPRK_OK;
  }
  H.valid = true;
  H.passes = hd.passes;
  for (int p = 0; p < hd.passes; ++p) H.iters[p] = rec_iters[slot * MAXPASS + p];
  return MPRK_OK;
}

// ------------------------------------------------------------------------------------------
// the stage solve (outer FP64 residual loop around the LP Krylov solve)
// ------------------------------------------------------------------------------------------

Red mprk_handle::red() const {
  return Red{(double*)(ws + o_part), (double*)(ws + o_part2), (unsigned int*)(ws + o_tick), pstride,
             pstride2};
}

BJDesc mprk_handle::bj_desc(int si) const {
  if (!bs || si < 0 || si >= (int)bjsets.size()) return BJDesc{nullptr, nullptr, 0};
  const BJSet& B = bjsets[si];
  return BJDesc{ws + B.o_inv, B.mode == 1 ? (const int*)(ws + B.o_idx) : nullptr, B.mode,
                B.mode == 4 ? (const int*)(ws + B.o_tag) : nullptr,
                B.mode == 4 ? (const long long*)(ws + B.o_aoff) : nullptr};
}

int mprk_handle::launch_residual(const SolveCfg& cfg, const double* rhs, double* y, double* kout,
                                 const FTerms& fx) {
  Ctl* ctl = (Ctl*)(ws + o_ctl);
  const Red rd = red();
  double* res = (double*)(ws + o_res);
  const Csr csr{(const int*)(ws + o_rowptr), (const int*)(ws + o_col)};
  const double* kval = (const double*)(ws + o_kval);
  if (op.format == MPRK_FMT_CSR)
    PLAUNCH(KC_RESIDUAL, (k_residual<1, 1>), dim3(ln_row_red.G), dim3(TPB), 0, stream, ln_row_red, geo, Kc, csr,
                       kval, y, rhs, kout, res, fx, cfg, ctl, rd);
  else if (zm_lz > 0)  // (zm_lz > 0 implies vec == 4)
    PLAUNCH(KC_RESIDUAL, (k_residual_zm<4>), dim3(zl_res.G), dim3(TPB), zmarch_lds(geo, zl_res, 8), stream,
            zl_res, geo, Kc, y, rhs, kout, res, fx, cfg, ctl, rd);
  else if (vec == 4)
    PLAUNCH(KC_RESIDUAL, (k_residual<4, 0>), dim3(ln_vec_red.G), dim3(TPB), 0, stream, ln_vec_red, geo, Kc, csr,
                       kval, y, rhs, kout, res, fx, cfg, ctl, rd);
  else
    PLAUNCH(KC_RESIDUAL, (k_residual<1, 0>), dim3(ln_vec_red.G), dim3(TPB), 0, stream, ln_vec_red, geo, Kc, csr,
                       kval, y, rhs, kout, res, fx, cfg, ctl, rd);
  HIPCHK(hipGetLastError());
  return MPRK_OK;
}

// One implicit stage: FP64 residual -> LP Krylov solve -> FP64 update, repeated until the
// device marks the stage finished.  With a valid history of this stage, each predicted pass
// enqueues its Krylov iterations (last count + margin) and its promotion without waiting: an
// inner solve cut short only leaves a larger FP64 residual for the next pass.  The host waits
// for the device only where the history says the stage may already be finished.  The one-solve
// mode has no later pass to absorb a solve cut short, so there the predicted count is only the
// first chunk: the host keeps enqueuing chunks until the device reports the solve finished.
int mprk_handle::run_solve(int si, int slot, const double* rhs, double* y, double* kout,
                           const FTerms& fx) {
  if (capturing) return run_solve_graph(si, slot, rhs, y, kout, fx);
  int rc = update_hist(slot);
  if (rc) return rc;
  const StageHist H = hist[slot];
  const SolveCfg& cfg = cfgs[si];
  EngineCtx c = ctx();
  c.y = y;
  c.fdm_sigma = cfg.sigma;
  const BJDesc dinv = bj_desc(si);
  const Coef<double> Mc = stage_coef(Kc, cfg.sigma);
  const bool cg = prec.krylov == MPRK_CG;
  const int P = cfg.paper_mode ? 1 : cfg.max_passes;
  const int maxp = cfg.maxit;
  const int chunk = cg ? cg_chunk : gm_chunk;
  for (int pass = 0; pass <= P; ++pass) {
    rc = launch_residual(cfg, rhs, y, kout, fx);
    if (rc) return rc;
    if (pass == P) break;
    const bool predicted = H.valid && pass < H.passes;
    const bool certain = predicted && !cfg.paper_mode;
    int slot_id = 0;
    // (the one-solve mode's only pass always runs: its residual sets no decision before it)
    if (!certain && !(cfg.paper_mode && pass == 0)) {
      rc = poll_enqueue(&slot_id);
      if (rc) return rc;
      CtlHead hd;
      rc = poll_wait(slot_id, &hd);
      if (rc) return rc;
      if (hd.outer_done) break;
    }
    if (cg) HIPCHK(eng->cg_begin(c, cfg, dinv));
    else HIPCHK(eng->gm_begin(c, cfg, dinv));
    int enq = 0;  // Krylov iterations enqueued in this pass
    if (certain) {
      const int n = std::min(maxp, H.iters[pass] + predict_margin);
      enq = n;
      for (int k = 0; k < n; ++k) {
        if (cg) HIPCHK(eng->cg_iter(c, cfg, Mc, dinv, k));
        else HIPCHK(eng->gm_iter(c, cfg, Mc, dinv, k));
      }
    } else {
      std::deque<int> pend;
      int its = 0;
      bool inner = false, outer = false;
      while (its < maxp && !inner && !outer) {
        const int want = (predicted && its == 0) ? H.iters[pass] + predict_margin : chunk;
        const int cnt = std::min(std::max(want, 1), maxp - its);
        for (int k = 0; k < cnt; ++k) {
          if (cg) HIPCHK(eng->cg_iter(c, cfg, Mc, dinv, its + k));
          else HIPCHK(eng->gm_iter(c, cfg, Mc, dinv, its + k));
        }
        its += cnt;
        enq = its;
        rc = poll_enqueue(&slot_id);
        if (rc) return rc;
        pend.push_back(slot_id);
        while ((int)pend.size() > lookahead) {
          const int sl = pend.front();
          pend.pop_front();
          CtlHead hd;
          rc = poll_wait(sl, &hd);
          if (rc) return rc;
          if (hd.outer_done) outer = true;
          if (hd.inner_done) inner = true;
          if (inner || outer) break;
        }
      }
      if (outer) break;
    }
    if (cg) HIPCHK(eng->cg_finish(c));
    else HIPCHK(eng->gm_finish(c, cfg, dinv, enq));
  }
  return stage_record(slot);
}

// The stage inside a step graph: the passes and Krylov iterations of the stage's last steered
// solve (each pass its recorded count plus the usual margin) and one spare pass, all enqueued
// without a host wait.  The pass limit is what was enqueued, and a stage that misses its
// tolerance within it holds its step and halts the call's remaining replays (the strict device
// rule), so that the host can finish the call on the steered path with the same results.
int mprk_handle::run_solve_graph(int si, int slot, const double* rhs, double* y, double* kout,
                                 const FTerms& fx) {
  const StageHist& H = hist[slot];
  SolveCfg cfg = cfgs[si];
  const int P = std::min(cfg.max_passes, H.passes + 1);
  cfg.max_passes = P;
  cfg.strict = 1;
  EngineCtx c = ctx();
  c.y = y;
  c.fdm_sigma = cfg.sigma;
  const BJDesc dinv = bj_desc(si);
  const Coef<double> Mc = stage_coef(Kc, cfg.sigma);
  const bool cg = prec.krylov == MPRK_CG;
  int most = 1;
  for (int p = 0; p < H.passes; ++p) most = std::max(most, H.iters[p]);
  for (int pass = 0; pass <= P; ++pass) {
    int rc = launch_residual(cfg, rhs, y, kout, fx);
    if (rc) return rc;
    if (pass == P) break;
    if (cg) HIPCHK(eng->cg_begin(c, cfg, dinv));
    else HIPCHK(eng->gm_begin(c, cfg, dinv));
    const int n = std::min(cfg.maxit, (pass < H.passes ? H.iters[pass] : most) + predict_margin);
    for (int k = 0; k < n; ++k) {
      if (cg) HIPCHK(eng->cg_iter(c, cfg, Mc, dinv, k));
      else HIPCHK(eng->gm_iter(c, cfg, Mc, dinv, k));
    }
    if (cg) HIPCHK(eng->cg_finish(c));
    else HIPCHK(eng->gm_finish(c, cfg, dinv, n));
  }
  hipLaunchKernelGGL(k_stage_snapshot, dim3(1), dim3(64), 0, stream, (Ctl*)(ws + o_ctl), slot);
  HIPCHK(hipGetLastError());
  return MPRK_OK;
}

int mprk_handle::enqueue_step(bool first_of_call) {
  Ctl* ctl = (Ctl*)(ws + o_ctl);
  double* rhs = (double*)(ws + o_rhs);
  double* y = (double*)(ws + o_y);
  auto kvec = [&](int j) { return (double*)(ws + o_k + (size_t)j * N * 8); };
  auto evec = [&](int j) { return (double*)(ws + o_keps + (size_t)j * N * 8); };
  const int s = nstages;
  // f(u), the slope at the step's start, for the start values (an explicit first stage
  // computes it as k_0)
  double* f0 = (double*)(ws + o_scr);
  const bool have_f0 = start_eval && implicit_[0];
  if (have_f0) {
    int rc = launch_apply64(u, f0, 0.0, 0, fterms());
    if (rc) return rc;
  }
  auto stage_c = [&](int r) {  // c_r = sum_j a_rj; the step's start (r = -1) is c = 0
    double c = 0.0;
    for (int j = 0; j <= r; ++j) c += tab.a_hi[r * s + j] + tab.a_lo[r * s + j];
    return c;
  };
  for (int i = 0; i < s; ++i) {
    CombArgs a{};
    a.nv = 0;
    for (int j = 0; j < i; ++j) {
      const double ah = tab.a_hi[i * s + j], al = tab.a_lo[i * s + j];
      if (!implicit_[j]) {  // f^eps = f for an explicit stage
        if (ah + al != 0.0) {
          a.v[a.nv] = kvec(j);
          a.c[a.nv++] = dt * (ah + al);
        }
        continue;
      }
      if (ah != 0.0) {
        a.v[a.nv] = kvec(j);
        a.c[a.nv++] = dt * ah;
      }
      if (al != 0.0) {
        a.v[a.nv] = evec(j);
        a.c[a.nv++] = dt * al;
      }
    }
    const double sg = implicit_[i] ? cfgs[sig_idx[i]].sigma : 0.0;  // (no shift when explicit)
    if (start_slope && implicit_[i] && i > 0) {  // start value rhs + sigma k_{i-1}
      a.pv = kvec(i - 1);
      a.pc = sg;
      // linear in c through k_{i-1} and k_{i-2} (f(u) at c = 0 before the first stage)
      const int j2 = i - 2;
      if (start_extrap && (j2 >= 0 || have_f0)) {
        const double d1 = stage_c(i) - stage_c(i - 1), d0 = stage_c(i - 1) - stage_c(j2);
        if (std::fabs(d0) > 1e-12) {
          const double th = d1 / d0;
          a.pc = sg * (1.0 + th);
          a.pv2 = j2 >= 0 ? kvec(j2) : f0;
          a.pc2 = -sg * th;
        }
      }
    } else if (start_first_eval && have_f0 && i == 0) {  // rhs + sigma f(u)
      a.pv = f0;
      a.pc = sg;
    }
    const int reset = i > 0 ? RESET_STAGE
                            : RESET_STAGE | RESET_STEP | (first_of_call ? RESET_CALL : 0);
    if (vec == 4)
      PLAUNCH(KC_STAGE_RHS, (k_stage_rhs<4>), dim3(ln_vec.G), dim3(TPB), 0, stream, ln_vec, u, a, rhs, y, ctl, reset);
    else
      PLAUNCH(KC_STAGE_RHS, (k_stage_rhs<1>), dim3(ln_vec.G), dim3(TPB), 0, stream, ln_vec, u, a, rhs, y, ctl, reset);
    HIPCHK(hipGetLastError());
    if (!implicit_[i]) {
      int rc = launch_apply64(y, kvec(i), 0.0, 0, fterms());
      if (rc) return rc;
      continue;
    }
    int rc = run_solve(sig_idx[i], i, rhs, y, kvec(i), fterms());
    if (rc) return rc;
    if (need_keps) {
      const double inv = 1.0 / cfgs[sig_idx[i]].sigma;
      if (vec == 4)
        PLAUNCH(KC_KEPS, (k_keps<4>), dim3(ln_vec.G), dim3(TPB), 0, stream, ln_vec, y, rhs, inv, evec(i));
      else
        PLAUNCH(KC_KEPS, (k_keps<1>), dim3(ln_vec.G), dim3(TPB), 0, stream, ln_vec, y, rhs, inv, evec(i));
      HIPCHK(hipGetLastError());
    }
  }
  CombArgs a{};
  a.nv = 0;
  for (int i = 0; i < s; ++i)
    if (tab.b[i] != 0.0) {
      a.v[a.nv] = kvec(i);
      a.c[a.nv++] = dt * tab.b[i];
    }
  if (vec == 4)
    PLAUNCH(KC_COMBINE, (k_combine<4>), dim3(ln_vec.G), dim3(TPB), 0, stream, ln_vec, u, a, ctl);
  else
    PLAUNCH(KC_COMBINE, (k_combine<1>), dim3(ln_vec.G), dim3(TPB), 0, stream, ln_vec, u, a, ctl);
  HIPCHK(hipGetLastError());
  return MPRK_OK;
}

int mprk_handle::launch_apply64(const double* x, double* y, double sigma, int mode,
                                const FTerms& fx) {
  const Csr csr{(const int*)(ws + o_rowptr), (const int*)(ws + o_col)};
  const double* kval = (const double*)(ws + o_kval);
  if (op.format == MPRK_FMT_CSR)
    PLAUNCH(KC_APPLY64, (k_apply64<1, 1>), dim3(ln_row.G), dim3(TPB), 0, stream, ln_row, geo, Kc, csr, kval,
                       x, y, sigma, mode, fx);
  else if (vec == 4)
    PLAUNCH(KC_APPLY64, (k_apply64<4, 0>), dim3(ln_vec.G), dim3(TPB), 0, stream, ln_vec, geo, Kc, csr, kval,
                       x, y, sigma, mode, fx);
  else
    PLAUNCH(KC_APPLY64, (k_apply64<1, 0>), dim3(ln_vec.G), dim3(TPB), 0, stream, ln_vec, geo, Kc, csr, kval,
                       x, y, sigma, mode, fx);
  HIPCHK(hipGetLastError());
  return MPRK_OK;
}

void mprk_handle::fill_stats(mprk_stats* st) {
  std::memset(st, 0, sizeof(*st));
  const CtlHead* hd = (const CtlHead*)slots;
  st->stages = nstages;
  for (int i = 0; i < nstages && hd; ++i) {
    if (!implicit_[i]) {
      st->converged[i] = 1;
      continue;
    }
    const CtlHead& r = hd[NSLOT + i];
    st->iters[i] = r.total_iters;
    st->passes[i] = r.passes;
    st->resid[i] = r.outer_rel;
    st->converged[i] = r.converged && !r.nonfinite;
  }
  st->steps = step_count;
  st->t = t_now;
  st->total_iters = life_iters;
  st->total_passes = life_passes;
  st->nonfinite = last_nonfinite;
  st->missed = last_missed;
  st->graph_steps = graph_steps_last;
}

void mprk_handle::set_gm_form(int f, int lz) {
  if (f < 0 || f > 2 || !(gform_ok & (1 << f))) f = 0;  // (a cached choice of another problem)
  gform = f;
  if (f > 0) zl_lp = make_zlaunch(geo, vec_lp, lz);
}

extern "C" int32_t mprk_launch_info_get(const mprk_handle* h, mprk_launch_info* out) {
  if (!h || !out) return set_error(MPRK_EINVAL, "NULL argument");
  out->nit_vec = h->ln_vec.nit;
  out->nit_row = h->ln_row.nit;
  out->nit_vec_red = h->ln_vec_red.nit;
  out->nit_row_red = h->ln_row_red.nit;
  out->nit_lp = h->ln_lp.nit;
  out->nit_lp_red = h->ln_lp_red.nit;
  out->residual_planes = h->zm_lz;
  out->gm_form = h->prec.krylov == MPRK_GMRES ? h->gform + 1 : 0;
  out->stage_start = h->start_mode;
  out->gm_planes = h->prec.krylov == MPRK_GMRES && h->gform > 0 ? h->zl_lp.LZ : 0;
  for (int t = 0; t < 4; ++t) out->bj_chunks[t] = 0;
  for (const auto& B : h->bjsets)
    for (int t : B.tag) out->bj_chunks[t] += 1;
  return MPRK_OK;
}

void mprk_handle::set_residual_tiles(int lz) {
  zm_lz = lz;
  if (lz > 0) zl_res = make_zlaunch(geo, vec, lz);
}

// ------------------------------------------------------------------------------------------
// step graph
// ------------------------------------------------------------------------------------------

// Replays need every implicit stage's solve history (from steered steps) and the outer loop.
bool mprk_handle::graph_ready() const {
  if (!graph_on || prof_on) return false;
  for (int i = 0; i < nstages; ++i) {
    if (!implicit_[i]) continue;
    if (cfgs[sig_idx[i]].paper_mode || !hist[i].valid) return false;
  }
  return true;
}

void mprk_handle::graph_drop() {
  if (gexec) (void)hipGraphExecDestroy(gexec);
  gexec = nullptr;
  gexec_epoch = 0;
}

// Captures one step on the library's own stream (the caller's may be the legacy default stream,
// which cannot be captured) and instantiates it.  Nothing runs during the capture.
int mprk_handle::graph_capture() {
  graph_drop();
  if (!cap_stream) HIPCHK(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
  for (int i = 0; i < nstages; ++i) ghist[i] = hist[i];
  hipStream_t user = stream;
  stream = cap_stream;
  capturing = true;
  const hipError_t eb = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
  int rc = eb == hipSuccess ? enqueue_step(false) : MPRK_OK;
  hipGraph_t g = nullptr;
  const hipError_t ee = eb == hipSuccess ? hipStreamEndCapture(cap_stream, &g) : hipSuccess;
  capturing = false;
  stream = user;
  if (eb != hipSuccess)
    return set_error(MPRK_EDEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(eb));
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (ee != hipSuccess || !g)
    return set_error(MPRK_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
  const hipError_t ei = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    gexec = nullptr;
    return set_error(MPRK_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  }
  gexec_epoch = graph_epoch;
  return MPRK_OK;
}

// Runs up to nsteps steps from the graph; *done = steps completed (combined).  The graph is
// captured again when anything it depends on changed or when a steered solve needed more passes
// or iterations than the capture enqueues.  A stage that missed inside the graph held its step:
// *done < nsteps, and the caller continues on the steered path from there.
int mprk_handle::graph_steps(int nsteps, int* done) {
  *done = 0;
  for (int i = 0; i < nstages; ++i)
    if (implicit_[i]) {
      int rc = update_hist(i);
      if (rc) return rc;
    }
  if (!graph_ready()) return MPRK_OK;
  bool same = gexec && gexec_epoch == graph_epoch;
  for (int i = 0; i < nstages && same; ++i) {
    if (!implicit_[i]) continue;
    if (hist[i].passes > ghist[i].passes) same = false;
    for (int p = 0; p < hist[i].passes && same; ++p)
      if (hist[i].iters[p] > ghist[i].iters[p]) same = false;
  }
  if (!same) {
    int rc = graph_capture();
    if (rc) return rc;
  }
  Ctl* ctl = (Ctl*)(ws + o_ctl);
  hipLaunchKernelGGL(k_release_halt, dim3(1), dim3(64), 0, stream, ctl);
  HIPCHK(hipGetLastError());
  for (int n = 0; n < nsteps; ++n) HIPCHK(hipGraphLaunch(gexec, stream));
  // the stage records of the last replayed step, for the statistics
  HIPCHK(hipMemcpyAsync((void*)&slots[NSLOT], ctl->srec, sizeof(CtlHead) * nstages,
                        hipMemcpyDeviceToHost, stream));
  // counters: completed steps; a miss inside the graph is not reported (its steps are re-run)
  int rc = sync_counters();
  *done = last_good;
  graph_steps_last = last_good;
  return rc;
}

int mprk_handle::rebase_missed() {
  Ctl* ctl = (Ctl*)(ws + o_ctl);
  long long m = 0;
  HIPCHK(hipMemcpyAsync(&m, &ctl->missed, sizeof(m), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  missed_base = m;
  return MPRK_OK;
}

int mprk_handle::sync_counters() {
  Ctl* ctl = (Ctl*)(ws + o_ctl);
  long long lf[4];  // life_iters, life_passes, missed, held_steps (adjacent in Ctl)
  static_assert(offsetof(Ctl, held_steps) == offsetof(Ctl, life_iters) + 3 * sizeof(long long),
                "counters read together");
  CtlHead hd;
  HIPCHK(hipMemcpyAsync(&hd, ctl, sizeof(CtlHead), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(lf, &ctl->life_iters, sizeof(lf), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  const long long good = hd.good_steps - good_base;
  const int bad = hd.bad_steps - bad_base;
  last_good = (int)good;
  good_base = hd.good_steps;
  bad_base = hd.bad_steps;
  step_count += good;
  t_now += dt * (double)good;
  life_iters = lf[0];
  life_passes = lf[1];
  last_missed = (int)(lf[2] - missed_base);
  missed_base = lf[2];
  last_held = (int)(lf[3] - held_base);
  held_base = lf[3];
  last_nonfinite = bad > 0;
  return bad > 0 ? MPRK_ENONFINITE : MPRK_OK;
}

extern "C" int32_t mprk_step(mprk_handle* h, int32_t nsteps, mprk_stats* stats) {
  if (!h) return set_error(MPRK_EINVAL, "NULL handle");
  if (!h->bound) return set_error(MPRK_ESTATE, "mprk_step before mprk_bind");
  if (int rcw = h->check_ws()) return rcw;
  if (nsteps < 0) return set_error(MPRK_EINVAL, "nsteps must be >= 0");
  int done = 0;
  h->graph_steps_last = 0;
  if (h->graph_on && nsteps > 0) {
    int rc = h->graph_steps(nsteps, &done);
    if (rc == MPRK_ENONFINITE) {
      if (stats) h->fill_stats(stats);
      return set_error(rc, "non-finite residual: u left at the last completed step");
    }
    if (rc) return rc;
  }
  // steered steps (all of them, or those after a step the graph held); the first releases the
  // halt of an earlier call or of the replays
  for (int n = done; n < nsteps; ++n) {
    int rc = h->enqueue_step(n == done);
    if (rc) return rc;
  }
  int rc = h->sync_counters();
  if (stats) h->fill_stats(stats);
  if (rc == MPRK_ENONFINITE) return set_error(rc, "non-finite residual: u left at the last completed step");
  // every stage of every step of this call counts, not only the last step's record; the
  // device stopped combining at the first step with a missed stage
  if (h->prec.strict && (h->last_missed > 0 || h->last_held > 0))
    return set_error(MPRK_ENOTCONV, "a stage missed its tolerance: u left at the last step whose "
                                    "stages all met it");
  return MPRK_OK;
}

extern "C" int32_t mprk_solve(mprk_handle* h, int32_t stage, const double* rhs_dev, double* x_dev,
                              mprk_solve_info* info) {
  if (!h || !rhs_dev || !x_dev) return set_error(MPRK_EINVAL, "NULL argument");
  if (!h->bound) return set_error(MPRK_ESTATE, "mprk_solve before mprk_bind");
  if (int rcw = h->check_ws()) return rcw;
  if (stage < 0 || stage >= h->nstages || !h->implicit_[stage])
    return set_error(MPRK_EINVAL, "stage must be an implicit stage of the tableau");
  Ctl* ctl = (Ctl*)(h->ws + h->o_ctl);
  CombArgs a{};
  a.nv = 0;
  // x = rhs (initial guess), rhs copy into the workspace; resets the stage record
  double* rhs = (double*)(h->ws + h->o_rhs);
  if (h->vec == 4)
    hipLaunchKernelGGL((k_stage_rhs<4>), dim3(h->ln_vec.G), dim3(TPB), 0, h->stream, h->ln_vec, rhs_dev, a, rhs,
                       x_dev, ctl, RESET_STAGE | RESET_CALL);
  else
    hipLaunchKernelGGL((k_stage_rhs<1>), dim3(h->ln_vec.G), dim3(TPB), 0, h->stream, h->ln_vec, rhs_dev, a, rhs,
                       x_dev, ctl, RESET_STAGE | RESET_CALL);
  HIPCHK(hipGetLastError());
  int rc = h->run_solve(h->sig_idx[stage], MPRK_MAX_STAGES, rhs, x_dev, (double*)(h->ws + h->o_scr),
                        FTerms{});
  if (rc) return rc;
  CtlHead hd;
  HIPCHK(hipMemcpyAsync(&hd, ctl, sizeof(CtlHead), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  // a missed solve here is reported in info, not by the next mprk_step
  rc = h->rebase_missed();
  if (rc) return rc;
  if (info) {
    info->iters = hd.total_iters;
    info->passes = hd.passes;
    info->converged = hd.converged && !hd.nonfinite;
    info->resid = hd.outer_rel;
  }
  if (hd.nonfinite) return set_error(MPRK_ENONFINITE, "non-finite residual in mprk_solve");
  return MPRK_OK;
}

extern "C" int32_t mprk_set_forcing(mprk_handle* h, const double* g_dev) {
  if (!h) return set_error(MPRK_EINVAL, "handle is NULL");
  h->force = g_dev;
  h->graph_epoch += 1;
  return MPRK_OK;
}

// The stage systems become y - sigma (K y + g + R(y)) = rhs: the FP64 residual and the explicit
// evaluations take R, the LP systems keep I - sigma K, so the outer defect-correction loop is a
// simplified Newton iteration whose Jacobian is the linear part.  The one-solve mode has no
// such loop and is refused.
extern "C" int32_t mprk_set_reaction(mprk_handle* h, double r1, double r2, double r3) {
  if (!h) return set_error(MPRK_EINVAL, "handle is NULL");
  if (!std::isfinite(r1) || !std::isfinite(r2) || !std::isfinite(r3))
    return set_error(MPRK_EINVAL, "reaction coefficients must be finite");
  const bool on = r1 != 0.0 || r2 != 0.0 || r3 != 0.0;
  if (on && h->prec.refine_max == 0)
    return set_error(MPRK_EUNSUPPORTED,
                     "a reaction needs the FP64 outer loop (refine_max > 0): the one-solve mode "
                     "would stop after a single linearised solve");
  h->react[0] = r1;
  h->react[1] = r2;
  h->react[2] = r3;
  h->react_on = on;
  h->graph_epoch += 1;
  return MPRK_OK;
}

extern "C" int32_t mprk_set_step_graph(mprk_handle* h, int32_t enable) {
  if (!h) return set_error(MPRK_EINVAL, "handle is NULL");
  static_assert(MPRK_MAX_STAGES <= MAXSTG, "a replayed step keeps a record per stage");
  h->graph_on = enable != 0;
  if (!h->graph_on) h->graph_drop();
  return MPRK_OK;
}

extern "C" int32_t mprk_apply(mprk_handle* h, int32_t which, int32_t stage, const void* x, void* y) {
  if (!h || !x || !y) return set_error(MPRK_EINVAL, "NULL argument");
  if (!h->bound) return set_error(MPRK_ESTATE, "mprk_apply before mprk_bind");
  if (int rcw = h->check_ws()) return rcw;
  double sigma = 0.0;
  int si = -1;
  if (which != MPRK_APPLY_K64) {
    if (stage < 0 || stage >= h->nstages || !h->implicit_[stage])
      return set_error(MPRK_EINVAL, "stage must be an implicit stage of the tableau");
    si = h->sig_idx[stage];
    sigma = h->sigmas[si];
  }
  EngineCtx c = h->ctx();
  switch (which) {
    case MPRK_APPLY_K64: {
      int rc = h->launch_apply64((const double*)x, (double*)y, 0.0, 0);
      if (rc) return rc;
      break;
    }
    case MPRK_APPLY_M64: {
      int rc = h->launch_apply64((const double*)x, (double*)y, sigma, 1);
      if (rc) return rc;
      break;
    }
    case MPRK_APPLY_M_LP:
      HIPCHK(h->eng->apply_m(c, stage_coef(h->Kc, sigma), sigma, x, y));
      break;
    case MPRK_APPLY_BJ_LP:
      if (!h->bs) return set_error(MPRK_EINVAL, "no block-Jacobi preconditioner configured");
      HIPCHK(h->eng->apply_bj(c, h->bj_desc(si), x, y));
      break;
    case MPRK_APPLY_FDM_LP: {
      if (!h->fdm) return set_error(MPRK_EINVAL, "no fast-diagonalisation preconditioner configured");
      // the contraction kernels skip once a solve is finished: clear the flags first
      Ctl* ctl = (Ctl*)(h->ws + h->o_ctl);
      const int zero[2] = {0, 0};
      HIPCHK(hipMemcpyAsync(&ctl->outer_done, zero, sizeof(int) * 2, hipMemcpyHostToDevice, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      HIPCHK(h->eng->fdm_apply(c, sigma, x, y));
      break;
    }
    default:
      return set_error(MPRK_EINVAL, "unknown apply op");
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  return MPRK_OK;
}

extern "C" int32_t mprk_get_state(const mprk_handle* h, double* t, int64_t* step) {
  if (!h) return set_error(MPRK_EINVAL, "NULL handle");
  if (h->bound) HIPCHK(hipStreamSynchronize(h->stream));
  if (t) *t = h->t_now;
  if (step) *step = h->step_count;
  return MPRK_OK;
}

extern "C" int32_t mprk_set_state(mprk_handle* h, double t, int64_t step) {
  if (!h) return set_error(MPRK_EINVAL, "NULL handle");
  if (!std::isfinite(t) || step < 0) return set_error(MPRK_EINVAL, "bad state");
  h->t_now = t;
  h->step_count = step;
  return MPRK_OK;
}

extern "C" int32_t mprk_stats_sync(mprk_handle* h, mprk_stats* out) {
  if (!h || !out) return set_error(MPRK_EINVAL, "NULL argument");
  if (h->bound) HIPCHK(hipStreamSynchronize(h->stream));
  h->fill_stats(out);
  return MPRK_OK;
}

static int read_counters(mprk_handle* h, long long* worked, long long* units) {
  Ctl* ctl = (Ctl*)(h->ws + h->o_ctl);
  HIPCHK(hipMemcpyAsync(worked, ctl->worked, sizeof(long long) * KC_COUNT, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(units, ctl->units, sizeof(long long) * KC_COUNT, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return MPRK_OK;
}

extern "C" int32_t mprk_profile(mprk_handle* h, int32_t enable) {
  if (!h) return set_error(MPRK_EINVAL, "NULL handle");
  if (!h->bound) return set_error(MPRK_ESTATE, "mprk_profile before mprk_bind");
  if (enable) {
    int rc = read_counters(h, h->worked0, h->units0);
    if (rc) return rc;
    h->prof.stream = h->stream;
    h->prof.reset();
    h->prof_on = true;
  } else {
    h->prof_on = false;
  }
  return MPRK_OK;
}

extern "C" int32_t mprk_profile_read(mprk_handle* h, int32_t kclass, int64_t* launches,
                                     int64_t* worked, int64_t* units, double* total_ms) {
  if (!h) return set_error(MPRK_EINVAL, "NULL handle");
  if (!h->bound) return set_error(MPRK_ESTATE, "mprk_profile_read before mprk_bind");
  if (kclass < 0 || kclass >= KC_COUNT) return set_error(MPRK_EINVAL, "bad kernel class");
  long long w[KC_COUNT], u[KC_COUNT];
  int rc = read_counters(h, w, u);
  if (rc) return rc;
  if (h->prof.failed) return set_error(MPRK_EDEVICE, "profiling event creation/record failed");
  double ms = 0.0;
  long long n = 0;
  for (const auto& r : h->prof.recs) {
    if (r.kc != kclass) continue;
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, h->prof.pool[r.e0], h->prof.pool[r.e1]));
    ms += t;
    n += r.n;
  }
  if (launches) *launches = n;
  if (worked) *worked = w[kclass] - h->worked0[kclass];
  if (units) *units = u[kclass] - h->units0[kclass];
  if (total_ms) *total_ms = ms;
  return MPRK_OK;
}

// ---- autotuner ----
namespace {
struct TuneKey {
  int nx, ny, nz, bc, kind, fmt, storage, compute;
  bool operator<(const TuneKey& o) const {
    return std::tie(nx, ny, nz, bc, kind, fmt, storage, compute) <
           std::tie(o.nx, o.ny, o.nz, o.bc, o.kind, o.fmt, o.storage, o.compute);
  }
};
struct TuneVal {
  int nv, nr, nvr, nrr;  // groups per thread: streaming vector/row, reducing vector/row
  int nl, nlr;           // LP kernels: streaming / reducing
  int zlz;               // FP64 residual: z-marching planes per tile (0 = gather kernel)
  int gform, glz;        // GMRES step form and its planes per tile (tiled forms)
};
std::map<TuneKey, TuneVal> g_tuned;
std::mutex g_tune_mu;
}  // namespace

extern "C" int32_t mprk_autotune(mprk_handle* h, int32_t* nit_vec, int32_t* nit_row) {
  if (!h) return set_error(MPRK_EINVAL, "NULL handle");
  if (!h->bound) return set_error(MPRK_ESTATE, "mprk_autotune before mprk_bind");
  if (int rcw = h->check_ws()) return rcw;
  h->graph_epoch += 1;  // launch shapes may change
  const bool csr = h->op.format == MPRK_FMT_CSR;
  const long ngv = h->N / h->vec, ngr = h->N, ngl = h->N / h->vec_lp;
  const TuneKey key{h->grid.nx, h->grid.ny, h->grid.nz, h->grid.bc, h->op.kind, h->op.format, h->prec.storage,
                    h->prec.compute};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      const TuneVal& v = it->second;
      h->ln_vec = make_launch_nit(ngv, v.nv);
      h->ln_row = make_launch_nit(ngr, v.nr);
      h->ln_vec_red = make_launch_nit(ngv, v.nvr);
      h->ln_row_red = make_launch_nit(ngr, v.nrr);
      h->ln_lp = make_launch_nit(ngl, v.nl);
      h->ln_lp_red = make_launch_nit(ngl, v.nlr);
      h->set_residual_tiles(v.zlz);
      if (h->prec.krylov == MPRK_GMRES && h->prec.gm_form == MPRK_GMFORM_AUTO) h->set_gm_form(v.gform, v.glz);
      if (nit_vec) *nit_vec = v.nv;
      if (nit_row) *nit_row = v.nr;
      return MPRK_OK;
    }
  }
  // scratch: LP Krylov vectors, the FP64 residual/scratch vectors (no step is in flight)
  const size_t vlp = ((size_t)h->N * h->lp_bytes + 255) & ~(size_t)255;
  void* x_lp = h->ws + (h->prec.krylov == MPRK_CG ? h->o_r : h->o_V);
  void* y_lp = (char*)x_lp + vlp;
  double* x64 = (double*)(h->ws + h->o_y);
  double* y64 = (double*)(h->ws + h->o_scr);
  double* rhs = (double*)(h->ws + h->o_rhs);
  HIPCHK(hipMemsetAsync(x_lp, 0, 2 * vlp, h->stream));
  HIPCHK(hipMemsetAsync(x64, 0, (size_t)h->N * 8, h->stream));
  HIPCHK(hipMemsetAsync(rhs, 0, (size_t)h->N * 8, h->stream));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int si = 0;
  Ctl* ctl = (Ctl*)(h->ws + h->o_ctl);
  const double sigma = h->sigmas.empty() ? 0.0 : h->sigmas[0];
  const Coef<double> Mc = stage_coef(h->Kc, sigma);
  int rc = MPRK_OK;
  auto time_it = [&](auto&& body, float* out) {
    float ms = 0.f;
    for (int rep = 0; rep < 2 && rc == MPRK_OK; ++rep) {  // rep 0 warms up
      if (hipEventRecord(e0, h->stream) != hipSuccess) rc = MPRK_EDEVICE;
      for (int k = 0; k < 4 && rc == MPRK_OK; ++k) rc = body();
      if (rc == MPRK_OK && hipEventRecord(e1, h->stream) != hipSuccess) rc = MPRK_EDEVICE;
      if (rc == MPRK_OK && hipEventSynchronize(e1) != hipSuccess) rc = MPRK_EDEVICE;
      if (rc == MPRK_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = MPRK_EDEVICE;
    }
    *out = ms;
  };
  // streaming kernels: LP SpMV + FP64 operator, groups per thread in {1..16}
  TuneVal best{h->ln_vec.nit, h->ln_row.nit, h->ln_vec_red.nit, h->ln_row_red.nit,
               h->ln_lp.nit, h->ln_lp_red.nit, h->zm_lz, h->gform, h->zl_lp.LZ};
  float bv = 1e30f;
  for (int nit : {1, 2, 4, 8, 16}) {
    const Launch sv = h->ln_vec, sr = h->ln_row, sl = h->ln_lp;
    h->ln_vec = make_launch_nit(ngv, nit);
    h->ln_lp = make_launch_nit(ngl, nit);
    if (csr) h->ln_row = make_launch_nit(ngr, nit);
    EngineCtx c = h->ctx();
    float ms;
    time_it([&]() {
      if (h->eng->apply_m(c, Mc, sigma, x_lp, y_lp) != hipSuccess) return (int)MPRK_EDEVICE;
      return h->launch_apply64(x64, y64, 0.0, 0);
    }, &ms);
    h->ln_vec = sv;
    h->ln_row = sr;
    h->ln_lp = sl;
    if (rc) break;
    if (ms < bv) {
      bv = ms;
      best.nv = nit;
      best.nl = nit;
      if (csr) best.nr = nit;
    }
  }
  // kernels with a grid reduction: time the real Krylov iteration (4 iterations after a
  // residual + begin on a patterned state) for 1, 2, 4 or 8 groups per thread
  float br = 1e30f;
  for (int nit : {1, 2, 4, 8}) {
    if (rc || h->cfgs.empty()) break;
    const Launch sv = h->ln_vec_red, sr = h->ln_row_red, sl = h->ln_lp_red;
    h->ln_vec_red = make_launch_nit(ngv, nit);
    h->ln_row_red = make_launch_nit(ngr, nit);
    h->ln_lp_red = make_launch_nit(ngl, nit);
    if (h->ln_vec_red.G > h->pstride || h->ln_row_red.G > h->pstride || h->ln_lp_red.G > h->pstride) {
      h->ln_vec_red = sv;
      h->ln_row_red = sr;
      h->ln_lp_red = sl;
      continue;
    }
    const SolveCfg& cfg = h->cfgs[si];
    EngineCtx c = h->ctx();
    c.y = x64;
    const BJDesc dinv = h->bj_desc(si);
    const bool cg = h->prec.krylov == MPRK_CG;
    float ms = 0.f;
    for (int rep = 0; rep < 2 && rc == MPRK_OK; ++rep) {
      // state: rhs = pattern A (via the stage-rhs kernel, which also reopens the stage record),
      // y = pattern B, so the first residual is non-zero
      CombArgs ca{};
      ca.nv = 0;
      const unsigned nb = (unsigned)((h->N + 255) / 256);
      hipLaunchKernelGGL(k_fill_pattern, dim3(nb), dim3(256), 0, h->stream, (long)h->N, 0.37, 0.011, y64);
      if (h->vec == 4)
        hipLaunchKernelGGL((k_stage_rhs<4>), dim3(h->ln_vec.G), dim3(TPB), 0, h->stream, h->ln_vec, y64, ca, rhs, x64, ctl,
                           RESET_STAGE | RESET_CALL);
      else
        hipLaunchKernelGGL((k_stage_rhs<1>), dim3(h->ln_vec.G), dim3(TPB), 0, h->stream, h->ln_vec, y64, ca, rhs, x64, ctl,
                           RESET_STAGE | RESET_CALL);
      hipLaunchKernelGGL(k_fill_pattern, dim3(nb), dim3(256), 0, h->stream, (long)h->N, 0.23, 0.017, x64);
      if (hipGetLastError() != hipSuccess) { rc = MPRK_EDEVICE; break; }
      rc = h->launch_residual(h->cfgs[si], rhs, x64, y64, FTerms{});
      if (rc) break;
      if ((cg ? h->eng->cg_begin(c, cfg, dinv) : h->eng->gm_begin(c, cfg, dinv)) != hipSuccess) { rc = MPRK_EDEVICE; break; }
      if (hipEventRecord(e0, h->stream) != hipSuccess) { rc = MPRK_EDEVICE; break; }
      for (int k = 0; k < 4 && rc == MPRK_OK; ++k)
        if ((cg ? h->eng->cg_iter(c, cfg, Mc, dinv, k) : h->eng->gm_iter(c, cfg, Mc, dinv, k)) != hipSuccess) rc = MPRK_EDEVICE;
      if (rc == MPRK_OK && hipEventRecord(e1, h->stream) != hipSuccess) rc = MPRK_EDEVICE;
      if (rc == MPRK_OK && hipEventSynchronize(e1) != hipSuccess) rc = MPRK_EDEVICE;
      if (rc == MPRK_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = MPRK_EDEVICE;
    }
    const int nvr = h->ln_vec_red.nit, nrr = h->ln_row_red.nit, nlr = h->ln_lp_red.nit;
    h->ln_vec_red = sv;
    h->ln_row_red = sr;
    h->ln_lp_red = sl;
    if (rc) break;
    if (ms < br) {
      br = ms;
      best.nvr = nvr;
      best.nrr = nrr;
      best.nlr = nlr;
    }
  }
  // FP64 residual: gather kernel (at the chosen groups per thread) or z-marching tiles of
  // 2 .. 32 planes, each timed over four launches on a patterned state
  if (rc == MPRK_OK && h->op.format == MPRK_FMT_STENCIL && zmarch_fits(h->geo, h->vec) &&
      !h->cfgs.empty()) {
    const Launch sv = h->ln_vec_red;
    h->ln_vec_red = make_launch_nit(ngv, best.nvr);
    const int keep = h->zm_lz;
    float bz = 1e30f;
    for (int lz : {0, 2, 4, 8, 16, 32}) {
      if (lz > 0 && make_zlaunch(h->geo, h->vec, lz).G > h->pstride) continue;
      h->set_residual_tiles(lz);
      CombArgs ca{};
      ca.nv = 0;
      const unsigned nb = (unsigned)((h->N + 255) / 256);
      hipLaunchKernelGGL(k_fill_pattern, dim3(nb), dim3(256), 0, h->stream, (long)h->N, 0.37, 0.011, y64);
      hipLaunchKernelGGL((k_stage_rhs<4>), dim3(h->ln_vec.G), dim3(TPB), 0, h->stream, h->ln_vec, y64, ca, rhs,
                         x64, ctl, RESET_STAGE | RESET_CALL);
      hipLaunchKernelGGL(k_fill_pattern, dim3(nb), dim3(256), 0, h->stream, (long)h->N, 0.23, 0.017, x64);
      if (hipGetLastError() != hipSuccess) { rc = MPRK_EDEVICE; break; }
      float ms;
      time_it([&]() { return h->launch_residual(h->cfgs[si], rhs, x64, y64, FTerms{}); }, &ms);
      if (rc) break;
      if (ms < bz) {
        bz = ms;
        best.zlz = lz;
      }
    }
    h->ln_vec_red = sv;
    h->set_residual_tiles(rc ? keep : best.zlz);
  }
  // GMRES step form: the gather kernels, or the product on z-marching tiles (+ update kernel),
  // or the folded step, at 2 .. 16 planes per tile; each timed over a cycle's begin, ten
  // Arnoldi steps (or the cycle length) and the cycle's end on a patterned state, with a
  // stopping rule that cannot end the cycle early (the step's cost grows with the basis)
  if (rc == MPRK_OK && h->prec.krylov == MPRK_GMRES && h->prec.gm_form == MPRK_GMFORM_AUTO &&
      (h->gform_ok & 6) && !h->cfgs.empty()) {
    const int keep_f = h->gform, keep_lz = h->zl_lp.LZ;
    const Launch sv = h->ln_vec_red, sl = h->ln_lp_red;
    h->ln_vec_red = make_launch_nit(ngv, best.nvr);
    h->ln_lp_red = make_launch_nit(ngl, best.nlr);
    SolveCfg cfg = h->cfgs[si];
    cfg.rtol = 0.0;
    cfg.atol = 0.0;
    cfg.maxit = cfg.m;
    const int ksteps = std::min(cfg.m, 10);
    const BJDesc dinv = h->bj_desc(si);
    float bg = 1e30f;
    for (int f = 0; f < 3 && rc == MPRK_OK; ++f) {
      if (!(h->gform_ok & (1 << f))) continue;
      for (int lz : {2, 4, 8, 16}) {
        if (f == 0 && lz != 2) continue;  // (the gather form has no tiles)
        if (f > 0 && make_zlaunch(h->geo, h->vec_lp, lz).G > h->pstride) continue;
        h->set_gm_form(f, lz);
        EngineCtx c = h->ctx();
        c.y = x64;
        float ms = 0.f;
        for (int rep = 0; rep < 2 && rc == MPRK_OK; ++rep) {
          CombArgs ca{};
          ca.nv = 0;
          const unsigned nb = (unsigned)((h->N + 255) / 256);
          hipLaunchKernelGGL(k_fill_pattern, dim3(nb), dim3(256), 0, h->stream, (long)h->N, 0.37, 0.011, y64);
          if (h->vec == 4)
            hipLaunchKernelGGL((k_stage_rhs<4>), dim3(h->ln_vec.G), dim3(TPB), 0, h->stream, h->ln_vec, y64, ca,
                               rhs, x64, ctl, RESET_STAGE | RESET_CALL);
          else
            hipLaunchKernelGGL((k_stage_rhs<1>), dim3(h->ln_vec.G), dim3(TPB), 0, h->stream, h->ln_vec, y64, ca,
                               rhs, x64, ctl, RESET_STAGE | RESET_CALL);
          hipLaunchKernelGGL(k_fill_pattern, dim3(nb), dim3(256), 0, h->stream, (long)h->N, 0.23, 0.017, x64);
          if (hipGetLastError() != hipSuccess) { rc = MPRK_EDEVICE; break; }
          rc = h->launch_residual(h->cfgs[si], rhs, x64, y64, FTerms{});
          if (rc) break;
          if (hipEventRecord(e0, h->stream) != hipSuccess) { rc = MPRK_EDEVICE; break; }
          if (h->eng->gm_begin(c, cfg, dinv) != hipSuccess) { rc = MPRK_EDEVICE; break; }
          for (int k = 0; k < ksteps && rc == MPRK_OK; ++k)
            if (h->eng->gm_iter(c, cfg, Mc, dinv, k) != hipSuccess) rc = MPRK_EDEVICE;
          if (rc == MPRK_OK && h->eng->gm_finish(c, cfg, dinv, ksteps) != hipSuccess) rc = MPRK_EDEVICE;
          if (rc == MPRK_OK && hipEventRecord(e1, h->stream) != hipSuccess) rc = MPRK_EDEVICE;
          if (rc == MPRK_OK && hipEventSynchronize(e1) != hipSuccess) rc = MPRK_EDEVICE;
          if (rc == MPRK_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = MPRK_EDEVICE;
        }
        if (rc) break;
        if (ms < bg) {
          bg = ms;
          best.gform = f;
          best.glz = lz;
        }
      }
    }
    h->ln_vec_red = sv;
    h->ln_lp_red = sl;
    if (rc) h->set_gm_form(keep_f, keep_lz);
    else h->set_gm_form(best.gform, best.glz);
  }
  // leave no open stage behind: the next step's first kernel resets the record anyway
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return set_error(MPRK_EDEVICE, "autotune launch failed");
  h->ln_vec = make_launch_nit(ngv, best.nv);
  h->ln_row = make_launch_nit(ngr, best.nr);
  h->ln_vec_red = make_launch_nit(ngv, best.nvr);
  h->ln_row_red = make_launch_nit(ngr, best.nrr);
  h->ln_lp = make_launch_nit(ngl, best.nl);
  h->ln_lp_red = make_launch_nit(ngl, best.nlr);
  // the timing residuals may have counted stages as missed; they are no step's stages
  if (h->rebase_missed()) return set_error(MPRK_EDEVICE, "autotune: counter read failed");
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[key] = best;
  }
  if (nit_vec) *nit_vec = best.nv;
  if (nit_row) *nit_row = best.nr;
  return MPRK_OK;
}

extern "C" const char* mprk_last_error(void) { return g_err.c_str(); }

extern "C" void mprk_destroy(mprk_handle* h) { delete h; }

// runtime_internal.hpp -- host-side handle of one problem (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/mprk.h"
#include "engine.hpp"

namespace mprk {

int set_error(int code, const std::string& msg);
Launch make_launch(long ng);
Launch make_launch_nit(long ng, int nit);
Coef<double> operator_coef(const mprk_grid& g, const mprk_operator& op);
Coef<double> stage_coef(const Coef<double>& K, double sigma);
long csr_count(const Geo& geo, const Coef<double>& K, double* maxabs);
void assemble_csr(const Geo& geo, const Coef<double>& K, std::vector<int>& rowptr,
                  std::vector<int>& col, std::vector<double>& val);

constexpr int NSLOT = 64;  // pinned poll slots

}  // namespace mprk

struct mprk_handle {
  // problem
  mprk_grid grid{};
  mprk_operator op{};
  mprk_tableau tab{};
  mprk_precisions prec{};
  double dt = 0.0;
  hipStream_t stream = nullptr;
  mprk::Geo geo{};
  int N = 0;
  int vec = 1;      // values per group of the FP64 kernels (4 when nx % 4 == 0)
  int vec_lp = 1;   // values per group of the LP kernels (8 for FP16 storage when nx % 8 == 0)
  mprk::Coef<double> Kc{};
  std::unique_ptr<mprk::Engine> eng;
  int lp_bytes = 8;
  int nstages = 0;
  bool implicit_[MPRK_MAX_STAGES] = {};
  int sig_idx[MPRK_MAX_STAGES] = {};
  std::vector<double> sigmas;
  std::vector<mprk::SolveCfg> cfgs;
  bool need_keps = false;
  // launch shapes
  mprk::Launch ln_vec{}, ln_row{};          // streaming kernels
  mprk::Launch ln_vec_red{}, ln_row_red{};  // kernels with a grid reduction
  // z-marching tiles of the FP64 residual (stencil format, whole groups per row): planes per
  // tile, 0 = the gather kernel
  int zm_lz = 0;
  mprk::ZLaunch zl_res{};
  // GMRES Arnoldi step form (0 gather, 1 z-marching product + update, 2 folded on z-marching
  // tiles), the forms this problem allows (bit f), the tiles of the LP kernels and the product
  // buffers of the folded form
  int gform = 0;
  int gform_ok = 1;
  mprk::ZLaunch zl_lp{};
  size_t o_w0 = 0, o_w1 = 0;
  mprk::Launch ln_lp{}, ln_lp_red{};        // LP kernels (groups of vec_lp)
  int pstride = 8;   // level-1 partials per reduced value (max blocks of a reducing launch)
  int pstride2 = 1;  // level-2 partials per reduced value
  int bs = 0;
  int nblk = 0;
  long nnz = 0;
  double kscale = 1.0;
  // workspace layout (byte offsets)
  size_t o_rhs = 0, o_y = 0, o_res = 0, o_k = 0, o_keps = 0, o_scr = 0;
  size_t o_r = 0, o_z = 0, o_p0 = 0, o_p1 = 0, o_q = 0, o_x = 0, o_V = 0, o_Zb = 0;
  size_t vstride = 0;
  // block-Jacobi inverse sets, one per distinct sigma
  struct BJSet {
    int mode = 0;          // 0 per-block (row-major), 1 distinct table + index, 2 one shared
                           // inverse, 3 per-block with rows interleaved for lanes of vec_lp rows,
                           // 4 as 3 with a storage type per chunk of 64 lane groups
    int nslot = 0;         // inverses stored
    bool table() const { return mode == 1 || mode == 2; }  // slots hold distinct inverses
    size_t o_inv = 0, o_reps = 0, o_idx = 0, o_tag = 0, o_aoff = 0;
    std::vector<int> reps; // representative block of each slot (modes 1, 2)
    std::vector<int> idx;  // slot of each block (mode 1)
    std::vector<int> tag;  // mode 4: storage type of each chunk (0 FP8 E4M3, 1 FP16, 2 FP32, 3 FP64)
    std::vector<long long> aoff;  // mode 4: byte offset of each chunk in the inverse area
  };
  std::vector<BJSet> bjsets;
  size_t o_rowptr = 0, o_col = 0, o_kval = 0, o_mval = 0;
  size_t o_ctl = 0, o_flag = 0, o_part = 0, o_part2 = 0, o_tick = 0;
  bool fdm = false;  // fast-diagonalisation preconditioner
  size_t o_fdm_Q[3] = {}, o_fdm_lam[3] = {}, o_fdm_t[2] = {};
  bool fdm_cx = false;  // complex eigenbases (periodic advection): imaginary parts below
  size_t o_fdm_Qi[3] = {}, o_fdm_lami[3] = {}, o_fdm_ti[2] = {};
  int fdm_half = 0;  // complex: x frequencies kept (real data; 0 = all), weighted x basis below
  size_t o_fdm_Qw[2] = {};
  size_t ws_bytes = 0;
  const double* force = nullptr;  // constant forcing g (caller-owned, N doubles) or null
  double react[3] = {0.0, 0.0, 0.0};  // reaction R(u) = r1 u + r2 u^2 + r3 u^3 of the steps
  bool react_on = false;
  // the FP64 terms of f besides K of the time steps (mprk_step)
  mprk::FTerms fterms() const {
    return mprk::FTerms{force, react[0], react[1], react[2], react_on ? 1 : 0};
  }
  // binding
  double* u = nullptr;
  char* ws = nullptr;
  bool bound = false;
  int static_dev = -1;              // device whose static scratch is the workspace (-1: caller's)
  unsigned long long static_gen = 0;  // that scratch's bind count when this handle bound it
  // host steering
  mprk::CtlHead* slots = nullptr;   // pinned: NSLOT poll slots + one record per stage
  hipEvent_t ev[mprk::NSLOT] = {};
  bool slot_used[mprk::NSLOT] = {};
  bool events_made = false;
  int slot_next = 0;
  int cg_chunk = 4;
  int gm_chunk = 2;
  int lookahead = 1;
  int predict_margin = 1;  // iterations enqueued beyond the last solve's count (0 with FDM)
  int start_mode = 0;        // the MPRK_START value in use (resolved from AUTO)
  bool start_slope = false;  // implicit stages after the first start from rhs + sigma k_{i-1}
  bool start_eval = false;        // f(u) evaluated at the step's start
  bool start_first_eval = false;  // the first implicit stage from rhs + sigma f(u)
  bool start_extrap = false;      // later stages from the slopes extrapolated linearly in c
  // per-stage history of the last completed solve (slot s = mprk_solve), used to enqueue each
  // pass's Krylov iterations without waiting for the device
  struct StageHist {
    bool valid = false;
    int passes = 0;
    int iters[mprk::MAXPASS] = {};
  };
  StageHist hist[MPRK_MAX_STAGES + 1];
  bool rec_pending[MPRK_MAX_STAGES + 1] = {};
  int* rec_iters = nullptr;                   // pinned: MAXPASS ints per slot
  hipEvent_t rec_ev[MPRK_MAX_STAGES + 1] = {};
  // step graph (mprk_set_step_graph): one step's launches captured once, replayed per step
  bool graph_on = false;
  bool capturing = false;             // enqueue_step is being captured (no host waits)
  hipStream_t cap_stream = nullptr;   // library-owned stream the step is captured on
  hipGraphExec_t gexec = nullptr;
  unsigned long long graph_epoch = 1;  // bumped by every change a captured step depends on
  unsigned long long gexec_epoch = 0;
  StageHist ghist[MPRK_MAX_STAGES];    // the histories the graph was captured with
  int graph_steps_last = 0;           // steps of the last mprk_step call replayed from the graph
  int last_good = 0;                  // steps combined since the previous counter sync
  // profiling
  mprk::Profiler prof;
  bool prof_on = false;
  long long worked0[mprk::KC_COUNT] = {}, units0[mprk::KC_COUNT] = {};
  // state
  double t_now = 0.0;
  long long step_count = 0;
  long long good_base = 0;
  int bad_base = 0;
  long long life_iters = 0, life_passes = 0;
  long long missed_base = 0;  // device count of missed stages at the last sync
  long long held_base = 0;    // device count of strict-held steps at the last sync
  int last_held = 0;          // steps held back by strict since the previous sync
  int last_nonfinite = 0;
  int last_missed = 0;        // stages that missed their tolerance since the previous sync

  int init(const mprk_grid& g, const mprk_operator& o, const mprk_tableau& t,
           const mprk_precisions& p, double dt_, hipStream_t s);
  ~mprk_handle();
  int make_device_resources();
  mprk::EngineCtx ctx() const;
  int poll_enqueue(int* slot);
  int poll_wait(int s, mprk::CtlHead* out);
  int stage_record(int slot);
  int update_hist(int slot);
  mprk::BJDesc bj_desc(int si) const;
  mprk::Red red() const;
  int launch_residual(const mprk::SolveCfg& cfg, const double* rhs, double* y, double* kout,
                      const mprk::FTerms& fx);
  int launch_apply64(const double* x, double* y, double sigma, int mode,
                     const mprk::FTerms& fx = mprk::FTerms{});
  int run_solve(int si, int slot, const double* rhs, double* y, double* kout, const mprk::FTerms& fx);
  int run_solve_graph(int si, int slot, const double* rhs, double* y, double* kout,
                      const mprk::FTerms& fx);
  bool graph_ready() const;
  int graph_capture();
  void graph_drop();
  int graph_steps(int nsteps, int* done);
  int enqueue_step(bool first_of_call);
  int sync_counters();
  int rebase_missed();
  int check_ws() const;
  void set_residual_tiles(int lz);
  void set_gm_form(int f, int lz);
  void fill_stats(mprk_stats* st);
};

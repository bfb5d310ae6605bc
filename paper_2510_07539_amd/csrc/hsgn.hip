// hsgn.hip -- C ABI of the gfx950 hSGN IMEX library (see include/hsgn.h).
//
// Host side: context, device workspace, the tiling of the batch, the launch
// sequence of one IMEX step, and HIP-graph capture of step blocks.
//
// Launch sequence of one step on the context's stream:
//   k_dt                                   dt per instance from the speed bound
//   stage 1: [k_stage<REDUCE> -> k_rsolve]  only if some instance has >1 tile
//            k_stage<FULL>                  all tiles; writes U^(1)
//   stage 2: same, reading U^n and U^(1); writes U^{n+1} and the next speed
//            bound.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <utility>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <cmath>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "hsgn.h"
#include "hsgn_kernels.hpp"
#include "hsgn_window.hpp"
#include "hsgn_persist.hpp"
#include "hsgn_adjoint.hpp"
#include "hsgn_explicit.hpp"
#include "hsgn_sgn.hpp"

namespace {

constexpr int kNT = 256;      // threads per stage workgroup
constexpr int kKMAX = 8;      // max cells per thread
constexpr int kTileMax = kNT * kKMAX;
constexpr int kNTR = 256;     // threads of the reduced-system solve
constexpr int kWK = 8;        // rows per thread of the windowed kernel
static_assert(kWK == hsgn::kPersistRows, "the persistent kernels are built for kWK rows");
constexpr double kWinMargin = 2.0;  // default safety factor on the decay estimate
constexpr int kAdjNT = 256;    // threads (cell positions) per reverse-stage tile

using hsgn::InstDesc;
using hsgn::StageArgs;
using hsgn::TileDesc;
using hsgn::WinDesc;

struct GraphEntry {
  int block;
  int cur;
  hipGraphExec_t exec;
};

// A roctx range over a scope of host code (the entry points, graph blocks,
// adjoint phases): shown by rocprofv3 --marker-trace, and a no-op call when
// no tool is attached.
struct Range {
  explicit Range(const char* what) { roctxRangePushA(what); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

}  // namespace

struct hsgn_ctx {
  int32_t n_inst = 0;
  int64_t ncell = 0;
  std::vector<int64_t> offsets;
  std::vector<hsgn_params> params;
  hipStream_t user_stream = nullptr;
  hipStream_t stream = nullptr;  // where work is enqueued
  bool own_stream = false;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  bool any_b = false;
  bool any_multi = false;
  int ntiles_all = 0, ntiles_multi = 0, n_multi_inst = 0;
  int64_t red_total = 0;
  // device memory
  InstDesc* d_inst = nullptr;
  TileDesc* d_tiles_all = nullptr;
  TileDesc* d_tiles_multi = nullptr;
  int32_t* d_multi = nullptr;
  double* d_b = nullptr;
  double* buf[3][4] = {};
  int cur = 0, s1 = 1, nxt = 2;
  // when set, the next step reads U^n from io_un, writes U^(1) to io_u1 and
  // U^{n+1} to io_out instead of the rotating buffers
  double* const* io_un = nullptr;
  double* const* io_u1 = nullptr;
  double* const* io_out = nullptr;
  bool io_stage1_only = false;  // the step stops after stage 1 (U^(1) only)
  bool io_skip_dt = false;      // the step reuses the current dt (fixed-step recompute)
  int order = 2;                // 2: two-stage IMEX step; 1: one first-order stage
  int scheme = HSGN_SCHEME_SEMI_IMPLICIT;  // or the explicit Heun step
  TileDesc* d_xtiles = nullptr;  // tiles of the explicit and SGN kernels (kExTile cells)
  int nxtiles = 0;
  double* d_sgn = nullptr;       // SGN: phi
  double* d_dt = nullptr;
  double* d_t = nullptr;
  unsigned long long* d_smax = nullptr;
  unsigned long long* d_umax = nullptr;
  int32_t* d_status = nullptr;
  int32_t* d_nstep = nullptr;  // steps taken per instance since the state was loaded
  double *d_rlo = nullptr, *d_rdi = nullptr, *d_rup = nullptr, *d_rrhs = nullptr,
         *d_rx = nullptr, *d_scp = nullptr, *d_sy = nullptr, *d_sv = nullptr, *d_sw = nullptr;
  std::vector<GraphEntry> graphs;
  // launch configuration the cached graphs were captured with: a re-plan
  // that reproduces it (same counts, same descriptor buffers) keeps them
  std::vector<uintptr_t> graph_sig;
  std::string err;
  bool no_alloc = false;  // hsgn_step_noalloc: every device buffer is carved from the static scratch
  // host copy of the full two-pass tiling (all instances)
  std::vector<TileDesc> h_tiles_all;
  std::vector<int32_t> h_ntiles;
  // execution plan (rebuilt by hsgn_set_state / hsgn_set_solver)
  int32_t solver = HSGN_SOLVER_AUTO;
  int win_nt = 512;
  // per-instance solver modes (HSGN_SOLVER_*), empty: every instance uses
  // the context-wide mode (solver, win_nt)
  std::vector<int32_t> h_inst_solver;
  int nwin_g[2] = {0, 0};  // windows of 256 threads (2048 rows) and of 512 (4096 rows)
  std::vector<double> h_smax, h_hmax;  // speed bound and depth maximum of the loaded state
  std::vector<int32_t> h_mode;         // per instance: 0 window, 1 two-pass
  std::vector<int32_t> h_halo;         // per instance window halo L (0 if none)
  TileDesc* d_ex_tiles = nullptr;
  TileDesc* d_ex_tiles_multi = nullptr;
  int32_t* d_ex_multi = nullptr;
  WinDesc* d_win = nullptr;
  int n_ex_tiles = 0, n_ex_tiles_multi = 0, n_ex_multi = 0, nwin = 0;
  size_t cap_ex_tiles = 0, cap_ex_tiles_multi = 0, cap_ex_multi = 0, cap_win = 0;
  unsigned long long* d_hmax = nullptr;
  // window-stage launch: one workgroup per window (HSGN_LAUNCH_GRID) or the
  // persistent kernel walking per-XCD work queues (HSGN_LAUNCH_PERSISTENT)
  int32_t launch = HSGN_LAUNCH_GRID;
  double halo_margin = kWinMargin;  // safety factor of the halo estimates
  // halo retry (hsgn_set_halo_retry): a copy of the mutable state taken at
  // the start of every block of steps, restored when a window could not
  // certify its truncation; the block then runs again with twice the margin
  bool halo_retry = false;
  int32_t n_retry = 0;                  // blocks run again since the state was loaded
  std::vector<double> h_margin_inst;    // per-instance margins grown by the retry (empty: none)
  double* rb_state = nullptr;           // 4 x ncell: h, q, m, W
  double* rb_t = nullptr;               // n_inst times
  unsigned long long* rb_sp = nullptr;  // 3 x n_inst: speed bounds, depth maxima
  int32_t* rb_st = nullptr;             // 2 x n_inst: status, step counts
  // 2 x 9 queue counters of the persistent kernel: the first set for the
  // library's stream, the second for the adjoint's recompute stream (zero
  // between launches: every launch resets its own)
  int32_t* d_queue = nullptr;
  int n_cu = 0;              // compute units of the device
  int occ[2][2] = {};        // resident workgroups per CU: [geometry][stage - 1], 0 = not read yet
  // adjoint workspace (allocated by the first hsgn_adjoint call)
  struct Adj {
    int nseg = 0;
    size_t tape_steps = 0;     // steps the tape holds (tape buffers x K)
    int64_t tape_budget = -1;  // bytes for the tapes (hsgn_set_adjoint_tape_bytes; < 0: auto)
    int64_t nres = 0;
    double* sys = nullptr;     // 9 x ncell: transposed rows, rhs, lam, solver scratch
    double* tape = nullptr;    // tape_steps x 8 x ncell (U^n, U^(1) per step)
    double* ckpt = nullptr;    // (nseg + 1) x 4 x ncell
    double* res = nullptr;     // n_inst x nsteps x n_gauge residuals
    double* st = nullptr;      // 12 x ncell adjoint states + 1 x ncell bed adjoint
    hsgn::adj::TileA* tiles = nullptr;
    int ntiles = 0;
    // the recompute of segment s - 1 runs on its own stream while the
    // reverse sweep of segment s runs on the library's stream
    hipStream_t rstream = nullptr;
    hipEvent_t ev_fwd = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};
  } adj;
};

namespace {

int fail(hsgn_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

#define HIPCHK(ctx, call)                                                                 \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail((ctx), HSGN_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));       \
  } while (0)

template <typename T>
int dmalloc(hsgn_ctx* c, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return HSGN_OK;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(c, HSGN_ENOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T),
                hipGetErrorString(e));
  }
  return HSGN_OK;
}

void free_all(hsgn_ctx* c) {
  for (auto& g : c->graphs) hipGraphExecDestroy(g.exec);
  c->graphs.clear();
  void* ptrs[] = {c->d_inst, c->d_tiles_all, c->d_tiles_multi, c->d_multi, c->d_b,
                  c->d_dt, c->d_t, c->d_smax, c->d_umax, c->d_status, c->d_nstep, c->d_rlo,
                  c->d_rdi,
                  c->d_rup, c->d_rrhs, c->d_rx, c->d_scp, c->d_sy, c->d_sv, c->d_sw,
                  c->d_ex_tiles, c->d_ex_tiles_multi, c->d_ex_multi, c->d_win, c->d_hmax,
                  c->d_xtiles, c->d_sgn, c->d_queue, c->rb_state, c->rb_t, c->rb_sp,
                  c->rb_st};
  for (void* p : ptrs)
    if (p) hipFree(p);
  for (int i = 0; i < 3; ++i)
    for (int f = 0; f < 4; ++f)
      if (c->buf[i][f]) hipFree(c->buf[i][f]);
  double* ap[] = {c->adj.sys, c->adj.tape, c->adj.ckpt, c->adj.res, c->adj.st};
  for (double* p : ap)
    if (p) hipFree(p);
  if (c->adj.tiles) hipFree(c->adj.tiles);
  if (c->adj.rstream) hipStreamDestroy(c->adj.rstream);
  hipEvent_t aev[5] = {c->adj.ev_fwd, c->adj.ev_rec[0], c->adj.ev_rec[1], c->adj.ev_rev[0],
                       c->adj.ev_rev[1]};
  for (hipEvent_t e : aev)
    if (e) hipEventDestroy(e);
  if (c->ev_in) hipEventDestroy(c->ev_in);
  if (c->ev_out) hipEventDestroy(c->ev_out);
  if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
}

// Make the library stream wait for prior work of the caller's stream.
int enter(hsgn_ctx* c) {
  if (c->stream == c->user_stream) return HSGN_OK;
  HIPCHK(c, hipEventRecord(c->ev_in, c->user_stream));
  HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_in, 0));
  return HSGN_OK;
}
// Make the caller's stream wait for the library's work.
int leave(hsgn_ctx* c) {
  if (c->stream == c->user_stream) return HSGN_OK;
  HIPCHK(c, hipEventRecord(c->ev_out, c->stream));
  HIPCHK(c, hipStreamWaitEvent(c->user_stream, c->ev_out, 0));
  return HSGN_OK;
}

template <bool BED, int STAGE, bool REDUCE>
void launch_stage(hsgn_ctx* c, const StageArgs& a, int ntiles) {
  hipLaunchKernelGGL((hsgn::k_stage<kNT, kKMAX, BED, STAGE, REDUCE>), dim3(ntiles), dim3(kNT), 0,
                     c->stream, a);
}

template <int STAGE>
void launch_stage_any(hsgn_ctx* c, const StageArgs& a, int ntiles, bool reduce) {
  if (c->any_b) {
    if (reduce) launch_stage<true, STAGE, true>(c, a, ntiles);
    else launch_stage<true, STAGE, false>(c, a, ntiles);
  } else {
    if (reduce) launch_stage<false, STAGE, true>(c, a, ntiles);
    else launch_stage<false, STAGE, false>(c, a, ntiles);
  }
}

StageArgs stage_args(hsgn_ctx* c, int stage) {
  StageArgs a;
  std::memset(&a, 0, sizeof a);
  double* const* un = c->io_un ? c->io_un : c->buf[c->cur];
  double* const* u1 = c->io_u1 ? c->io_u1 : c->buf[c->s1];
  // first-order scheme: its single stage writes U^{n+1}
  double* const* out = (stage == 1 && c->order != 1)
                           ? u1
                           : (c->io_out ? c->io_out : c->buf[c->nxt]);
  a.un_h = un[0]; a.un_q = un[1]; a.un_m = un[2]; a.un_W = un[3];
  a.u1_h = u1[0]; a.u1_q = u1[1]; a.u1_m = u1[2]; a.u1_W = u1[3];
  a.o_h = out[0]; a.o_q = out[1]; a.o_m = out[2]; a.o_W = out[3];
  a.b = c->d_b;
  a.inst = c->d_inst;
  a.dt = c->d_dt;
  a.tau_factor = c->order == 1 ? 1.0 : hsgn::kGamma;
  a.slope = c->order == 1 ? 0.0 : 0.25;
  a.rlo = c->d_rlo; a.rdi = c->d_rdi; a.rup = c->d_rup; a.rrhs = c->d_rrhs;
  a.rx = c->d_rx;
  a.smax = c->d_smax;
  a.umax = c->d_umax;
  a.status = c->d_status;
  return a;
}

// Enqueue one IMEX step (no synchronisation), then rotate the buffers.
// With `tm`, every launch is bracketed by a pair of events (kind k).
template <int NT, int K, bool BED>
hipError_t launch_win_b(hsgn_ctx* c, hsgn::WinArgs& w, int stage) {
  const int g = NT == 512 ? 1 : 0;
  if (c->launch == HSGN_LAUNCH_PERSISTENT && c->d_queue) {
    int& occ = c->occ[g][stage - 1];
    if (occ == 0 && hsgn::win_persist_occupancy(NT, BED, stage, &occ) != hipSuccess) occ = 0;
    if (occ > 0 && c->n_cu >= 8) {
      // as many workgroups as are resident at once (a multiple of 8, so
      // that block b runs on XCD b mod 8), at most one per window
      const int grid = std::min(8 * w.xcd_stride, (c->n_cu / 8) * 8 * occ);
      w.queue = c->d_queue + (c->adj.rstream && c->stream == c->adj.rstream ? 9 : 0);
      return hsgn::launch_win_persist(NT, BED, stage, grid, c->stream, w);
    }
  }
  const int grid = 8 * w.xcd_stride;
  if (stage == 1) hipLaunchKernelGGL((hsgn::k_win<NT, K, BED, 1>), dim3(grid), dim3(NT), 0, c->stream, w);
  else hipLaunchKernelGGL((hsgn::k_win<NT, K, BED, 2>), dim3(grid), dim3(NT), 0, c->stream, w);
  return hipSuccess;  // errors of this launch reach hipGetLastError
}

template <int NT, int K>
hipError_t launch_win(hsgn_ctx* c, hsgn::WinArgs& w, int stage) {
  if (c->any_b) return launch_win_b<NT, K, true>(c, w, stage);
  return launch_win_b<NT, K, false>(c, w, stage);
}

int enqueue_step(hsgn_ctx* c, std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>>* tm = nullptr) {
  bool marks_ok = true;  // timing events (measurement variant only)
  auto mark = [&](int kind, bool begin) {
    if (!tm || !marks_ok) return;
    if (begin) {
      hipEvent_t a = nullptr, b = nullptr;
      marks_ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
      tm->push_back({kind, {a, b}});
      if (marks_ok) marks_ok = hipEventRecord(a, c->stream) == hipSuccess;
    } else {
      marks_ok = hipEventRecord(tm->back().second.second, c->stream) == hipSuccess;
    }
  };
  const int nb = (c->n_inst + 255) / 256;
  if (!c->io_skip_dt) {
    mark(HSGN_K_DT, true);
    hipLaunchKernelGGL(hsgn::k_dt, dim3(nb), dim3(256), 0, c->stream, c->n_inst, c->d_inst, c->d_dt,
                       c->d_t, c->d_smax, c->d_umax, c->d_status, c->d_nstep);
    mark(HSGN_K_DT, false);
  }
  if (c->scheme == HSGN_SCHEME_SGN) {
    // Heun on the SGN operator: solve of the phi system (rows formed in the
    // solve; windowed single pass, or exact on the two-pass tiling where no
    // window is planned), flux update with the source h phi
    double* const* un = c->buf[c->cur];
    double* const* u1 = c->buf[c->s1];
    double* const* out = c->buf[c->nxt];
    hsgn::SgnArgs x;
    std::memset(&x, 0, sizeof x);
    x.un_h = un[0]; x.un_q = un[1]; x.un_m = un[2]; x.un_W = un[3];
    x.phi = c->d_sgn;
    x.inst = c->d_inst;
    x.tiles = c->d_xtiles;
    x.dt = c->d_dt;
    x.smax = c->d_smax;
    x.umax = c->d_umax;
    x.status = c->d_status;
    // exact tiled solve of phi on the two-pass tiling (tiles of kTileMax rows)
    hsgn::SgnTriArgs ta;
    ta.inst = c->d_inst;
    ta.dt = c->d_dt;
    ta.phi = c->d_sgn;
    ta.rlo = c->d_rlo; ta.rdi = c->d_rdi; ta.rup = c->d_rup; ta.rrhs = c->d_rrhs;
    ta.rx = c->d_rx;
    ta.status = c->d_status;
    hsgn::SgnWinArgs wa;
    wa.inst = c->d_inst;
    wa.win = c->d_win;
    wa.dt = c->d_dt;
    wa.phi = c->d_sgn;
    wa.status = c->d_status;
    for (int stage = 1; stage <= 2; ++stage) {
      double* const* in = stage == 1 ? un : u1;
      double* const* o = stage == 1 ? u1 : out;
      x.in_h = in[0]; x.in_q = in[1];
      x.o_h = o[0]; x.o_q = o[1]; x.o_m = o[2]; x.o_W = o[3];
      ta.h = in[0];
      ta.q = in[1];
      mark(HSGN_K_SGN_SOLVE, true);
      if (c->nwin > 0) {  // windowed single pass
        wa.h = in[0];
        wa.q = in[1];
        hipLaunchKernelGGL((hsgn::k_sgn_win<512, kWK>), dim3(c->nwin), dim3(512), 0, c->stream, wa);
      }
      // the other instances: exact solve on the two-pass tiling
      if (c->n_ex_multi > 0) {
        ta.tiles = c->d_ex_tiles_multi;
        hipLaunchKernelGGL((hsgn::k_sgn_tri<kTileMax / 8, 8, true>), dim3(c->n_ex_tiles_multi),
                           dim3(kTileMax / 8), 0, c->stream, ta);
        hipLaunchKernelGGL(hsgn::k_rsolve<kNTR>, dim3(c->n_ex_multi), dim3(kNTR), 0, c->stream,
                           c->d_inst, c->d_ex_multi, c->d_dt, c->d_rlo, c->d_rdi, c->d_rup,
                           c->d_rrhs, c->d_rx, c->d_scp, c->d_sy, c->d_sv, c->d_sw);
      }
      if (c->n_ex_tiles > 0) {
        ta.tiles = c->d_ex_tiles;
        hipLaunchKernelGGL((hsgn::k_sgn_tri<kTileMax / 8, 8, false>), dim3(c->n_ex_tiles),
                           dim3(kTileMax / 8), 0, c->stream, ta);
      }
      mark(HSGN_K_SGN_SOLVE, false);
      mark(HSGN_K_SGN_UPDATE, true);
      if (stage == 1)
        hipLaunchKernelGGL((hsgn::k_sgn_update<hsgn::kSgnNT, hsgn::kSgnK, 1>), dim3(c->nxtiles),
                           dim3(hsgn::kSgnNT), 0, c->stream, x);
      else
        hipLaunchKernelGGL((hsgn::k_sgn_update<hsgn::kSgnNT, hsgn::kSgnK, 2>), dim3(c->nxtiles),
                           dim3(hsgn::kSgnNT), 0, c->stream, x);
      mark(HSGN_K_SGN_UPDATE, false);
    }
    HIPCHK(c, hipGetLastError());
    if (!marks_ok) return fail(c, HSGN_EHIP, "hsgn_step_timed: timing events failed");
    const int old = c->cur;
    c->cur = c->nxt;
    c->nxt = old;
    return HSGN_OK;
  }
  if (c->scheme == HSGN_SCHEME_EXPLICIT) {
    // Heun: U1 = U^n + dt L(U^n), U^{n+1} = (U^n + U1 + dt L(U1)) / 2
    double* const* un = c->buf[c->cur];
    double* const* u1 = c->buf[c->s1];
    double* const* out = c->buf[c->nxt];
    hsgn::ExArgs x;
    std::memset(&x, 0, sizeof x);
    x.un_h = un[0]; x.un_q = un[1]; x.un_m = un[2]; x.un_W = un[3];
    x.inst = c->d_inst;
    x.tiles = c->d_xtiles;
    x.dt = c->d_dt;
    x.smax = c->d_smax;
    x.umax = c->d_umax;
    x.status = c->d_status;
    x.in_h = un[0]; x.in_q = un[1]; x.in_m = un[2]; x.in_W = un[3];
    x.o_h = u1[0]; x.o_q = u1[1]; x.o_m = u1[2]; x.o_W = u1[3];
    mark(HSGN_K_EX1, true);
    hipLaunchKernelGGL((hsgn::k_ex<hsgn::kExNT, hsgn::kExK, 1>), dim3(c->nxtiles),
                       dim3(hsgn::kExNT), 0, c->stream, x);
    mark(HSGN_K_EX1, false);
    x.in_h = u1[0]; x.in_q = u1[1]; x.in_m = u1[2]; x.in_W = u1[3];
    x.o_h = out[0]; x.o_q = out[1]; x.o_m = out[2]; x.o_W = out[3];
    mark(HSGN_K_EX2, true);
    hipLaunchKernelGGL((hsgn::k_ex<hsgn::kExNT, hsgn::kExK, 2>), dim3(c->nxtiles),
                       dim3(hsgn::kExNT), 0, c->stream, x);
    mark(HSGN_K_EX2, false);
    HIPCHK(c, hipGetLastError());
    if (!marks_ok) return fail(c, HSGN_EHIP, "hsgn_step_timed: timing events failed");
    const int old = c->cur;
    c->cur = c->nxt;
    c->nxt = old;
    return HSGN_OK;
  }
  const int last_stage = (c->io_stage1_only || c->order == 1) ? 1 : 2;
  for (int stage = 1; stage <= last_stage; ++stage) {
    StageArgs a = stage_args(c, stage);
    if (c->n_ex_multi > 0) {
      a.tiles = c->d_ex_tiles_multi;
      mark(stage == 1 ? HSGN_K_REDUCE1 : HSGN_K_REDUCE2, true);
      if (stage == 1) launch_stage_any<1>(c, a, c->n_ex_tiles_multi, true);
      else launch_stage_any<2>(c, a, c->n_ex_tiles_multi, true);
      mark(stage == 1 ? HSGN_K_REDUCE1 : HSGN_K_REDUCE2, false);
      mark(stage == 1 ? HSGN_K_RSOLVE1 : HSGN_K_RSOLVE2, true);
      hipLaunchKernelGGL(hsgn::k_rsolve<kNTR>, dim3(c->n_ex_multi), dim3(kNTR), 0, c->stream,
                         c->d_inst, c->d_ex_multi, c->d_dt, c->d_rlo, c->d_rdi, c->d_rup,
                         c->d_rrhs, c->d_rx, c->d_scp, c->d_sy, c->d_sv, c->d_sw);
      mark(stage == 1 ? HSGN_K_RSOLVE1 : HSGN_K_RSOLVE2, false);
    }
    if (c->n_ex_tiles > 0) {
      a.tiles = c->d_ex_tiles;
      mark(stage == 1 ? HSGN_K_STAGE1 : HSGN_K_STAGE2, true);
      if (stage == 1) launch_stage_any<1>(c, a, c->n_ex_tiles, false);
      else launch_stage_any<2>(c, a, c->n_ex_tiles, false);
      mark(stage == 1 ? HSGN_K_STAGE1 : HSGN_K_STAGE2, false);
    }
    if (c->nwin > 0) {
      // one launch per window geometry in use: the window list holds the
      // 2048-row windows first, then the 4096-row ones
      mark(stage == 1 ? HSGN_K_WIN1 : HSGN_K_WIN2, true);
      for (int g = 0; g < 2; ++g) {
        if (c->nwin_g[g] == 0) continue;
        hsgn::WinArgs w;
        w.s = a;
        w.win = c->d_win + (g == 0 ? 0 : c->nwin_g[0]);
        w.nwin = c->nwin_g[g];
        w.xcd_stride = (w.nwin + 7) / 8;
        w.queue = nullptr;
        const hipError_t le = g == 1 ? launch_win<512, kWK>(c, w, stage) : launch_win<256, kWK>(c, w, stage);
        if (le != hipSuccess) return fail(c, HSGN_EHIP, "window launch: %s", hipGetErrorString(le));
      }
      mark(stage == 1 ? HSGN_K_WIN1 : HSGN_K_WIN2, false);
    }
  }
  if (c->order == 1) {  // speed bound of the new state for the next step's dt
    double* const* un = c->io_out ? c->io_out : c->buf[c->nxt];
    hipLaunchKernelGGL(hsgn::k_speed<256>, dim3(c->ntiles_all), dim3(256), 0, c->stream,
                       c->d_inst, c->d_tiles_all, un[0], un[1], c->d_smax, c->d_umax, c->d_hmax);
  }
  HIPCHK(c, hipGetLastError());
  if (!marks_ok) return fail(c, HSGN_EHIP, "hsgn_step_timed: timing events failed");
  const int old = c->cur;
  c->cur = c->nxt;
  c->nxt = old;
  return HSGN_OK;
}


// One step between explicit buffers (no rotation of the state buffers);
// with out == NULL only stage 1 runs.
int enqueue_step_io(hsgn_ctx* c, double* const* un, double* const* u1, double* const* out) {
  c->io_un = un;
  c->io_u1 = u1;
  c->io_out = out;
  c->io_stage1_only = out == nullptr;
  const int cur = c->cur, nxt = c->nxt;
  const int rc = enqueue_step(c);
  c->io_un = c->io_u1 = c->io_out = nullptr;
  c->io_stage1_only = false;
  c->cur = cur;
  c->nxt = nxt;
  return rc;
}

// Halo width (window rows beyond the core on a truncated side) for one
// instance: the depth system behaves like I + r beta (second difference),
// whose inverse decays per cell by rho = q - sqrt(q^2 - 1), q = 1 + 1/(2 r beta);
// r beta is estimated from the loaded state at rest-state beta
// (g h + (2 lambda / 3) / beta_1) at the deepest cell, times a margin.  The
// halo makes rho^L <= 2^-60.  The kernel verifies the truncation on every
// tile and flags the instance if it is not negligible.
int halo_width(const hsgn_params& p, double smax, double hmax, double tau_factor,
               double margin) {
  const double dt = p.dt_fixed > 0 ? p.dt_fixed : p.cfl * p.dx / smax;
  const double tau = tau_factor * dt;
  const double b1 = 1.0 + p.lambda * tau * tau / (hmax * hmax);
  const double beta = p.g * hmax + (2.0 * p.lambda / 3.0) / b1;
  const double R = margin * (tau / p.dx) * (tau / p.dx) * beta;
  if (!(R > 0.0) || !std::isfinite(R)) return 1 << 30;
  const double q = 1.0 + 0.5 / R;
  const double rho = q - std::sqrt(q * q - 1.0);
  double L = 60.0 * std::log(2.0) / (-std::log(rho));
  if (!(L < 1e8)) return 1 << 30;
  int Li = (int)std::ceil(L);
  Li = ((Li + kWK - 1) / kWK) * kWK;
  return Li < kWK ? kWK : Li;
}

// Halo of the windowed phi solve of the SGN scheme: a phi row has the
// diagonal h + c3 (H- + H+) and the couplings -c3 H-+ (c3 H = h^3 / (3 dx^2)
// at a uniform depth), so at the deepest cell the inverse decays per cell by
// rho = q - sqrt(q^2 - 1), q = 1 + h / (2 c3 H); the estimate multiplies c3 H
// there by the margin (by default 2: the depth may grow by a quarter before
// it fails).  The halo makes rho^L <= 2^-60; the kernel certifies every
// window.
int sgn_halo_width(const hsgn_params& p, double hmax, double margin) {
  const double c3H = margin * hmax * hmax * hmax / (3.0 * p.dx * p.dx);
  if (!(c3H > 0.0) || !std::isfinite(c3H)) return 1 << 30;
  const double q = 1.0 + hmax / (2.0 * c3H);
  const double rho = q - std::sqrt(q * q - 1.0);
  double L = 60.0 * std::log(2.0) / (-std::log(rho));
  if (!(L < 1e8)) return 1 << 30;
  int Li = (int)std::ceil(L);
  Li = ((Li + kWK - 1) / kWK) * kWK;
  return Li < kWK ? kWK : Li;
}

template <typename T>
int upload(hsgn_ctx* c, T** d, size_t* cap, const std::vector<T>& h) {
  if (h.size() > *cap && c->no_alloc)
    return fail(c, HSGN_EINVAL, "plan list of %zu entries exceeds the static scratch (%zu)",
                h.size(), *cap);
  if (h.size() > *cap) {
    if (*d) hipFree(*d);
    *d = nullptr;
    *cap = 0;
    int rc = dmalloc(c, d, h.size());
    if (rc) return rc;
    *cap = h.size();
  }
  if (!h.empty())
    HIPCHK(c, hipMemcpyAsync(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  return HSGN_OK;
}

// Decide per instance between the windowed single pass and the exact
// two-pass solve, and build the launch lists.
int make_plan(hsgn_ctx* c) {
  std::vector<TileDesc> ex_all, ex_multi;
  std::vector<int32_t> ex_inst;
  std::vector<WinDesc> win, win512;  // windows of 2048 and of 4096 rows
  c->h_mode.assign(c->n_inst, 1);
  c->h_halo.assign(c->n_inst, 0);
  size_t tpos = 0;
  for (int j = 0; j < c->n_inst; ++j) {
    const int n = (int)(c->offsets[j + 1] - c->offsets[j]);
    const hsgn_params& p = c->params[j];
    const int nt = c->h_ntiles[j];
    bool use_win = false;
    std::vector<WinDesc> wj;
    // this instance's mode: its own, or the context's
    const int32_t mj = !c->h_inst_solver.empty()
                           ? c->h_inst_solver[j]
                           : (c->solver == HSGN_SOLVER_EXACT
                                  ? HSGN_SOLVER_EXACT
                                  : (c->win_nt == 256 ? HSGN_SOLVER_AUTO_SMALL : HSGN_SOLVER_AUTO));
    // the SGN scheme's phi solve takes windows of 4096 rows (512 threads x
    // 8 rows, two workgroups per CU: measured 4 % faster than 2048 rows)
    const bool sgn = c->scheme == HSGN_SCHEME_SGN;
    const int WN = (!sgn && mj == HSGN_SOLVER_AUTO_SMALL ? 256 : 512) * kWK;
    const int Lmax = WN / 4;
    // the halo estimate of the loaded state (reported for every instance)
    const bool have_state = !c->h_smax.empty() && c->h_smax[j] > 0 && c->h_hmax[j] > 0;
    const double margin = c->h_margin_inst.empty() ? c->halo_margin : c->h_margin_inst[j];
    const int L = !have_state ? 0
                  : sgn ? sgn_halo_width(p, c->h_hmax[j], margin)
                        : halo_width(p, c->h_smax[j], c->h_hmax[j],
                                     c->order == 1 ? 1.0 : hsgn::kGamma, margin);
    c->h_halo[j] = L;
    if (mj != HSGN_SOLVER_EXACT && have_state) {
      auto add = [&](int ws, int wl, int cs, int cl, int flags) {
        WinDesc d;
        std::memset(&d, 0, sizeof d);
        d.off = c->offsets[j]; d.n = n; d.bc = p.bc; d.has_b = p.has_bathymetry ? 1 : 0;
        d.inst = j; d.ws = ws; d.wl = wl; d.cs = cs; d.cl = cl; d.flags = flags;
        wj.push_back(d);
      };
      if (p.bc != 0) {  // transmissive
        if (n <= WN) {
          add(0, n, 0, n, 0);
          use_win = true;
        } else if (L <= Lmax) {
          if (n <= 2 * WN - 2 * L) {
            add(0, WN, 0, n / 2, 2);
            add(n - WN, WN, n / 2, n - n / 2, 1);
          } else {
            add(0, WN, 0, WN - L, 2);
            const int M = n - 2 * WN + 2 * L;
            const int C = WN - 2 * L - kWK;
            const int nm = (M + C - 1) / C;
            for (int k = 0; k < nm; ++k) {
              const int cs = (WN - L) + (int)((int64_t)k * M / nm);
              const int ce = (WN - L) + (int)((int64_t)(k + 1) * M / nm);
              const int ws = cs - L;
              const int wl = ((ce + L - ws + kWK - 1) / kWK) * kWK;
              add(ws, wl, cs, ce - cs, 3);
            }
            add(n - WN, WN, n - WN + L, WN - L, 1);
          }
          use_win = true;
        }
      } else {  // periodic
        if (n + 2 * L <= WN) {
          add(-((WN - n) / 2), WN, 0, n, 3);
          use_win = true;
        } else if (L <= Lmax) {
          const int C = WN - 2 * L - kWK;
          const int ntw = (n + C - 1) / C;
          for (int k = 0; k < ntw; ++k) {
            const int cs = (int)((int64_t)k * n / ntw);
            const int ce = (int)((int64_t)(k + 1) * n / ntw);
            const int wl = ((ce - cs + 2 * L + kWK - 1) / kWK) * kWK;
            add(cs - L, wl, cs, ce - cs, 3);
          }
          use_win = true;
        }
      }
    }
    if (use_win) {
      c->h_mode[j] = 0;
      std::vector<WinDesc>& dst = WN == 2048 ? win : win512;
      dst.insert(dst.end(), wj.begin(), wj.end());
    } else {
      for (int k = 0; k < nt; ++k) {
        ex_all.push_back(c->h_tiles_all[tpos + k]);
        if (nt > 1) ex_multi.push_back(c->h_tiles_all[tpos + k]);
      }
      if (nt > 1) ex_inst.push_back(j);
    }
    tpos += nt;
  }
  c->nwin_g[0] = (int)win.size();
  c->nwin_g[1] = (int)win512.size();
  win.insert(win.end(), win512.begin(), win512.end());
  int rc = upload(c, &c->d_ex_tiles, &c->cap_ex_tiles, ex_all);
  if (!rc) rc = upload(c, &c->d_ex_tiles_multi, &c->cap_ex_tiles_multi, ex_multi);
  if (!rc) rc = upload(c, &c->d_ex_multi, &c->cap_ex_multi, ex_inst);
  if (!rc) rc = upload(c, &c->d_win, &c->cap_win, win);
  if (rc) return rc;
  c->n_ex_tiles = (int)ex_all.size();
  c->n_ex_tiles_multi = (int)ex_multi.size();
  c->n_ex_multi = (int)ex_inst.size();
  c->nwin = (int)win.size();
  // uploads read host vectors that die here
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const std::vector<uintptr_t> sig = {
      (uintptr_t)c->nwin_g[0], (uintptr_t)c->nwin_g[1], (uintptr_t)c->n_ex_tiles,
      (uintptr_t)c->n_ex_tiles_multi,
      (uintptr_t)c->n_ex_multi, (uintptr_t)c->nwin, (uintptr_t)c->d_ex_tiles,
      (uintptr_t)c->d_ex_tiles_multi, (uintptr_t)c->d_ex_multi, (uintptr_t)c->d_win};
  if (sig != c->graph_sig) {
    for (auto& g : c->graphs) hipGraphExecDestroy(g.exec);
    c->graphs.clear();
    c->graph_sig = sig;
  }
  return HSGN_OK;
}

// Host layout of a batch (shared by hsgn_init and hsgn_step_noalloc): the
// parameters checked, the per-instance descriptors and the two-pass tiling
// (tiles of at most kTileMax cells), with the context's counts set from them.
struct Layout {
  std::vector<InstDesc> inst;
  std::vector<TileDesc> tall, tmulti, xt;
  std::vector<int32_t> multi;
};

int build_layout(hsgn_ctx* c, int32_t n_inst, const int64_t* offsets, const hsgn_params* params,
                 const double* d_b, Layout& lay) {
  int rc = HSGN_OK;
  c->n_inst = n_inst;
  c->offsets.assign(offsets, offsets + n_inst + 1);
  c->params.assign(params, params + n_inst);
  if (offsets[0] != 0) rc = fail(c, HSGN_EINVAL, "offsets[0] must be 0");
  std::vector<InstDesc>& inst = lay.inst;
  std::vector<TileDesc>& tall = lay.tall;
  std::vector<TileDesc>& tmulti = lay.tmulti;
  std::vector<TileDesc>& xt = lay.xt;
  std::vector<int32_t>& multi = lay.multi;
  inst.assign(n_inst, InstDesc{});
  int64_t red = 0;
  for (int j = 0; j < n_inst && rc == HSGN_OK; ++j) {
    const int64_t n = offsets[j + 1] - offsets[j];
    const hsgn_params& p = params[j];
    if (n < 4 || n > (int64_t)1 << 30) {
      rc = fail(c, HSGN_EINVAL, "instance %d has %lld cells (need 4 .. 2^30)", j, (long long)n);
      break;
    }
    if (!(p.g > 0) || !(p.lambda > 0) || !(p.dx > 0) || (p.bc != 0 && p.bc != 1) ||
        (!(p.dt_fixed > 0) && !(p.cfl > 0))) {
      rc = fail(c, HSGN_EINVAL, "instance %d: invalid parameters", j);
      break;
    }
    if (p.has_bathymetry && !d_b) {
      rc = fail(c, HSGN_EINVAL, "instance %d uses a bed but d_b is NULL", j);
      break;
    }
    const int ord = p.order == 1 ? 1 : 2;
    if ((p.order != 0 && p.order != 1 && p.order != 2) || (j > 0 && ord != c->order)) {
      rc = fail(c, HSGN_EINVAL, "instance %d: order must be 1 or 2 and the same for every "
                "instance", j);
      break;
    }
    c->order = ord;
    if ((p.scheme != HSGN_SCHEME_SEMI_IMPLICIT && p.scheme != HSGN_SCHEME_EXPLICIT &&
         p.scheme != HSGN_SCHEME_SGN) ||
        (j > 0 && p.scheme != c->scheme)) {
      rc = fail(c, HSGN_EINVAL, "instance %d: scheme must be 0, 1 or 2 and the same for every "
                "instance", j);
      break;
    }
    c->scheme = p.scheme;
    if (p.scheme != HSGN_SCHEME_SEMI_IMPLICIT && (p.has_bathymetry || ord != 2)) {
      rc = fail(c, HSGN_EINVAL, "instance %d: the explicit and SGN schemes need a flat bottom "
                "and order 0 or 2", j);
      break;
    }
    InstDesc& d = inst[j];
    std::memset(&d, 0, sizeof d);
    d.off = offsets[j];
    d.n = (int32_t)n;
    d.bc = p.bc;
    d.has_b = p.has_bathymetry ? 1 : 0;
    d.g = p.g; d.lam = p.lambda; d.dx = p.dx; d.cfl = p.cfl; d.mcfl = p.mcfl;
    d.dt_fixed = p.dt_fixed; d.t_end = p.t_end;
    c->any_b |= d.has_b != 0;
    const int nt = (int)((n + kTileMax - 1) / kTileMax);
    d.ntiles = nt;
    d.red_off = nt > 1 ? (int32_t)red : -1;
    for (int k = 0; k < nt; ++k) {
      TileDesc t;
      t.inst = j;
      t.tidx = k;
      t.start = (int32_t)((n * k) / nt);
      t.len = (int32_t)((n * (k + 1)) / nt) - t.start;
      tall.push_back(t);
      if (nt > 1) tmulti.push_back(t);
    }
    if (nt > 1) {
      multi.push_back(j);
      red += 2 * nt;
    }
    if (p.scheme != HSGN_SCHEME_SEMI_IMPLICIT) {  // tiles of the explicit and SGN kernels
      const int nx = (int)((n + hsgn::kExTile - 1) / hsgn::kExTile);
      for (int k = 0; k < nx; ++k) {
        TileDesc t;
        t.inst = j;
        t.tidx = k;
        t.start = (int32_t)((n * k) / nx);
        t.len = (int32_t)((n * (k + 1)) / nx) - t.start;
        xt.push_back(t);
      }
    }
    c->ncell += n;
  }
  if (rc == HSGN_OK && red > INT32_MAX) rc = fail(c, HSGN_EINVAL, "reduced system too large");
  c->h_tiles_all = tall;
  c->h_ntiles.resize(n_inst);
  for (int j = 0; j < n_inst && rc == HSGN_OK; ++j) c->h_ntiles[j] = inst[j].ntiles;
  c->ntiles_all = (int)tall.size();
  c->ntiles_multi = (int)tmulti.size();
  c->n_multi_inst = (int)multi.size();
  c->any_multi = c->n_multi_inst > 0;
  c->red_total = red;
  c->nxtiles = (int)xt.size();
  return rc;
}

// The graph of `block` steps from the current buffer rotation, captured on
// first use (capture executes nothing, so the rotation is restored after it).
int graph_of(hsgn_ctx* c, int block, hipGraphExec_t* out) {
  for (auto& g : c->graphs)
    if (g.block == block && g.cur == c->cur) {
      *out = g.exec;
      return HSGN_OK;
    }
  const int cur0 = c->cur, nxt0 = c->nxt;
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  int erc = HSGN_OK;
  for (int s = 0; s < block && erc == HSGN_OK; ++s) erc = enqueue_step(c);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(c->stream, &graph);
  c->cur = cur0;
  c->nxt = nxt0;
  if (erc) return erc;
  if (e != hipSuccess) return fail(c, HSGN_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(c, HSGN_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  c->graphs.push_back({block, c->cur, exec});
  *out = exec;
  return HSGN_OK;
}

// Copy the mutable state (the current buffers' four fields, times, speed
// bounds, depth maxima, status flags, step counts) to the retry copy
// (to_copy) or back (!to_copy), on the library's stream.
int retry_copy(hsgn_ctx* c, bool to_copy) {
  const size_t nc = (size_t)c->ncell, ni = (size_t)c->n_inst;
  auto cp = [&](void* keep, void* live, size_t bytes) {
    return hipMemcpyAsync(to_copy ? keep : live, to_copy ? live : keep, bytes,
                          hipMemcpyDeviceToDevice, c->stream);
  };
  for (int f = 0; f < 4; ++f)
    HIPCHK(c, cp(c->rb_state + f * nc, c->buf[c->cur][f], nc * sizeof(double)));
  HIPCHK(c, cp(c->rb_t, c->d_t, ni * sizeof(double)));
  HIPCHK(c, cp(c->rb_sp, c->d_smax, ni * sizeof(unsigned long long)));
  HIPCHK(c, cp(c->rb_sp + ni, c->d_umax, ni * sizeof(unsigned long long)));
  HIPCHK(c, cp(c->rb_sp + 2 * ni, c->d_hmax, ni * sizeof(unsigned long long)));
  HIPCHK(c, cp(c->rb_st, c->d_status, ni * sizeof(int32_t)));
  HIPCHK(c, cp(c->rb_st + ni, c->d_nstep, ni * sizeof(int32_t)));
  return HSGN_OK;
}

constexpr double kMaxMargin = 64.0;  // the largest halo margin (hsgn_set_halo_margin)

// Enqueue a block of steps (chunk).  With the halo retry on (semi-implicit
// and SGN schemes, whose windows certify their truncation), the mutable
// state is copied first and the status read after the block (synchronising
// the stream); if a window flagged its truncation, the copy is restored,
// the halo margin of each flagged instance doubled (up to kMaxMargin; the
// other instances keep theirs) and the solver re-planned, and the block
// runs again.  Other flags, and a window flag at the largest margin, are
// left for hsgn_status.
template <class Chunk>
int run_retrying(hsgn_ctx* c, Chunk chunk) {
  if (!c->halo_retry || c->scheme == HSGN_SCHEME_EXPLICIT) return chunk();
  const size_t nc = (size_t)c->ncell, ni = (size_t)c->n_inst;
  int rc = HSGN_OK;
  if (!c->rb_state || !c->rb_t || !c->rb_sp || !c->rb_st) {  // first use, or a failed one
    void* old[4] = {c->rb_state, c->rb_t, c->rb_sp, c->rb_st};
    for (void* q : old)
      if (q) (void)hipFree(q);
    c->rb_state = nullptr;
    c->rb_t = nullptr;
    c->rb_sp = nullptr;
    c->rb_st = nullptr;
    rc = dmalloc(c, &c->rb_state, 4 * nc);
    if (!rc) rc = dmalloc(c, &c->rb_t, ni);
    if (!rc) rc = dmalloc(c, &c->rb_sp, 3 * ni);
    if (!rc) rc = dmalloc(c, &c->rb_st, 2 * ni);
    if (rc) return rc;
  }
  std::vector<int32_t> flags(ni);
  for (;;) {
    const int cur0 = c->cur, nxt0 = c->nxt;
    rc = retry_copy(c, true);
    if (!rc) rc = chunk();
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(flags.data(), c->d_status, ni * sizeof(int32_t),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // the flagged instances whose margin can still grow
    if (c->h_margin_inst.empty()) c->h_margin_inst.assign(ni, c->halo_margin);
    bool grow = false;
    for (size_t j = 0; j < ni; ++j)
      grow |= (flags[j] & hsgn::kFlagWindow) != 0 && c->h_margin_inst[j] < kMaxMargin;
    if (!grow) return HSGN_OK;
    c->cur = cur0;
    c->nxt = nxt0;
    rc = retry_copy(c, false);
    if (rc) return rc;
    for (size_t j = 0; j < ni; ++j)
      if (flags[j] & hsgn::kFlagWindow)
        c->h_margin_inst[j] = std::min(kMaxMargin, 2.0 * c->h_margin_inst[j]);
    ++c->n_retry;
    roctxMarkA("hsgn halo retry: block runs again, flagged instances at twice their margin");
    rc = make_plan(c);
    if (rc) return rc;
  }
}

}  // namespace

extern "C" {

const char* hsgn_version(void) { return "hsgn-gfx950 0.2"; }

int hsgn_init(hsgn_ctx** out, int32_t n_inst, const int64_t* offsets, const hsgn_params* params,
              const double* d_b, void* hip_stream) {
  if (!out) return HSGN_EINVAL;
  *out = nullptr;
  if (n_inst <= 0 || !offsets || !params) return HSGN_EINVAL;
  hsgn_ctx* c = new (std::nothrow) hsgn_ctx();
  if (!c) return HSGN_ENOMEM;
  c->user_stream = (hipStream_t)hip_stream;
  Layout lay;
  int rc = build_layout(c, n_inst, offsets, params, d_b, lay);
  const std::vector<InstDesc>& inst = lay.inst;
  const std::vector<TileDesc>& tall = lay.tall;
  const std::vector<TileDesc>& tmulti = lay.tmulti;
  const std::vector<TileDesc>& xt = lay.xt;
  const std::vector<int32_t>& multi = lay.multi;
  const int64_t red = c->red_total;
  if (rc == HSGN_OK) {
    if (c->user_stream) {
      c->stream = c->user_stream;
    } else {
      hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
      if (e != hipSuccess) rc = fail(c, HSGN_EHIP, "hipStreamCreate: %s", hipGetErrorString(e));
      c->own_stream = rc == HSGN_OK;
      if (c->own_stream) roctxNameHipStream("hsgn", c->stream);
    }
  }
  if (rc == HSGN_OK) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      rc = fail(c, HSGN_EHIP, "hipDeviceGetAttribute failed");
  }
  if (rc == HSGN_OK) {
    if (hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess)
      rc = fail(c, HSGN_EHIP, "hipEventCreate failed");
  }
  const size_t nc = (size_t)c->ncell;
  if (rc == HSGN_OK) rc = dmalloc(c, &c->d_inst, inst.size());
  if (rc == HSGN_OK) rc = dmalloc(c, &c->d_tiles_all, tall.size());
  if (rc == HSGN_OK) rc = dmalloc(c, &c->d_tiles_multi, tmulti.size());
  if (rc == HSGN_OK) rc = dmalloc(c, &c->d_xtiles, xt.size());
  if (rc == HSGN_OK && c->scheme == HSGN_SCHEME_SGN) rc = dmalloc(c, &c->d_sgn, nc);
  if (rc == HSGN_OK) rc = dmalloc(c, &c->d_multi, multi.size());
  for (int i = 0; i < 3 && rc == HSGN_OK; ++i)
    for (int f = 0; f < 4 && rc == HSGN_OK; ++f) rc = dmalloc(c, &c->buf[i][f], nc);
  if (rc == HSGN_OK && c->any_b) rc = dmalloc(c, &c->d_b, nc);
  if (rc == HSGN_OK) rc = dmalloc(c, &c->d_dt, (size_t)n_inst);
  if (rc == HSGN_OK) rc = dmalloc(c, &c->d_t, (size_t)n_inst);
  if (rc == HSGN_OK) rc = dmalloc(c, &c->d_smax, (size_t)n_inst);
  if (rc == HSGN_OK) rc = dmalloc(c, &c->d_umax, (size_t)n_inst);
  if (rc == HSGN_OK) rc = dmalloc(c, &c->d_hmax, (size_t)n_inst);
  if (rc == HSGN_OK) rc = dmalloc(c, &c->d_status, (size_t)n_inst);
  if (rc == HSGN_OK) rc = dmalloc(c, &c->d_nstep, (size_t)n_inst);
  if (rc == HSGN_OK) rc = dmalloc(c, &c->d_queue, (size_t)18);
  double** rp[] = {&c->d_rlo, &c->d_rdi, &c->d_rup, &c->d_rrhs, &c->d_rx,
                   &c->d_scp, &c->d_sy, &c->d_sv, &c->d_sw};
  for (double** p : rp)
    if (rc == HSGN_OK) rc = dmalloc(c, p, (size_t)red);
  auto up = [&](void* dst, const void* src, size_t bytes) -> int {
    if (!bytes) return HSGN_OK;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return fail(c, HSGN_EHIP, "hipMemcpyAsync: %s", hipGetErrorString(e));
    return HSGN_OK;
  };
  if (rc == HSGN_OK) rc = enter(c);
  if (rc == HSGN_OK) rc = up(c->d_inst, inst.data(), inst.size() * sizeof(InstDesc));
  if (rc == HSGN_OK) rc = up(c->d_tiles_all, tall.data(), tall.size() * sizeof(TileDesc));
  if (rc == HSGN_OK) rc = up(c->d_tiles_multi, tmulti.data(), tmulti.size() * sizeof(TileDesc));
  if (rc == HSGN_OK) rc = up(c->d_xtiles, xt.data(), xt.size() * sizeof(TileDesc));
  if (rc == HSGN_OK) rc = up(c->d_multi, multi.data(), multi.size() * sizeof(int32_t));
  if (rc == HSGN_OK && c->any_b) {
    hipError_t e = hipMemcpyAsync(c->d_b, d_b, nc * sizeof(double), hipMemcpyDeviceToDevice,
                                  c->stream);
    if (e != hipSuccess) rc = fail(c, HSGN_EHIP, "copy of b: %s", hipGetErrorString(e));
    // the library's bed is 0 on flat instances (runs of them cleared at once)
    for (int j = 0; j < n_inst && rc == HSGN_OK;) {
      if (params[j].has_bathymetry) { ++j; continue; }
      int k = j;
      while (k < n_inst && !params[k].has_bathymetry) ++k;
      if (hipMemsetAsync(c->d_b + offsets[j], 0, (size_t)(offsets[k] - offsets[j]) * sizeof(double),
                         c->stream) != hipSuccess)
        rc = fail(c, HSGN_EHIP, "hipMemsetAsync failed");
      j = k;
    }
  }
  if (rc == HSGN_OK) {
    for (int i = 0; i < 3 && rc == HSGN_OK; ++i)
      for (int f = 0; f < 4 && rc == HSGN_OK; ++f)
        if (hipMemsetAsync(c->buf[i][f], 0, nc * sizeof(double), c->stream) != hipSuccess)
          rc = fail(c, HSGN_EHIP, "hipMemsetAsync failed");
  }
  if (rc == HSGN_OK) {
    if (hipMemsetAsync(c->d_t, 0, n_inst * sizeof(double), c->stream) != hipSuccess ||
        hipMemsetAsync(c->d_dt, 0, n_inst * sizeof(double), c->stream) != hipSuccess ||
        hipMemsetAsync(c->d_smax, 0, n_inst * sizeof(unsigned long long), c->stream) != hipSuccess ||
        hipMemsetAsync(c->d_umax, 0, n_inst * sizeof(unsigned long long), c->stream) != hipSuccess ||
        hipMemsetAsync(c->d_status, 0, n_inst * sizeof(int32_t), c->stream) != hipSuccess ||
        hipMemsetAsync(c->d_nstep, 0, n_inst * sizeof(int32_t), c->stream) != hipSuccess ||
        hipMemsetAsync(c->d_queue, 0, 18 * sizeof(int32_t), c->stream) != hipSuccess)
      rc = fail(c, HSGN_EHIP, "hipMemsetAsync failed");
  }
  // host vectors are freed on return: wait for the uploads
  if (rc == HSGN_OK && hipStreamSynchronize(c->stream) != hipSuccess)
    rc = fail(c, HSGN_EHIP, "hipStreamSynchronize failed");
  if (rc == HSGN_OK) rc = make_plan(c);  // no state yet: every instance two-pass
  if (rc == HSGN_OK) rc = leave(c);
  if (rc != HSGN_OK) {
    fprintf(stderr, "hsgn_init: %s\n", c->err.c_str());
    free_all(c);
    delete c;
    return rc;
  }
  *out = c;
  return HSGN_OK;
}

// Clear the status flags, compute the speed bound and depth maximum of the
// current state, and make the solver plan from them (synchronises the stream).
static int reset_and_plan(hsgn_ctx* c) {
  double** U = c->buf[c->cur];
  c->n_retry = 0;
  const int nb = (c->n_inst + 255) / 256;
  hipLaunchKernelGGL(hsgn::k_fill_i32, dim3(nb), dim3(256), 0, c->stream, c->n_inst, c->d_status,
                     0);
  hipLaunchKernelGGL(hsgn::k_fill_i32, dim3(nb), dim3(256), 0, c->stream, c->n_inst, c->d_nstep,
                     0);
  hipLaunchKernelGGL(hsgn::k_fill_u64, dim3(nb), dim3(256), 0, c->stream, c->n_inst, c->d_smax,
                     0ull);
  hipLaunchKernelGGL(hsgn::k_fill_u64, dim3(nb), dim3(256), 0, c->stream, c->n_inst, c->d_umax,
                     0ull);
  hipLaunchKernelGGL(hsgn::k_fill_u64, dim3(nb), dim3(256), 0, c->stream, c->n_inst, c->d_hmax,
                     0ull);
  if (c->scheme == HSGN_SCHEME_EXPLICIT)
    hipLaunchKernelGGL(hsgn::k_speed_ex<256>, dim3(c->ntiles_all), dim3(256), 0, c->stream,
                       c->d_inst, c->d_tiles_all, U[0], U[1], U[2], c->d_smax, c->d_umax,
                       c->d_hmax);
  else
    hipLaunchKernelGGL(hsgn::k_speed<256>, dim3(c->ntiles_all), dim3(256), 0, c->stream,
                       c->d_inst, c->d_tiles_all, U[0], U[1], c->d_smax, c->d_umax, c->d_hmax);
  HIPCHK(c, hipGetLastError());
  // plan the solve from this state's speed bound and depth maximum
  std::vector<unsigned long long> sm(c->n_inst), hm(c->n_inst);
  HIPCHK(c, hipMemcpyAsync(sm.data(), c->d_smax, c->n_inst * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(hm.data(), c->d_hmax, c->n_inst * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->h_smax.resize(c->n_inst);
  c->h_hmax.resize(c->n_inst);
  for (int j = 0; j < c->n_inst; ++j) {
    std::memcpy(&c->h_smax[j], &sm[j], sizeof(double));
    std::memcpy(&c->h_hmax[j], &hm[j], sizeof(double));
  }
  return make_plan(c);
}

int hsgn_set_state(hsgn_ctx* c, const double* d_h, const double* d_q, const double* d_m,
                   const double* d_W, const double* d_t) {
  if (!c) return HSGN_EINVAL;
  if (!d_h || !d_q) return fail(c, HSGN_EINVAL, "hsgn_set_state: h and q are required");
  int rc = enter(c);
  if (rc) return rc;
  const size_t bytes = (size_t)c->ncell * sizeof(double);
  // the buffer rotation restarts: a graph captured after an earlier load
  // replays from the same buffers
  c->cur = 0;
  c->nxt = 2;
  double** U = c->buf[c->cur];
  HIPCHK(c, hipMemcpyAsync(U[0], d_h, bytes, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(U[1], d_q, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (d_m) HIPCHK(c, hipMemcpyAsync(U[2], d_m, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (d_W) HIPCHK(c, hipMemcpyAsync(U[3], d_W, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (!d_m || !d_W)
    hipLaunchKernelGGL(hsgn::k_default_mW<256>, dim3(c->ntiles_all), dim3(256), 0, c->stream,
                       c->d_inst, c->d_tiles_all, U[0], U[1], U[2], U[3], d_m ? 0 : 1,
                       d_W ? 0 : 1);
  if (d_t) {
    HIPCHK(c, hipMemcpyAsync(c->d_t, d_t, c->n_inst * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
  } else {
    HIPCHK(c, hipMemsetAsync(c->d_t, 0, c->n_inst * sizeof(double), c->stream));
  }
  rc = reset_and_plan(c);
  if (rc) return rc;
  return leave(c);
}

int hsgn_get_state(hsgn_ctx* c, double* d_h, double* d_q, double* d_m, double* d_W,
                   double* d_t) {
  if (!c) return HSGN_EINVAL;
  int rc = enter(c);
  if (rc) return rc;
  const size_t bytes = (size_t)c->ncell * sizeof(double);
  double** U = c->buf[c->cur];
  double* dst[4] = {d_h, d_q, d_m, d_W};
  for (int f = 0; f < 4; ++f)
    if (dst[f]) HIPCHK(c, hipMemcpyAsync(dst[f], U[f], bytes, hipMemcpyDeviceToDevice, c->stream));
  if (d_t)
    HIPCHK(c, hipMemcpyAsync(d_t, c->d_t, c->n_inst * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
  return leave(c);
}

int hsgn_get_dt(hsgn_ctx* c, double* d_dt) {
  if (!c || !d_dt) return HSGN_EINVAL;
  int rc = enter(c);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(d_dt, c->d_dt, c->n_inst * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
  return leave(c);
}

int hsgn_set_solver(hsgn_ctx* c, int32_t mode) {
  if (!c) return HSGN_EINVAL;
  if (mode != HSGN_SOLVER_AUTO && mode != HSGN_SOLVER_EXACT && mode != HSGN_SOLVER_AUTO_SMALL)
    return fail(c, HSGN_EINVAL, "hsgn_set_solver: unknown mode %d", mode);
  c->solver = mode == HSGN_SOLVER_EXACT ? HSGN_SOLVER_EXACT : HSGN_SOLVER_AUTO;
  c->win_nt = mode == HSGN_SOLVER_AUTO_SMALL ? 256 : 512;
  c->h_inst_solver.clear();
  int rc = enter(c);
  if (rc) return rc;
  rc = make_plan(c);
  if (rc) return rc;
  return leave(c);
}

int hsgn_plan_info(hsgn_ctx* c, int32_t* h_mode, int32_t* h_halo, int32_t* h_counts) {
  if (!c) return HSGN_EINVAL;
  if (h_mode) std::memcpy(h_mode, c->h_mode.data(), c->n_inst * sizeof(int32_t));
  if (h_halo) std::memcpy(h_halo, c->h_halo.data(), c->n_inst * sizeof(int32_t));
  if (h_counts) {
    h_counts[0] = c->nwin;
    h_counts[1] = c->n_ex_tiles;
    h_counts[2] = c->n_ex_multi;
    h_counts[3] = c->nwin_g[0] > 0 && c->nwin_g[1] > 0 ? -1
                  : (c->nwin_g[1] > 0 ? 512 * kWK
                     : (c->nwin_g[0] > 0 ? 256 * kWK : c->win_nt * kWK));
  }
  return HSGN_OK;
}

int hsgn_step(hsgn_ctx* c, int32_t nsteps) {
  if (!c) return HSGN_EINVAL;
  Range range("hsgn_step");
  if (nsteps < 0) return fail(c, HSGN_EINVAL, "hsgn_step: nsteps < 0");
  int rc = enter(c);
  if (rc) return rc;
  rc = run_retrying(c, [&]() {
    int r = HSGN_OK;
    for (int s = 0; s < nsteps && r == HSGN_OK; ++s) r = enqueue_step(c);
    return r;
  });
  if (rc) return rc;
  return leave(c);
}

int hsgn_run(hsgn_ctx* c, int32_t nsteps, int32_t block) {
  if (!c) return HSGN_EINVAL;
  Range range("hsgn_run");
  if (nsteps < 0 || block < 1) return fail(c, HSGN_EINVAL, "hsgn_run: bad nsteps/block");
  if (block & 1) block += 1;  // the buffer rotation repeats every 2 steps
  int rc = enter(c);
  if (rc) return rc;
  int done = 0;
  for (; done + block <= nsteps && rc == HSGN_OK; done += block)
    rc = run_retrying(c, [&]() {
      Range block_range("hsgn_run graph block");
      hipGraphExec_t exec = nullptr;
      int r = graph_of(c, block, &exec);
      if (r == HSGN_OK) HIPCHK(c, hipGraphLaunch(exec, c->stream));
      return r;
    });
  if (rc) return rc;
  if (done < nsteps)
    rc = run_retrying(c, [&]() {
      int r = HSGN_OK;
      for (int s = done; s < nsteps && r == HSGN_OK; ++s) r = enqueue_step(c);
      return r;
    });
  if (rc) return rc;
  return leave(c);
}

int hsgn_set_adjoint_tape_bytes(hsgn_ctx* c, int64_t bytes) {
  if (!c) return HSGN_EINVAL;
  c->adj.tape_budget = bytes < 0 ? -1 : bytes;
  return HSGN_OK;
}

int hsgn_set_halo_retry(hsgn_ctx* c, int32_t enable) {
  if (!c) return HSGN_EINVAL;
  if (enable != 0 && enable != 1)
    return fail(c, HSGN_EINVAL, "hsgn_set_halo_retry: enable must be 0 or 1");
  c->halo_retry = enable == 1;
  return HSGN_OK;
}

int hsgn_halo_state(hsgn_ctx* c, double* h_margin, int32_t* h_retries) {
  if (!c) return HSGN_EINVAL;
  if (h_margin)
    for (int j = 0; j < c->n_inst; ++j)
      h_margin[j] = c->h_margin_inst.empty() ? c->halo_margin : c->h_margin_inst[j];
  if (h_retries) *h_retries = c->n_retry;
  return HSGN_OK;
}

int hsgn_step_timed(hsgn_ctx* c, int32_t nsteps, double* h_ms, int32_t* h_count) {
  if (!c) return HSGN_EINVAL;
  if (nsteps < 0) return fail(c, HSGN_EINVAL, "hsgn_step_timed: nsteps < 0");
  int rc = enter(c);
  if (rc) return rc;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> tm;
  for (int s = 0; s < nsteps && rc == HSGN_OK; ++s) rc = enqueue_step(c, &tm);
  hipError_t e = hipStreamSynchronize(c->stream);
  double ms[HSGN_NKERNEL] = {0};
  int32_t cnt[HSGN_NKERNEL] = {0};
  for (auto& x : tm) {
    float f = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, x.second.first, x.second.second);
    ms[x.first] += f;
    cnt[x.first] += 1;
    hipEventDestroy(x.second.first);
    hipEventDestroy(x.second.second);
  }
  if (rc) return rc;
  if (e != hipSuccess) return fail(c, HSGN_EHIP, "hsgn_step_timed: %s", hipGetErrorString(e));
  if (h_ms) std::memcpy(h_ms, ms, sizeof ms);
  if (h_count) std::memcpy(h_count, cnt, sizeof cnt);
  return leave(c);
}

}  // extern "C"

namespace {

// Time candidate plans on the loaded state and keep the fastest.  The state
// (and time, status, step counts and speed bounds) is saved before the
// trials and restored after each of them.  set_plan(k) makes plan k; its
// milliseconds per step go to ms[k]; the fastest plan is made again at the
// end and returned in *best.
template <class SetPlan>
int time_plans(hsgn_ctx* c, int32_t nsteps, int nplans, SetPlan set_plan, double* ms, int* best) {
  const size_t nc = (size_t)c->ncell, ni = (size_t)c->n_inst;
  double *s_state = nullptr, *s_t = nullptr;
  unsigned long long* s_sp = nullptr;
  int32_t* s_st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (s_state) hipFree(s_state);
    if (s_t) hipFree(s_t);
    if (s_sp) hipFree(s_sp);
    if (s_st) hipFree(s_st);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
  };
  int rc = dmalloc(c, &s_state, 4 * nc);
  if (!rc) rc = dmalloc(c, &s_t, ni);
  if (!rc) rc = dmalloc(c, &s_sp, 3 * ni);
  if (!rc) rc = dmalloc(c, &s_st, 2 * ni);
  if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = fail(c, HSGN_EHIP, "autotune: hipEventCreate failed");
  if (rc) {
    cleanup();
    return rc;
  }
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream) == hipSuccess;
  };
  const size_t fb = nc * sizeof(double), ib = ni * sizeof(double), ub = ni * sizeof(unsigned long long),
               sb = ni * sizeof(int32_t);
  auto save = [&]() {
    bool ok = true;
    for (int f = 0; f < 4; ++f) ok &= cp(s_state + f * nc, c->buf[c->cur][f], fb);
    ok &= cp(s_t, c->d_t, ib) && cp(s_sp, c->d_smax, ub) && cp(s_sp + ni, c->d_umax, ub) &&
          cp(s_sp + 2 * ni, c->d_hmax, ub) && cp(s_st, c->d_status, sb) &&
          cp(s_st + ni, c->d_nstep, sb);
    return ok;
  };
  auto restore = [&]() {
    bool ok = true;
    for (int f = 0; f < 4; ++f) ok &= cp(c->buf[c->cur][f], s_state + f * nc, fb);
    ok &= cp(c->d_t, s_t, ib) && cp(c->d_smax, s_sp, ub) && cp(c->d_umax, s_sp + ni, ub) &&
          cp(c->d_hmax, s_sp + 2 * ni, ub) && cp(c->d_status, s_st, sb) &&
          cp(c->d_nstep, s_st + ni, sb);
    return ok;
  };
  if (!save()) rc = fail(c, HSGN_EHIP, "autotune: state copy failed");
  for (int k = 0; k < nplans && !rc; ++k) {
    rc = set_plan(k);
    if (!rc) rc = enqueue_step(c);  // first launch of this configuration
    if (!rc && !restore()) rc = fail(c, HSGN_EHIP, "autotune: state copy failed");
    if (!rc && hipEventRecord(e0, c->stream) != hipSuccess) rc = fail(c, HSGN_EHIP, "hipEventRecord");
    for (int st = 0; st < nsteps && !rc; ++st) rc = enqueue_step(c);
    if (!rc && hipEventRecord(e1, c->stream) != hipSuccess) rc = fail(c, HSGN_EHIP, "hipEventRecord");
    float f = 0.0f;
    if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&f, e0, e1) != hipSuccess))
      rc = fail(c, HSGN_EHIP, "autotune: event timing failed");
    ms[k] = (double)f / nsteps;
    if (!rc && !restore()) rc = fail(c, HSGN_EHIP, "autotune: state copy failed");
  }
  int b = 0;
  for (int k = 1; k < nplans; ++k)
    if (ms[k] < ms[b]) b = k;
  if (!rc) rc = set_plan(b);
  if (!rc && hipStreamSynchronize(c->stream) != hipSuccess)
    rc = fail(c, HSGN_EHIP, "autotune: hipStreamSynchronize failed");
  cleanup();
  *best = b;
  return rc;
}

// Read the status flags and step counts (synchronises the stream); on a
// flagged instance set the context's message (naming the instance, the step
// in which the flag was raised and the time reached) and return its code.
int read_status(hsgn_ctx* c, const char* what, int32_t* h_flags) {
  std::vector<int32_t> f(c->n_inst), ns(c->n_inst);
  std::vector<double> t(c->n_inst);
  HIPCHK(c, hipMemcpyAsync(f.data(), c->d_status, c->n_inst * sizeof(int32_t),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(ns.data(), c->d_nstep, c->n_inst * sizeof(int32_t),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(t.data(), c->d_t, c->n_inst * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (h_flags) std::memcpy(h_flags, f.data(), f.size() * sizeof(int32_t));
  int any = 0;
  for (int j = 0; j < c->n_inst; ++j) any |= f[j];
  struct Kind {
    int32_t bit;
    int code;
    const char* text;
  };
  const Kind kinds[3] = {
      {hsgn::kFlagNonPhys, HSGN_ENONPHYS, "h <= 0 or a non-finite value"},
      {hsgn::kFlagWindow, HSGN_EWINDOW,
       "window truncation not negligible (use HSGN_SOLVER_EXACT)"},
      {hsgn::kFlagNonCoercive, HSGN_ENONCOERCIVE, "beta <= 0 (coercivity lost)"}};
  for (const Kind& k : kinds) {
    if (!(any & k.bit)) continue;
    int count = 0, first = -1;
    for (int j = 0; j < c->n_inst; ++j)
      if (f[j] & k.bit) {
        if (first < 0) first = j;
        ++count;
      }
    return fail(c, k.code, "%s: instance %d: %s in step %d after its state was loaded "
                "(t = %.6g); %d instance(s) flagged",
                what, first, k.text, ns[first], t[first], count);
  }
  return HSGN_OK;
}


// Make the uniform plan of a solver mode (every instance in that mode).
int set_uniform_mode(hsgn_ctx* c, int mode) {
  c->solver = mode == HSGN_SOLVER_EXACT ? HSGN_SOLVER_EXACT : HSGN_SOLVER_AUTO;
  c->win_nt = mode == HSGN_SOLVER_AUTO_SMALL ? 256 : 512;
  c->h_inst_solver.clear();
  return make_plan(c);
}

}  // namespace

extern "C" {

// Autotuner: time the three uniform solver modes and keep the fastest.
int hsgn_autotune(hsgn_ctx* c, int32_t nsteps, double* h_ms, int32_t* h_mode) {
  if (!c) return HSGN_EINVAL;
  Range range("hsgn_autotune");
  if (nsteps < 1) return fail(c, HSGN_EINVAL, "hsgn_autotune: nsteps < 1");
  if (c->scheme != HSGN_SCHEME_SEMI_IMPLICIT)
    return fail(c, HSGN_EINVAL, "hsgn_autotune: the tuner times the semi-implicit step only");
  int rc = enter(c);
  if (rc) return rc;
  const int modes[3] = {HSGN_SOLVER_AUTO, HSGN_SOLVER_EXACT, HSGN_SOLVER_AUTO_SMALL};
  double t[3] = {0, 0, 0};
  int best = 0;
  rc = time_plans(c, nsteps, 3, [&](int k) { return set_uniform_mode(c, modes[k]); }, t, &best);
  if (rc) return rc;
  double ms[3] = {0, 0, 0};
  for (int k = 0; k < 3; ++k) ms[modes[k]] = t[k];
  if (h_ms) std::memcpy(h_ms, ms, sizeof ms);
  if (h_mode) *h_mode = modes[best];
  return leave(c);
}

int hsgn_status(hsgn_ctx* c, int32_t* h_flags) {
  if (!c) return HSGN_EINVAL;
  return read_status(c, "hsgn_status", h_flags);
}

int hsgn_set_instance_solvers(hsgn_ctx* c, const int32_t* h_modes) {
  if (!c) return HSGN_EINVAL;
  if (!h_modes) return fail(c, HSGN_EINVAL, "hsgn_set_instance_solvers: h_modes is NULL");
  if (c->scheme != HSGN_SCHEME_SEMI_IMPLICIT)
    return fail(c, HSGN_EINVAL, "hsgn_set_instance_solvers: per-instance modes are for the semi-implicit "
                "step only");
  for (int j = 0; j < c->n_inst; ++j)
    if (h_modes[j] != HSGN_SOLVER_AUTO && h_modes[j] != HSGN_SOLVER_EXACT &&
        h_modes[j] != HSGN_SOLVER_AUTO_SMALL)
      return fail(c, HSGN_EINVAL, "hsgn_set_instance_solvers: instance %d: unknown mode %d", j,
                  h_modes[j]);
  c->h_inst_solver.assign(h_modes, h_modes + c->n_inst);
  int rc = enter(c);
  if (rc) return rc;
  rc = make_plan(c);
  if (rc) return rc;
  return leave(c);
}

int hsgn_set_halo_margin(hsgn_ctx* c, double margin) {
  if (!c) return HSGN_EINVAL;
  if (!(margin > 0.0 && margin <= kMaxMargin))
    return fail(c, HSGN_EINVAL, "hsgn_set_halo_margin: margin %g outside (0, 64]", margin);
  c->halo_margin = margin;
  c->h_margin_inst.clear();  // the retry's per-instance margins start over
  int rc = enter(c);
  if (rc) return rc;
  rc = make_plan(c);
  if (rc) return rc;
  return leave(c);
}

int hsgn_set_launch(hsgn_ctx* c, int32_t launch) {
  if (!c) return HSGN_EINVAL;
  if (launch != HSGN_LAUNCH_GRID && launch != HSGN_LAUNCH_PERSISTENT)
    return fail(c, HSGN_EINVAL, "hsgn_set_launch: unknown launch %d", launch);
  if (launch == HSGN_LAUNCH_PERSISTENT && !c->d_queue)
    return fail(c, HSGN_EINVAL, "hsgn_set_launch: this context has no work queues");
  if (launch != c->launch) {  // cached graphs hold the other kernels
    for (auto& g : c->graphs) hipGraphExecDestroy(g.exec);
    c->graphs.clear();
    c->launch = launch;
  }
  return HSGN_OK;
}

// Time the two window-stage launches on the current plan and keep the faster.
int hsgn_autotune_launch(hsgn_ctx* c, int32_t nsteps, double* h_ms, int32_t* h_launch) {
  if (!c) return HSGN_EINVAL;
  Range range("hsgn_autotune_launch");
  if (nsteps < 1) return fail(c, HSGN_EINVAL, "hsgn_autotune_launch: nsteps < 1");
  if (c->scheme != HSGN_SCHEME_SEMI_IMPLICIT)
    return fail(c, HSGN_EINVAL, "hsgn_autotune_launch: the window launch of the semi-implicit step only");
  if (!c->d_queue)
    return fail(c, HSGN_EINVAL, "hsgn_autotune_launch: this context has no work queues");
  int rc = enter(c);
  if (rc) return rc;
  double ms[2] = {0, 0};
  int best = 0;
  rc = time_plans(c, nsteps, 2, [&](int k) { return hsgn_set_launch(c, k); }, ms, &best);
  if (rc) return rc;
  if (h_ms) std::memcpy(h_ms, ms, sizeof ms);
  if (h_launch) *h_launch = best;
  return leave(c);
}

const char* hsgn_last_error(const hsgn_ctx* c) { return c ? c->err.c_str() : "null context"; }

void hsgn_destroy(hsgn_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);  // nothing to report to: the context goes away
  free_all(c);
  delete c;
}

}  // extern "C"

namespace {

// Adjoint helper kernels (one thread per cell or per instance).
__global__ void k_state_from_surface(int64_t ncell, const double* __restrict__ zeta,
                                     const double* __restrict__ b, double* __restrict__ h,
                                     double* __restrict__ q, double* __restrict__ m,
                                     double* __restrict__ W) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncell) return;
  const double hh = zeta[i] - (b ? b[i] : 0.0);
  h[i] = hh;
  q[i] = 0.0;
  m[i] = hh * hh;
  W[i] = 0.0;
}

__global__ void k_fill_f64(int64_t n, double* __restrict__ p, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// loss after step s: (1/2) sum_g (h(gauge) - target)^2, residuals kept
__global__ void k_gauge_fwd(int n_inst, const InstDesc* __restrict__ inst, int ng,
                            const int32_t* __restrict__ gauge, const double* __restrict__ target,
                            int nsteps, int s, const double* __restrict__ h,
                            double* __restrict__ loss, double* __restrict__ res) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_inst) return;
  const int64_t off = inst[j].off;
  double acc = loss[j];
  for (int g = 0; g < ng; ++g) {
    const int64_t k = ((int64_t)j * nsteps + s) * ng + g;
    const double r = h[off + gauge[(int64_t)j * ng + g]] - target[k];
    res[k] = r;
    acc += 0.5 * r * r;
  }
  loss[j] = acc;
}

__global__ void k_gauge_adj(int n_inst, const InstDesc* __restrict__ inst, int ng,
                            const int32_t* __restrict__ gauge, int nsteps, int s,
                            const double* __restrict__ res, double* __restrict__ ah) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_inst) return;
  const int64_t off = inst[j].off;
  for (int g = 0; g < ng; ++g)
    ah[off + gauge[(int64_t)j * ng + g]] += res[((int64_t)j * nsteps + s) * ng + g];
}

// gradient of the initial-state map h = zeta - b, q = 0, m = h^2, W = 0
// (one workgroup per instance; flat instances have no bed gradient)
__global__ void k_adj_surface(const InstDesc* __restrict__ inst, const double* __restrict__ zeta,
                              const double* __restrict__ b, const double* __restrict__ ah,
                              const double* __restrict__ am, const double* __restrict__ gb_dyn,
                              double* __restrict__ gz, double* __restrict__ gb) {
  const InstDesc I = inst[blockIdx.x];
  const bool bed = b && I.has_b;
  for (int k = threadIdx.x; k < I.n; k += blockDim.x) {
    const int64_t i = I.off + k;
    const double hh = zeta[i] - (b ? b[i] : 0.0);
    const double dz = ah[i] + 2.0 * hh * am[i];
    if (gz) gz[i] = dz;
    if (gb) gb[i] = bed ? gb_dyn[i] - dz : 0.0;
  }
}

int adj_alloc(hsgn_ctx* c, int K, int nseg, int64_t nres, bool grad, int ntb) {
  auto& a = c->adj;
  const size_t nc = (size_t)c->ncell;
  if (nres > a.nres) {
    if (a.res) hipFree(a.res);
    a.res = nullptr;
    a.nres = 0;
    int rc = dmalloc(c, &a.res, (size_t)nres);
    if (rc) return rc;
    a.nres = nres;
  }
  if (!grad) return HSGN_OK;
  if (!a.sys) {
    int rc = dmalloc(c, &a.sys, 9 * nc);
    if (!rc) rc = dmalloc(c, &a.st, 13 * nc);
    if (rc) return rc;
    // tiles of the reverse stage: cores of at most kAdjNT - 2H cells
    std::vector<hsgn::adj::TileA> tl;
    const int C = kAdjNT - 2 * hsgn::adj::H;
    for (int j = 0; j < c->n_inst; ++j) {
      const int n = (int)(c->offsets[j + 1] - c->offsets[j]);
      const int nt = (n + C - 1) / C;
      for (int k = 0; k < nt; ++k) {
        hsgn::adj::TileA t;
        t.inst = j;
        t.ts = (int)((int64_t)k * n / nt);
        t.te = (int)((int64_t)(k + 1) * n / nt);
        t.pad = 0;
        tl.push_back(t);
      }
    }
    rc = dmalloc(c, &a.tiles, tl.size());
    if (rc) return rc;
    HIPCHK(c, hipMemcpy(a.tiles, tl.data(), tl.size() * sizeof(hsgn::adj::TileA),
                        hipMemcpyHostToDevice));
    a.ntiles = (int)tl.size();
  }
  if ((size_t)ntb * K > a.tape_steps) {
    if (a.tape) hipFree(a.tape);
    a.tape = nullptr;
    a.tape_steps = 0;
    int rc = dmalloc(c, &a.tape, (size_t)ntb * K * 8 * nc);
    if (rc) return rc;
    a.tape_steps = (size_t)ntb * K;
  }
  if (!a.rstream) {
    HIPCHK(c, hipStreamCreateWithFlags(&a.rstream, hipStreamNonBlocking));
    roctxNameHipStream("hsgn adjoint recompute", a.rstream);
    HIPCHK(c, hipEventCreateWithFlags(&a.ev_fwd, hipEventDisableTiming));
    for (int i = 0; i < 2; ++i) {
      HIPCHK(c, hipEventCreateWithFlags(&a.ev_rec[i], hipEventDisableTiming));
      HIPCHK(c, hipEventCreateWithFlags(&a.ev_rev[i], hipEventDisableTiming));
    }
  }
  if (nseg > a.nseg) {
    if (a.ckpt) hipFree(a.ckpt);
    a.ckpt = nullptr;
    a.nseg = 0;
    int rc = dmalloc(c, &a.ckpt, (size_t)(nseg + 1) * 4 * nc);
    if (rc) return rc;
    a.nseg = nseg;
  }
  return HSGN_OK;
}

int copy_state(hsgn_ctx* c, double* const* dst, double* const* src) {
  const size_t bytes = (size_t)c->ncell * sizeof(double);
  for (int f = 0; f < 4; ++f)
    HIPCHK(c, hipMemcpyAsync(dst[f], src[f], bytes, hipMemcpyDeviceToDevice, c->stream));
  return HSGN_OK;
}

}  // namespace

extern "C" int hsgn_adjoint(hsgn_ctx* c, int32_t nsteps, int32_t K, int32_t ng,
                            const int32_t* d_gauge, const double* d_target,
                            const double* d_zeta0, double* d_loss, double* d_grad_zeta0,
                            double* d_grad_b) {
  if (!c) return HSGN_EINVAL;
  Range range("hsgn_adjoint");
  if (nsteps < 1 || K < 1 || ng < 1 || !d_gauge || !d_target || !d_zeta0 || !d_loss)
    return fail(c, HSGN_EINVAL, "hsgn_adjoint: bad arguments");
  if (c->order != 2 || c->scheme != HSGN_SCHEME_SEMI_IMPLICIT)
    return fail(c, HSGN_EINVAL, "hsgn_adjoint: the adjoint is of the two-stage semi-implicit "
                "step (order 2, scheme 0)");
  for (int j = 0; j < c->n_inst; ++j) {
    if (!(c->params[j].dt_fixed > 0) || c->params[j].t_end > 0)
      return fail(c, HSGN_EINVAL,
                  "hsgn_adjoint: instance %d needs dt_fixed > 0 and no t_end (the step map "
                  "must not depend on the state through dt)", j);
  }
  {  // gauge cells must lie inside their instance
    std::vector<int32_t> hg((size_t)c->n_inst * ng);
    HIPCHK(c, hipMemcpy(hg.data(), d_gauge, hg.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int j = 0; j < c->n_inst; ++j) {
      const int64_t n = c->offsets[j + 1] - c->offsets[j];
      for (int g = 0; g < ng; ++g) {
        const int32_t v = hg[(size_t)j * ng + g];
        if (v < 0 || v >= n)
          return fail(c, HSGN_EINVAL, "hsgn_adjoint: gauge %d of instance %d is cell %d (n = %lld)",
                      g, j, (int)v, (long long)n);
      }
    }
  }
  if (K > nsteps) K = nsteps;
  const int nseg = (nsteps + K - 1) / K;
  const int64_t nres = (int64_t)c->n_inst * nsteps * ng;
  const bool grad = d_grad_zeta0 || d_grad_b;
  // Tape every segment in the forward pass (no recompute) when the tapes of
  // all of them fit the budget; else two tape buffers, the last two
  // segments taped and every earlier one recomputed from its checkpoint.
  bool full_tape = false;
  if (grad && nseg > 2) {
    const double need = (double)nseg * K * 8 * (double)c->ncell * sizeof(double);
    double budget = (double)c->adj.tape_budget;
    if (c->adj.tape_budget < 0) {  // half the free device memory (counting a tape held already)
      size_t fr = 0, tot = 0;
      HIPCHK(c, hipMemGetInfo(&fr, &tot));
      budget = 0.5 * ((double)fr + (double)c->adj.tape_steps * 8 * (double)c->ncell * sizeof(double));
    }
    full_tape = need <= budget;
  }
  int rc = adj_alloc(c, K, nseg, nres, grad, full_tape ? nseg : 2);
  if (rc == HSGN_ENOMEM && full_tape) {  // the full tape did not fit after all
    full_tape = false;
    (void)hipGetLastError();
    c->err.clear();
    rc = adj_alloc(c, K, nseg, nres, grad, 2);
  }
  if (rc) return rc;
  const int ntb = full_tape ? nseg : 2;
  rc = enter(c);
  if (rc) return rc;
  auto& a = c->adj;
  const size_t nc = (size_t)c->ncell;
  const unsigned nbc = (unsigned)((c->ncell + 255) / 256);
  const unsigned nbi = (unsigned)((c->n_inst + 255) / 256);
  double** U = nullptr;
  auto ckpt = [&](int k, int f) { return a.ckpt + ((size_t)k * 4 + f) * nc; };
  // tape buffers of K steps: segment s uses buffer s % ntb
  auto tape = [&](int s, int k, int f) {
    return a.tape + (((size_t)(s % ntb) * K + k) * 8 + f) * nc;
  };
  double* AS[4];
  double* A1[4];
  double* ANP[4];
  for (int f = 0; f < 4; ++f) {
    AS[f] = a.st + (size_t)f * nc;
    A1[f] = a.st + (size_t)(4 + f) * nc;
    ANP[f] = a.st + (size_t)(8 + f) * nc;
  }
  double* GB = a.st + (size_t)12 * nc;

  // ---- forward: initial state from the surface, checkpoints, loss
  roctxMarkA(!grad       ? "hsgn_adjoint forward pass (loss only)"
             : full_tape ? "hsgn_adjoint forward pass (every segment taped)"
                         : "hsgn_adjoint forward pass (the last two segments taped)");
  U = c->buf[c->cur];
  hipLaunchKernelGGL(k_state_from_surface, dim3(nbc), dim3(256), 0, c->stream, c->ncell, d_zeta0,
                     c->d_b, U[0], U[1], U[2], U[3]);
  HIPCHK(c, hipMemsetAsync(c->d_t, 0, c->n_inst * sizeof(double), c->stream));
  rc = reset_and_plan(c);  // flags, speed bound and solver plan of the initial state
  if (rc) return rc;
  hipLaunchKernelGGL(k_fill_f64, dim3(nbi), dim3(256), 0, c->stream, (int64_t)c->n_inst, d_loss, 0.0);
  // The last two segments (one per tape buffer), or every segment with the
  // full tape, write their tapes, their checkpoints and the final state
  // directly, so none of them is recomputed: the reverse sweep of the last
  // one starts at once, and the recompute stream first recomputes the third
  // segment from the end.
  const int n_fwd_tape = full_tape ? nseg : std::min(nseg, 2);
  const int s_tape = (nseg - n_fwd_tape) * K;
  for (int s = 0; s < nsteps; ++s) {
    if (grad && s % K == 0 && s <= s_tape) {  // later checkpoints are written by the steps
      double* dst[4] = {ckpt(s / K, 0), ckpt(s / K, 1), ckpt(s / K, 2), ckpt(s / K, 3)};
      rc = copy_state(c, dst, c->buf[c->cur]);
      if (rc) return rc;
    }
    const double* hnew;
    if (grad && s >= s_tape) {
      const int seg = s / K, k = s - seg * K, ks = std::min(K, nsteps - seg * K);
      double *un[4], *u1[4], *out[4];
      for (int f = 0; f < 4; ++f) {
        un[f] = k == 0 ? ckpt(seg, f) : tape(seg, k, f);
        u1[f] = tape(seg, k, 4 + f);
        out[f] = (k + 1 < ks) ? tape(seg, k + 1, f) : ckpt(seg + 1, f);
      }
      rc = enqueue_step_io(c, un, u1, out);
      hnew = out[0];
    } else {
      rc = enqueue_step(c);
      hnew = c->buf[c->cur][0];
    }
    if (rc) return rc;
    hipLaunchKernelGGL(k_gauge_fwd, dim3(nbi), dim3(256), 0, c->stream, c->n_inst, c->d_inst, ng,
                       d_gauge, d_target, nsteps, s, hnew, d_loss, a.res);
  }
  // A flagged instance is frozen (dt = 0) from the step of its flag on; its
  // loss and gradients would belong to another map, and the segment
  // recompute would reuse that dt = 0: report it instead.
  rc = read_status(c, "hsgn_adjoint", nullptr);
  if (rc) return rc;
  if (!grad) {  // loss only
    hipLaunchKernelGGL(k_fill_f64, dim3(nbi), dim3(256), 0, c->stream, (int64_t)c->n_inst,
                       c->d_t, 0.0);
    HIPCHK(c, hipGetLastError());
    return leave(c);
  }
  // (the final state is in checkpoint nseg; it is restored at the end)
  // ---- reverse
  roctxMarkA("hsgn_adjoint reverse sweep");
  for (int f = 0; f < 4; ++f)
    hipLaunchKernelGGL(k_fill_f64, dim3(nbc), dim3(256), 0, c->stream, (int64_t)c->ncell, AS[f], 0.0);
  hipLaunchKernelGGL(k_fill_f64, dim3(nbc), dim3(256), 0, c->stream, (int64_t)c->ncell, GB, 0.0);
  hsgn::AdjTileArgs P;
  std::memset(&P, 0, sizeof P);
  P.inst = c->d_inst;
  P.tiles = a.tiles;
  P.dt = c->d_dt;
  P.b = c->d_b;
  P.gb = GB;
  auto sysa = [&](int k) { return a.sys + (size_t)k * nc; };
  P.lot = sysa(0);
  P.dit = sysa(1);
  P.upt = sysa(2);
  P.hba = sysa(3);
  P.lam = sysa(4);
  hsgn::AdjSolveArgs Q;
  Q.inst = c->d_inst;
  Q.dt = c->d_dt;
  Q.lot = sysa(0);
  Q.dit = sysa(1);
  Q.upt = sysa(2);
  Q.hba = sysa(3);
  Q.lam = sysa(4);
  Q.scp = sysa(5);
  Q.sy = sysa(6);
  Q.sv = sysa(7);
  Q.sw = sysa(8);
  const dim3 gt(a.ntiles), bt(kAdjNT);
  // Recompute of a segment from its checkpoint on the recompute stream,
  // keeping U^n and U^(1) of every step on the segment's tape (the steps
  // write there directly; dt is fixed, so the steps reuse it).  The last
  // step needs only U^(1): its U^{n+1} is the next checkpoint.
  auto recompute = [&](int seg) -> int {
    const int s0 = seg * K, ks = std::min(K, nsteps - s0);
    hipStream_t main_stream = c->stream;
    c->stream = a.rstream;
    c->io_skip_dt = true;
    int r = HSGN_OK;
    for (int k = 0; k < ks && r == HSGN_OK; ++k) {
      double *un[4], *u1[4], *nx[4];
      for (int f = 0; f < 4; ++f) {
        un[f] = k == 0 ? ckpt(seg, f) : tape(seg, k, f);
        u1[f] = tape(seg, k, 4 + f);
        nx[f] = k + 1 < ks ? tape(seg, k + 1, f) : nullptr;
      }
      r = enqueue_step_io(c, un, u1, k + 1 < ks ? nx : nullptr);
    }
    c->io_skip_dt = false;
    c->stream = main_stream;
    return r;
  };
  // the recompute stream starts once the forward pass (checkpoints, dt) is done
  HIPCHK(c, hipEventRecord(a.ev_fwd, c->stream));
  HIPCHK(c, hipStreamWaitEvent(a.rstream, a.ev_fwd, 0));
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int s0 = seg * K;
    const int ks = std::min(K, nsteps - s0);
    // the previous segment is recomputed (unless the forward pass wrote its
    // tape) while this one is swept in reverse; its tape buffer was last
    // read by the reverse sweep of segment seg + 1
    if (seg >= 1 && seg - 1 < nseg - n_fwd_tape) {
      if (seg + 1 <= nseg - 1) HIPCHK(c, hipStreamWaitEvent(a.rstream, a.ev_rev[(seg + 1) % 2], 0));
      rc = recompute(seg - 1);
      if (rc) return rc;
      HIPCHK(c, hipEventRecord(a.ev_rec[(seg - 1) % 2], a.rstream));
    }
    if (seg < nseg - n_fwd_tape) HIPCHK(c, hipStreamWaitEvent(c->stream, a.ev_rec[seg % 2], 0));
    double* cks[4] = {ckpt(seg, 0), ckpt(seg, 1), ckpt(seg, 2), ckpt(seg, 3)};
    auto un_of = [&](int k, int f) { return k == 0 ? cks[f] : tape(seg, k, f); };
    for (int k = ks - 1; k >= 0; --k) {
      hipLaunchKernelGGL(k_gauge_adj, dim3(nbi), dim3(256), 0, c->stream, c->n_inst, c->d_inst,
                         ng, d_gauge, nsteps, s0 + k, a.res, AS[0]);
      for (int f = 0; f < 4; ++f) {
        P.un[f] = un_of(k, f);
        P.u1[f] = tape(seg, k, 4 + f);
      }
      // stage 2: hbar is the depth of U^{n+1}
      P.hbar = (k + 1 < ks) ? tape(seg, k + 1, 0) : ckpt(seg + 1, 0);
      for (int f = 0; f < 4; ++f) {
        P.abar[f] = AS[f];
        P.out1[f] = A1[f];
        P.outn[f] = ANP[f];
      }
      hipLaunchKernelGGL((hsgn::k_adj_r1<kAdjNT, 2>), gt, bt, 0, c->stream, P);
      hipLaunchKernelGGL((hsgn::k_adj_r2<512, 8>), dim3(c->n_inst), dim3(512), 0, c->stream, Q);
      hipLaunchKernelGGL((hsgn::k_adj_r3<kAdjNT, 2>), gt, bt, 0, c->stream, P);
      // stage 1: hbar is the depth of U^(1)
      P.hbar = tape(seg, k, 4);
      for (int f = 0; f < 4; ++f) P.abar[f] = A1[f];
      hipLaunchKernelGGL((hsgn::k_adj_r1<kAdjNT, 1>), gt, bt, 0, c->stream, P);
      hipLaunchKernelGGL((hsgn::k_adj_r2<512, 8>), dim3(c->n_inst), dim3(512), 0, c->stream, Q);
      hipLaunchKernelGGL((hsgn::k_adj_r3<kAdjNT, 1>), gt, bt, 0, c->stream, P);
      for (int f = 0; f < 4; ++f) std::swap(AS[f], ANP[f]);
    }
    HIPCHK(c, hipEventRecord(a.ev_rev[seg % 2], c->stream));
  }
  // ---- gradients of the initial-state map; restore the final state
  hipLaunchKernelGGL(k_adj_surface, dim3(c->n_inst), dim3(256), 0, c->stream, c->d_inst, d_zeta0,
                     c->d_b, AS[0], AS[2], GB, d_grad_zeta0, d_grad_b);
  {
    double* src[4] = {ckpt(nseg, 0), ckpt(nseg, 1), ckpt(nseg, 2), ckpt(nseg, 3)};
    rc = copy_state(c, c->buf[c->cur], src);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_fill_f64, dim3(nbi), dim3(256), 0, c->stream, (int64_t)c->n_inst, c->d_t,
                     0.0);
  HIPCHK(c, hipGetLastError());
  return leave(c);
}

// ---------------------------------------------------------------------------
// hsgn_autotune_classes: the solver mode chosen per class of instances.
// ---------------------------------------------------------------------------
namespace {

// Copy runs of cells: entry k of tab is (source offset, destination offset,
// length); one workgroup per entry.
__global__ void k_gather_runs(const int64_t* __restrict__ tab, const double* __restrict__ src,
                              double* __restrict__ dst) {
  const int64_t so = tab[3 * blockIdx.x], dof = tab[3 * blockIdx.x + 1],
                len = tab[3 * blockIdx.x + 2];
  for (int64_t i = threadIdx.x; i < len; i += blockDim.x) dst[dof + i] = src[so + i];
}

// Class key of instance j: bit length of n - 1 (the N bucket), boundary
// type, bed flag, and the bit length of the halo estimate of the windowed
// solve (0 before a state is loaded).
void class_key(const hsgn_ctx* c, int j, int32_t key[4]) {
  const int64_t n = c->offsets[j + 1] - c->offsets[j];
  int nb = 0;
  while (((int64_t)1 << nb) < n) ++nb;
  int hb = 0;
  const int L = c->h_halo.empty() ? 0 : c->h_halo[j];
  while (L > 0 && (1 << hb) < L && hb < 30) ++hb;
  key[0] = nb;
  key[1] = c->params[j].bc;
  key[2] = c->params[j].has_bathymetry ? 1 : 0;
  key[3] = hb;
}

// Time every solver mode on the instances of one class in a context of
// their own (a copy of their state, time, bed and parameters).
int tune_class(hsgn_ctx* c, const std::vector<int>& idx, int32_t nsteps, double ms[3],
               int32_t* kept) {
  const int m = (int)idx.size();
  std::vector<int64_t> off(m + 1, 0);
  std::vector<hsgn_params> prm(m);
  std::vector<int64_t> tab, tabt;
  for (int k = 0; k < m; ++k) {
    const int j = idx[k];
    const int64_t n = c->offsets[j + 1] - c->offsets[j];
    off[k + 1] = off[k] + n;
    prm[k] = c->params[j];
    tab.insert(tab.end(), {c->offsets[j], off[k], n});
    tabt.insert(tabt.end(), {(int64_t)j, (int64_t)k, (int64_t)1});
  }
  const int64_t nc = off[m];
  bool any_b = false;
  for (const hsgn_params& p : prm) any_b |= p.has_bathymetry != 0;
  double* tmp = nullptr;
  int64_t* dtab = nullptr;
  int rc = dmalloc(c, &tmp, (size_t)(5 * nc + m));
  if (!rc) rc = dmalloc(c, &dtab, tab.size() + tabt.size());
  hsgn_ctx* sub = nullptr;
  if (!rc) {
    HIPCHK(c, hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(int64_t),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dtab + tab.size(), tabt.data(), tabt.size() * sizeof(int64_t),
                             hipMemcpyHostToDevice, c->stream));
    for (int f = 0; f < 4; ++f)
      hipLaunchKernelGGL(k_gather_runs, dim3(m), dim3(256), 0, c->stream, dtab,
                         c->buf[c->cur][f], tmp + (size_t)f * nc);
    if (any_b)
      hipLaunchKernelGGL(k_gather_runs, dim3(m), dim3(256), 0, c->stream, dtab, c->d_b,
                         tmp + (size_t)4 * nc);
    hipLaunchKernelGGL(k_gather_runs, dim3(m), dim3(64), 0, c->stream, dtab + tab.size(), c->d_t,
                       tmp + (size_t)5 * nc);
    HIPCHK(c, hipGetLastError());
    rc = hsgn_init(&sub, m, off.data(), prm.data(), any_b ? tmp + (size_t)4 * nc : nullptr,
                   (void*)c->stream);
    if (rc) rc = fail(c, rc, "hsgn_autotune_classes: sub-context init failed");
  }
  if (!rc) {
    sub->halo_margin = c->halo_margin;
    rc = hsgn_set_state(sub, tmp, tmp + nc, tmp + 2 * (size_t)nc, tmp + 3 * (size_t)nc,
                        tmp + 5 * (size_t)nc);
    if (!rc) rc = hsgn_autotune(sub, nsteps, ms, kept);
    if (rc) rc = fail(c, rc, "hsgn_autotune_classes: %s", hsgn_last_error(sub));
  }
  if (sub) hsgn_destroy(sub);
  // the sub-context's work is on this stream: wait before freeing its inputs
  if (hipStreamSynchronize(c->stream) != hipSuccess && !rc)
    rc = fail(c, HSGN_EHIP, "hsgn_autotune_classes: hipStreamSynchronize failed");
  if (tmp) hipFree(tmp);
  if (dtab) hipFree(dtab);
  return rc;
}

}  // namespace

extern "C" int hsgn_autotune_classes(hsgn_ctx* c, int32_t nsteps, int32_t max_classes,
                                     int32_t* h_nclass, int32_t* h_class_of, int32_t* h_keys,
                                     double* h_ms, int32_t* h_kept, double* h_whole) {
  if (!c) return HSGN_EINVAL;
  Range range("hsgn_autotune_classes");
  if (nsteps < 1 || max_classes < 1 || !h_nclass)
    return fail(c, HSGN_EINVAL, "hsgn_autotune_classes: bad arguments");
  if (c->scheme != HSGN_SCHEME_SEMI_IMPLICIT)
    return fail(c, HSGN_EINVAL, "hsgn_autotune_classes: the tuner times the semi-implicit step only");
  int rc = enter(c);
  if (rc) return rc;
  // classes in order of first appearance
  std::vector<std::array<int32_t, 4>> keys;
  std::vector<std::vector<int>> members;
  std::vector<int32_t> cls(c->n_inst);
  for (int j = 0; j < c->n_inst; ++j) {
    std::array<int32_t, 4> k;
    class_key(c, j, k.data());
    int id = -1;
    for (size_t q = 0; q < keys.size(); ++q)
      if (keys[q] == k) id = (int)q;
    if (id < 0) {
      id = (int)keys.size();
      keys.push_back(k);
      members.emplace_back();
    }
    members[id].push_back(j);
    cls[j] = id;
  }
  const int ncls = (int)keys.size();
  if (ncls > max_classes)
    return fail(c, HSGN_EINVAL, "hsgn_autotune_classes: %d classes, room for %d", ncls,
                max_classes);
  std::vector<double> ms(3 * ncls, 0.0);
  std::vector<int32_t> kept(ncls, HSGN_SOLVER_AUTO);
  for (int q = 0; q < ncls && !rc; ++q) rc = tune_class(c, members[q], nsteps, &ms[3 * q], &kept[q]);
  if (rc) return rc;
  // the per-class plan (which may need a launch per window geometry) against
  // the three uniform modes on the whole batch: the fastest is kept
  std::vector<int32_t> modes(c->n_inst);
  for (int j = 0; j < c->n_inst; ++j) modes[j] = kept[cls[j]];
  const int umodes[3] = {HSGN_SOLVER_AUTO, HSGN_SOLVER_EXACT, HSGN_SOLVER_AUTO_SMALL};
  double whole[4] = {0, 0, 0, 0};
  int best = 0;
  rc = time_plans(c, nsteps, 4,
                  [&](int k) {
                    if (k < 3) return set_uniform_mode(c, umodes[k]);
                    c->h_inst_solver = modes;
                    return make_plan(c);
                  },
                  whole, &best);
  if (rc) return rc;
  *h_nclass = ncls;
  if (h_whole) {
    for (int k = 0; k < 3; ++k) h_whole[umodes[k]] = whole[k];
    h_whole[3] = whole[3];
    h_whole[4] = best == 3 ? -1.0 : (double)umodes[best];
  }
  if (h_class_of) std::memcpy(h_class_of, cls.data(), cls.size() * sizeof(int32_t));
  if (h_keys)
    for (int q = 0; q < ncls; ++q) std::memcpy(h_keys + 4 * q, keys[q].data(), 4 * sizeof(int32_t));
  if (h_ms) std::memcpy(h_ms, ms.data(), ms.size() * sizeof(double));
  if (h_kept) std::memcpy(h_kept, kept.data(), kept.size() * sizeof(int32_t));
  return leave(c);
}

// ---------------------------------------------------------------------------
// hsgn_step_noalloc: the steps of hsgn_step on the caller's arrays with every
// device buffer the library needs carved from one static array (one copy
// per GPU, kept until the process ends), so that the call allocates nothing.
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kNaCells = HSGN_NOALLOC_MAX_CELLS;
constexpr int64_t kNaInst = HSGN_NOALLOC_MAX_INST;
// two-pass tiles of at most kTileMax cells: at most one partial tile per instance
constexpr int64_t kNaTiles = kNaInst + kNaCells / kTileMax;
// windows per instance: at most 3 plus one per core of at least half a
// 2048-row window minus 8 rows (the halo is at most a quarter window)
constexpr int64_t kNaWins = 3 * kNaInst + kNaCells / 1016 + 1;
constexpr size_t na_round(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kNaBytes =
    na_round(8 * kNaCells * sizeof(double)) +                   // U^(1), U^{n+1}
    na_round(kNaInst * sizeof(InstDesc)) +                      // instance descriptors
    4 * na_round(kNaTiles * sizeof(TileDesc)) +                 // tilings and plan lists
    2 * na_round(kNaInst * sizeof(int32_t)) +                   // multi-tile instance lists
    na_round(kNaWins * sizeof(WinDesc)) +                       // window descriptors
    5 * na_round(kNaInst * sizeof(double)) +                    // dt, t, speed and depth maxima
    2 * na_round(kNaInst * sizeof(int32_t)) +                   // status, step counts
    9 * na_round(2 * kNaTiles * sizeof(double));                // reduced rows and solver scratch

}  // namespace

// The static workspace.  Host code never uses this name as an address: the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

std::mutex na_mutex;
constexpr int kNaMaxDevices = 64;
unsigned char* na_ptr[kNaMaxDevices] = {};

// Device address of this device's copy of the static workspace.
int na_scratch(hsgn_ctx* c, unsigned char** out) {
  int dev = -1;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= kNaMaxDevices)
    return fail(c, HSGN_EINVAL, "device %d beyond the %d this entry point supports", dev,
                kNaMaxDevices);
  std::lock_guard<std::mutex> lock(na_mutex);
  if (!na_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(c, HSGN_EHIP, "hipGetSymbolAddress returned a null address");
    na_ptr[dev] = (unsigned char*)p;
  }
  *out = na_ptr[dev];
  return HSGN_OK;
}

int na_run(hsgn_ctx* c, int32_t n_inst, const int64_t* offsets, const hsgn_params* params,
           const double* d_b, double* const* U, double* d_t, int32_t nsteps, int32_t solver,
           int32_t* h_flags) {
  Layout lay;
  int rc = build_layout(c, n_inst, offsets, params, d_b, lay);
  if (rc) return rc;
  if (c->ncell > kNaCells)
    return fail(c, HSGN_EINVAL, "%lld cells exceed the static scratch (at most %lld cells)",
                (long long)c->ncell, (long long)kNaCells);
  if (c->scheme != HSGN_SCHEME_SEMI_IMPLICIT)
    return fail(c, HSGN_EINVAL, "only the semi-implicit step (scheme 0) runs without allocation");
  unsigned char* base = nullptr;
  rc = na_scratch(c, &base);
  if (rc) return rc;
  // carve the buffers; every one is written before it is read, or cleared below
  size_t pos = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base + pos;
    pos += na_round(bytes);
    return (void*)p;
  };
  double* st = (double*)take(8 * kNaCells * sizeof(double));
  for (int f = 0; f < 4; ++f) {
    c->buf[0][f] = U[f];  // U^n: the caller's arrays
    c->buf[1][f] = st + (size_t)f * kNaCells;
    c->buf[2][f] = st + (size_t)(4 + f) * kNaCells;
  }
  c->d_inst = (InstDesc*)take(kNaInst * sizeof(InstDesc));
  c->d_tiles_all = (TileDesc*)take(kNaTiles * sizeof(TileDesc));
  c->d_tiles_multi = (TileDesc*)take(kNaTiles * sizeof(TileDesc));
  c->d_ex_tiles = (TileDesc*)take(kNaTiles * sizeof(TileDesc));
  c->d_ex_tiles_multi = (TileDesc*)take(kNaTiles * sizeof(TileDesc));
  c->cap_ex_tiles = c->cap_ex_tiles_multi = (size_t)kNaTiles;
  c->d_multi = (int32_t*)take(kNaInst * sizeof(int32_t));
  c->d_ex_multi = (int32_t*)take(kNaInst * sizeof(int32_t));
  c->cap_ex_multi = (size_t)kNaInst;
  c->d_win = (WinDesc*)take(kNaWins * sizeof(WinDesc));
  c->cap_win = (size_t)kNaWins;
  c->d_dt = (double*)take(kNaInst * sizeof(double));
  double* t_scr = (double*)take(kNaInst * sizeof(double));
  c->d_t = d_t ? d_t : t_scr;
  c->d_smax = (unsigned long long*)take(kNaInst * sizeof(double));
  c->d_umax = (unsigned long long*)take(kNaInst * sizeof(double));
  c->d_hmax = (unsigned long long*)take(kNaInst * sizeof(double));
  c->d_status = (int32_t*)take(kNaInst * sizeof(int32_t));
  c->d_nstep = (int32_t*)take(kNaInst * sizeof(int32_t));
  double** rp[] = {&c->d_rlo, &c->d_rdi, &c->d_rup, &c->d_rrhs, &c->d_rx,
                   &c->d_scp, &c->d_sy, &c->d_sv, &c->d_sw};
  for (double** q : rp) *q = (double*)take(2 * kNaTiles * sizeof(double));
  if (pos > kNaBytes || (int64_t)lay.tall.size() > kNaTiles || c->red_total > 2 * kNaTiles)
    return fail(c, HSGN_EINVAL, "the layout exceeds the static scratch");
  c->d_b = (double*)d_b;  // read only where an instance has a bed
  c->d_xtiles = nullptr;
  c->nxtiles = 0;
  c->cur = 0;
  c->s1 = 1;
  c->nxt = 2;
  c->solver = solver == HSGN_SOLVER_EXACT ? HSGN_SOLVER_EXACT : HSGN_SOLVER_AUTO;
  c->win_nt = solver == HSGN_SOLVER_AUTO_SMALL ? 256 : 512;
  auto up = [&](void* dst, const void* src, size_t bytes) -> int {
    if (!bytes) return HSGN_OK;
    HIPCHK(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
    return HSGN_OK;
  };
  rc = up(c->d_inst, lay.inst.data(), lay.inst.size() * sizeof(InstDesc));
  if (!rc) rc = up(c->d_tiles_all, lay.tall.data(), lay.tall.size() * sizeof(TileDesc));
  if (!rc) rc = up(c->d_tiles_multi, lay.tmulti.data(), lay.tmulti.size() * sizeof(TileDesc));
  if (!rc) rc = up(c->d_multi, lay.multi.data(), lay.multi.size() * sizeof(int32_t));
  if (rc) return rc;
  if (!d_t) {
    const unsigned nb = (unsigned)((n_inst + 255) / 256);
    hipLaunchKernelGGL(k_fill_f64, dim3(nb), dim3(256), 0, c->stream, (int64_t)n_inst, c->d_t, 0.0);
  }
  // flags, step counts and speed bounds cleared, the plan made (this
  // synchronises the stream, so the uploads above are complete on return)
  rc = reset_and_plan(c);
  if (rc) return rc;
  for (int s = 0; s < nsteps && rc == HSGN_OK; ++s) rc = enqueue_step(c);
  if (rc) return rc;
  if (c->cur != 0) {  // odd step count: the state is in the scratch
    const size_t bytes = (size_t)c->ncell * sizeof(double);
    for (int f = 0; f < 4; ++f)
      HIPCHK(c, hipMemcpyAsync(U[f], c->buf[c->cur][f], bytes, hipMemcpyDeviceToDevice,
                               c->stream));
  }
  return read_status(c, "hsgn_step_noalloc", h_flags);
}

}  // namespace

extern "C" int hsgn_step_noalloc(int32_t n_inst, const int64_t* offsets,
                                 const hsgn_params* params, const double* d_b, double* d_h,
                                 double* d_q, double* d_m, double* d_W, double* d_t,
                                 int32_t nsteps, int32_t solver, void* hip_stream,
                                 int32_t* h_flags, char* h_msg) {
  if (h_msg) h_msg[0] = '\0';
  hsgn_ctx c;  // host bookkeeping only; its device pointers all point into the scratch
  c.no_alloc = true;
  c.user_stream = c.stream = (hipStream_t)hip_stream;
  int rc = HSGN_OK;
  if (n_inst <= 0 || !offsets || !params || !d_h || !d_q || !d_m || !d_W || nsteps < 0)
    rc = fail(&c, HSGN_EINVAL, "hsgn_step_noalloc: bad arguments");
  else if (n_inst > kNaInst)
    rc = fail(&c, HSGN_EINVAL, "hsgn_step_noalloc: %d instances exceed the static scratch "
              "(at most %lld)", n_inst, (long long)kNaInst);
  else if (solver != HSGN_SOLVER_AUTO && solver != HSGN_SOLVER_EXACT &&
           solver != HSGN_SOLVER_AUTO_SMALL)
    rc = fail(&c, HSGN_EINVAL, "hsgn_step_noalloc: unknown solver mode %d", solver);
  else {
    double* U[4] = {d_h, d_q, d_m, d_W};
    rc = na_run(&c, n_inst, offsets, params, d_b, U, d_t, nsteps, solver, h_flags);
  }
  if (rc && h_msg) {
    std::strncpy(h_msg, c.err.c_str(), HSGN_MSG_LEN - 1);
    h_msg[HSGN_MSG_LEN - 1] = '\0';
  }
  return rc;
}

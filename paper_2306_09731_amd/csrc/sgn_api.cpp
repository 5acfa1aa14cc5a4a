// C-ABI of libsgn: argument checks, workspace layout, the GMRES control
// loop and the RK4 / RHS / invariants sequences of kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "sgn.h"
#include "sgn_cnn_internal.hpp"
#include "sgn_internal.hpp"
#include "sgn_launch.hpp"
#include "sgn_host.hpp"

typedef double2 cplx;

struct sgn_ctx {
  sgn_config cfg;
  int device;  // HIP device current at sgn_init
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  size_t ws_stride;  // bytes between ensemble members' workspaces
  sgn::Geom g;
  size_t vstride;      // complex entries (of the working precision) per field
  size_t field_bytes;  // bytes per field (256-byte multiple)
  sgn::GmresState* st;
  double* partials;   // block partials of the reductions
  double* partials2;  // second buffer: kernel C's, reduced by kernel A while it writes its own
  // fields of the working precision (FP64 or FP32), untyped on the host
  void *V, *Z, *W, *E, *G, *P, *Q, *R1, *R2, *SIG;
  char* D;  // guess 1: four per-stage sigma increments (2D spectra), else null
  void *hs, *vxs, *vys, *acc_h, *acc_vx, *acc_vy;
  sgn::GmresStatus* hstat;  // pinned host copy of the device status (one per ensemble member)
  hipEvent_t stat_ev = nullptr;  // recorded after the status copy of a speculative batch
  int batch_margin = 0;  // Arnoldi steps enqueued beyond the previous solve's count
  int last_iters[5];  // iterations of the previous solve per slot (RK stages 0-3, other calls 4)
  int arnoldi;   // 0 serial 4-kernel, 1 chain-parallel 4-kernel, 2 three-kernel (default where allowed)
  std::string err;
  // kernel timing (measurement support)
  int timed_kind = -1;
  std::vector<hipEvent_t> ev_free;
  std::deque<std::pair<hipEvent_t, hipEvent_t>> ev_pending;  // oldest first
  int64_t timed_launches = 0;  // launches that carried events (durations collected)
  int64_t timed_all = 0;       // all launches of the class while timing was on
  int timed_period = 1;        // events on every timed_period-th launch
  double timed_ms = 0.0;
  double timed_bytes = 0.0;  // algorithmic bytes of the timed launches that did work
  // captured RK4 step (sgn_rk4_step_graph)
  // h, vx, vy and the carried solver state (SIG, E, G, with the stage-increment
  // guess D_0..D_3) at the start of a chunk of captured steps
  char* ckpt = nullptr;
  hipStream_t gstream = nullptr;    // private stream: capture and replays
  hipEvent_t gev[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};  // first step of a call, later steps
  struct GraphKey {
    const void *h = nullptr, *vx = nullptr, *vy = nullptr;
    double dt = 0.0;
    int budget[4] = {0, 0, 0, 0};
    int arnoldi = 0, tile_blocks = 0, row_threads = 0;  // the launch shapes captured
    bool operator==(const GraphKey& o) const {
      return h == o.h && vx == o.vx && vy == o.vy && dt == o.dt && std::equal(budget, budget + 4, o.budget) &&
             arnoldi == o.arnoldi && tile_blocks == o.tile_blocks && row_threads == o.row_threads;
    }
  } gkey[2];
  // Arnoldi steps per captured solve, per RK stage (0: not yet calibrated):
  // the most the stage needed in the host-driven steps seen, plus graph_margin
  int graph_budgets[4] = {0, 0, 0, 0};
  int graph_margin = 0;
  // captured kernels test the GMRES status before their loads (1) or after (0,
  // as the host-driven loop does); 1 measured faster in replays (1024x512
  // FP64: 1.874 against 1.958 ms per step)
  int graph_status_first = 1;
  int stage_max[4] = {0, 0, 0, 0};  // most iterations per RK stage in the host-driven steps since a reset
  // learned initial guess (sgn_learned_guess_attach)
  sgn_cnn* learn_net = nullptr;  // network correcting the warm start, or null
  int32_t learn_stages = 0xF;    // RK stages whose solves the network corrects (bit s: stage s)
  float* learn_rec = nullptr;    // recorder: learn_cap slots of (input [n][3], target [n])
  int32_t learn_cap = 0;
  int64_t learn_count = 0;       // solves recorded
};

namespace {
bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }
}  // namespace

namespace sgn {

int check_config(const sgn_config* c) {
  if (!c) return SGN_ERR_INVALID_ARG;
  if (!(std::isfinite(c->Lx) && c->Lx > 0 && std::isfinite(c->Ly) && c->Ly > 0)) return SGN_ERR_INVALID_ARG;
  if (!(std::isfinite(c->g) && c->g > 0 && std::isfinite(c->h_inf) && c->h_inf > 0)) return SGN_ERR_INVALID_ARG;
  if (!(std::isfinite(c->gmres_tol) && c->gmres_tol > 0)) return SGN_ERR_INVALID_ARG;
  if (!(std::isfinite(c->invariants_tol) && c->invariants_tol > 0)) return SGN_ERR_INVALID_ARG;
  if (!(std::isfinite(c->krasny) && c->krasny >= 0)) return SGN_ERR_INVALID_ARG;
  if (c->dealias != 0 && c->dealias != 1) return SGN_ERR_INVALID_ARG;
  if (c->guess != SGN_GUESS_PREVIOUS && c->guess != SGN_GUESS_STAGE_INCREMENT) return SGN_ERR_INVALID_ARG;
  if (c->gmres_max_iters < 1) return SGN_ERR_INVALID_ARG;
  if (c->gmres_restart < 1) return SGN_ERR_INVALID_ARG;
  if (c->gmres_restart > sgn::kMaxRestart) return SGN_ERR_UNSUPPORTED;
  if (c->precision != SGN_FP64 && c->precision != SGN_FP32_MIXED) return SGN_ERR_UNSUPPORTED;
  if (c->batch < 1 || c->batch > SGN_MAX_MEMBERS) return SGN_ERR_UNSUPPORTED;
  if (!pow2_in(c->nx, 8, 4096) || !pow2_in(c->ny, 8, 4096)) return SGN_ERR_UNSUPPORTED;
  return SGN_OK;
}

// Grid geometry, spectral constants and launch shapes of a configuration (the
// table pointers are set by the caller, which owns the tables' memory).
void geom_init(const sgn_config& c, Geom& g) {
  g = Geom{};
  g.nx = c.nx;
  g.ny = c.ny;
  g.nh = c.nx / 2;
  g.inv_Lx = 1.0 / c.Lx;
  g.inv_Ly = 1.0 / c.Ly;
  g.inv_nx = 1.0 / c.nx;
  g.inv_ny = 1.0 / c.ny;
  g.inv_n = 1.0 / ((double)c.nx * c.ny);
  g.g = c.g;
  g.h_inf = c.h_inf;
  g.m0 = 3.0 / (c.h_inf * c.h_inf * c.h_inf);
  g.m1 = 1.0 / c.h_inf;
  g.dA = (2.0 * M_PI * c.Lx / c.nx) * (2.0 * M_PI * c.Ly / c.ny);
  g.fp32 = c.precision == SGN_FP32_MIXED;
  g.m = c.gmres_restart;
  // launch shapes (tuning and testing switches; sgn_autotune searches them):
  // SGN_TILE_BLOCKS, the number of blocks below which column tiles stop
  // widening, and SGN_ROW_THREADS, the threads a row block reaches by taking
  // several row pairs (powers of two)
  g.tile_blocks = 256;
  g.row_threads = 64;
  g.status_first = 0;
  g.members = 1;
  g.row_split = 1;
  if (const char* rs = std::getenv("SGN_ROW_SPLIT")) g.row_split = std::atoi(rs) != 0;
  g.row_radix = 0;
  if (const char* rr = std::getenv("SGN_ROW_RADIX")) g.row_radix = std::atoi(rr) == 8 ? 8 : 0;
  g.ws_lo = 0;
  g.ws_span = g.ws_stride = g.f_stride = 0;
  if (const char* tb = std::getenv("SGN_TILE_BLOCKS")) {
    const int v = std::atoi(tb);
    if (v >= 1 && v <= 4096 && (v & (v - 1)) == 0) g.tile_blocks = v;
  }
  if (const char* rt = std::getenv("SGN_ROW_THREADS")) {
    const int v = std::atoi(rt);
    if (v >= 64 && v <= 512 && (v & (v - 1)) == 0) g.row_threads = v;
  }
}

// Message of the last failed call that has no context (sgn_last_error(NULL)).
static thread_local char t_global_err[256];
void set_global_error(const char* msg) { snprintf(t_global_err, sizeof t_global_err, "%s", msg); }
const char* global_error() { return t_global_err; }

}  // namespace sgn

namespace {
using sgn::check_config;

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// GMRES tolerance actually used: an FP32 operator cannot reduce the residual
// much below 1e-6 relative, so the mixed-precision mode stops there.
constexpr double kFp32MinTol = 1e-6;
double effective_tol(const sgn_config& c, double tol) {
  return c.precision == SGN_FP32_MIXED && tol < kFp32MinTol ? kFp32MinTol : tol;
}

// The spectral filter applied to h, v_x, v_y after every RK4 step: the Krasny
// threshold (Section 3) and, if enabled, the two-thirds rule.
bool step_filter_on(const sgn_config& c) { return c.krasny > 0.0 || c.dealias != 0; }
int step_filter_op(const sgn_config& c) { return c.dealias ? 2 : 1; }

struct Layout {
  size_t tw, st, partials, partials2, fields;
  size_t member;  // bytes of one member's workspace (256-byte multiple)
  size_t total;   // batch * member
  size_t field_bytes;
  int nfields;
};

int ckpt_fields(const sgn_config* c) { return 6 + (c->guess == SGN_GUESS_STAGE_INCREMENT ? 4 : 0); }

Layout layout(const sgn_config* c) {
  Layout L;
  const size_t n = (size_t)c->nx * c->ny;
  L.field_bytes = align_up(n * (c->precision == SGN_FP32_MIXED ? sizeof(float) : sizeof(double)));
  sgn::Geom g{};
  g.nx = c->nx;
  g.ny = c->ny;
  g.nh = c->nx / 2;
  g.fp32 = c->precision == SGN_FP32_MIXED;
  const int pblocks = sgn::max_partial_blocks(g);
  size_t off = 0;
  L.tw = off;
  off += align_up((size_t)(c->nx + c->ny) * sizeof(double2));  // FP64 twiddles
  off += align_up((size_t)(c->nx + c->ny) * sizeof(float2));   // FP32 twiddles
  L.st = off;
  off += align_up(sizeof(sgn::GmresState));
  L.partials = off;
  off += align_up((size_t)pblocks * sgn::kPartialStride * sizeof(double));
  L.partials2 = off;
  off += align_up((size_t)pblocks * sgn::kPartialStride * sizeof(double));
  L.fields = off;
  // V (restart + 1), Z, W, E, G, P, Q, R1, R2, SIG, hs, vxs, vys, acc_h, acc_vx, acc_vy,
  // the checkpoint of captured steps (h, vx, vy, SIG, E, G, and D_0..D_3 with the
  // stage-increment guess), and with that guess D_0..D_3
  L.nfields = c->gmres_restart + 1 + 15 + ckpt_fields(c) + (c->guess == SGN_GUESS_STAGE_INCREMENT ? 4 : 0);
  off += (size_t)L.nfields * L.field_bytes;
  L.member = align_up(off);
  L.total = L.member * (size_t)c->batch;
  return L;
}

int fail(sgn_ctx* ctx, hipError_t e, const char* what) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
  ctx->err = buf;
  return SGN_ERR_HIP;
}

#define HIPCK(expr)                                   \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return fail(ctx, e_, #expr); \
  } while (0)

bool aligned(const void* p) { return p && (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

hipEvent_t take_event(sgn_ctx* ctx) {
  if (!ctx->ev_free.empty()) {
    hipEvent_t e = ctx->ev_free.back();
    ctx->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  // no system-scope fence: the timing events are never waited on by the host
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

// Accumulate the durations of the recorded event pairs (synchronises).
int drain_timing(sgn_ctx* ctx) {
  if (ctx->ev_pending.empty()) return SGN_OK;
  HIPCK(hipStreamSynchronize(ctx->stream));
  for (auto& pr : ctx->ev_pending) {
    float ms = 0.f;
    HIPCK(hipEventElapsedTime(&ms, pr.first, pr.second));
    ctx->timed_ms += ms;
    ctx->timed_launches += 1;
    ctx->ev_free.push_back(pr.first);
    ctx->ev_free.push_back(pr.second);
  }
  ctx->ev_pending.clear();
  return SGN_OK;
}

// When a kernel class is being timed, every timed_period-th launch of it
// carries a pair of events that the runtime records at the start and end of
// the dispatch.
struct KernelTimer {
  sgn_ctx* ctx;
  hipEvent_t a = nullptr, b = nullptr;
  KernelTimer(sgn_ctx* c, int kind) : ctx(c) {
    if (c->timed_kind != kind) return;
    if (c->timed_all++ % c->timed_period != 0) return;
    a = take_event(c);
    b = take_event(c);
    if (a && b) sgn::set_launch_events(a, b);
  }
  void stop() {
    sgn::set_launch_events(nullptr, nullptr);
    if (!a || !b) return;
    ctx->ev_pending.emplace_back(a, b);
    a = b = nullptr;
    // collect finished pairs a few at a time, oldest first, so that the list
    // stays short without a synchronisation inside the timed work
    for (int k = 0; k < 2 && ctx->ev_pending.size() > 256; ++k) {
      const auto pr = ctx->ev_pending.front();
      if (hipEventQuery(pr.second) != hipSuccess) break;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess) break;
      ctx->timed_ms += ms;
      ctx->timed_launches += 1;
      ctx->ev_free.push_back(pr.first);
      ctx->ev_free.push_back(pr.second);
      ctx->ev_pending.pop_front();
    }
    if (ctx->ev_pending.size() >= 65536) (void)drain_timing(ctx);
  }
};

#define TIMED(kind, expr)              \
  do {                                 \
    KernelTimer kt_(ctx, kind);        \
    HIPCK(expr);                       \
    kt_.stop();                        \
  } while (0)

int members(const sgn_ctx* ctx) { return ctx->cfg.batch; }

// The device status of every member into hstat (one strided copy).
int copy_status(sgn_ctx* ctx) {
  if (members(ctx) == 1)
    HIPCK(hipMemcpyAsync(ctx->hstat, &ctx->st->st, sizeof(sgn::GmresStatus), hipMemcpyDeviceToHost, ctx->stream));
  else
    HIPCK(hipMemcpy2DAsync(ctx->hstat, sizeof(sgn::GmresStatus), &ctx->st->st, ctx->ws_stride,
                           sizeof(sgn::GmresStatus), members(ctx), hipMemcpyDeviceToHost, ctx->stream));
  return SGN_OK;
}

int read_status(sgn_ctx* ctx) {
  int rc = copy_status(ctx);
  if (rc) return rc;
  HIPCK(hipStreamSynchronize(ctx->stream));
  return SGN_OK;
}

// A scalar of every member's GMRES state set from the host.
template <class T>
int set_state_scalar(sgn_ctx* ctx, T* field0, T v) {
  for (int k = 0; k < members(ctx); ++k)
    HIPCK(hipMemcpyAsync(reinterpret_cast<char*>(field0) + (size_t)k * ctx->ws_stride, &v, sizeof v,
                         hipMemcpyHostToDevice, ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));  // v is a host local
  return SGN_OK;
}

int set_tol(sgn_ctx* ctx, double tol_requested) {
  return set_state_scalar(ctx, &ctx->st->tol, effective_tol(ctx->cfg, tol_requested));
}

// sigma (physical) -> E = F_x sigma, SIG = F sigma, G = F_x d_y sigma
int load_sigma(sgn_ctx* ctx, const void* sigma) {
  HIPCK(sgn::launch_row_r2c(ctx->g, sigma, ctx->E, ctx->stream));
  HIPCK(sgn::launch_col_fwd_eg(ctx->g, ctx->E, ctx->SIG, ctx->G, ctx->stream));
  return SGN_OK;
}

int check_state(sgn_ctx* ctx, const void* a, const void* b, const void* c) {
  HIPCK(sgn::launch_field_stats(ctx->g, a, b, c, (size_t)ctx->g.nx * ctx->g.ny, ctx->st, ctx->partials, ctx->stream));
  int rc = read_status(ctx);
  if (rc) return rc;
  for (int k = 0; k < members(ctx); ++k) {
    if (ctx->hstat[k].stat_nonfinite) {
      ctx->err = "non-finite value in the input";
      if (members(ctx) > 1) ctx->err += " of member " + std::to_string(k);
      return SGN_ERR_NONFINITE;
    }
    if (!(ctx->hstat[k].stat_minh > 0.0)) {
      ctx->err = "min h <= 0";
      if (members(ctx) > 1) ctx->err += " in member " + std::to_string(k);
      return SGN_ERR_CAVITATION;
    }
  }
  return SGN_OK;
}

struct SolveResult {
  int iters = 0, restarts = 0, converged = 0;
  double rel_resid = 0.0;
  bool post_done = false;  // the caller's post-solve work ran predicated (run_solve)
};

// ---- kernel sequences shared by the host-driven loop and the captured step

// Start of a GMRES cycle: residual (and b, if need_b) of the current sigma.
// flags: 1 a new solve; 4 | (round << 8) an ensemble restart in that cycle
// round (only the members that restart run it).
int enqueue_residual(sgn_ctx* ctx, int mode, const void* h, const void* vx, const void* vy, int need_b, int flags) {
  const sgn::Geom& g = ctx->g;
  hipStream_t s = ctx->stream;
  const int rowpred = (flags & 4) ? 2 : 0;
  HIPCK(sgn::launch_row_op(g, mode, ctx->E, ctx->G, h, vx, vy, ctx->P, ctx->Q, ctx->R1, ctx->R2, need_b, rowpred,
                           ctx->st, s));
  // an explicit b (mode 2) has b_hat = F_y(R1) only.  In the three-kernel
  // schedule the residual pass also produces E, G of the residual (the work
  // of kernel A at step 0); its last block sets beta
  const bool fused = ctx->arnoldi == 2;
  HIPCK(sgn::launch_col_resid(g, ctx->P, ctx->Q, ctx->R1, mode == 2 ? nullptr : ctx->R2, need_b, flags, ctx->st,
                              ctx->W, ctx->partials, fused ? ctx->E : nullptr, fused ? ctx->G : nullptr, s));
  if (fused) {
    TIMED(SGN_KERNEL_ROW_MATVEC,
          sgn::launch_row_matvec3(g, ctx->E, ctx->G, h, ctx->P, ctx->Q, ctx->st, s));
  } else if (ctx->arnoldi == 1) {  // basis kernel of step 0: V_0, E, G
    TIMED(SGN_KERNEL_COL_BASIS,
          sgn::launch_col_basis2(g, ctx->W, ctx->V, ctx->vstride, 0, ctx->st, ctx->E, ctx->G, nullptr, s));
  } else {
    TIMED(SGN_KERNEL_COL_BASIS,
          sgn::launch_col_basis_eg(g, ctx->W, ctx->V, ctx->vstride, 0, ctx->st, ctx->E, ctx->G, nullptr, s));
  }
  return SGN_OK;
}

// Arnoldi step `it` of the cycle (every kernel exits at once once the device
// status says done).
int enqueue_arnoldi(sgn_ctx* ctx, const void* h, int it) {
  const sgn::Geom& g = ctx->g;
  hipStream_t s = ctx->stream;
  if (ctx->arnoldi == 2) {
    // C_it, A_it+1, B_it+1: A_it+1 finishes step it (and stops the cycle
    // there when it ends), so the device status is current after every step
    TIMED(SGN_KERNEL_COL_PRECOND_DOT, sgn::launch_col_precond_new(g, ctx->P, ctx->Q, ctx->W, ctx->V, ctx->Z,
                                                                  ctx->vstride, it, ctx->st, ctx->partials2, s));
    TIMED(SGN_KERNEL_COL_BASIS, sgn::launch_col_proj(g, ctx->Z, ctx->W, ctx->V, ctx->vstride, it + 1, ctx->st,
                                                     ctx->E, ctx->G, ctx->partials2, s));
    TIMED(SGN_KERNEL_ROW_MATVEC,
          sgn::launch_row_matvec3(g, ctx->E, ctx->G, h, ctx->P, ctx->Q, ctx->st, s));
    return SGN_OK;
  }
  // four-kernel step it: x part, projections, update, and the basis kernel of
  // step it + 1, which finishes step it (so the status is current)
  const bool two = ctx->arnoldi == 1;
  if (two) {
    TIMED(SGN_KERNEL_ROW_MATVEC,
          sgn::launch_row_matvec3(g, ctx->E, ctx->G, h, ctx->P, ctx->Q, ctx->st, s));
    TIMED(SGN_KERNEL_COL_PRECOND_DOT, sgn::launch_col_precond_dot2(g, ctx->P, ctx->Q, ctx->V, ctx->vstride, it,
                                                                   ctx->st, ctx->W, ctx->partials2, s));
  } else {
    TIMED(SGN_KERNEL_ROW_MATVEC, sgn::launch_row_op(g, 0, ctx->E, ctx->G, h, nullptr, nullptr, ctx->P, ctx->Q,
                                                    nullptr, nullptr, 0, 1, ctx->st, s));
    TIMED(SGN_KERNEL_COL_PRECOND_DOT, sgn::launch_col_precond_dot(g, ctx->P, ctx->Q, ctx->V, ctx->vstride, it,
                                                                  ctx->st, ctx->W, ctx->partials2, s));
  }
  TIMED(SGN_KERNEL_GS_UPDATE, sgn::launch_upd(g, ctx->W, ctx->V, ctx->vstride, it, ctx->st, ctx->partials,
                                              ctx->partials2, two ? 1 : 0, s));
  if (two)
    TIMED(SGN_KERNEL_COL_BASIS, sgn::launch_col_basis2(g, ctx->W, ctx->V, ctx->vstride, it + 1, ctx->st, ctx->E,
                                                       ctx->G, ctx->partials, s));
  else
    TIMED(SGN_KERNEL_COL_BASIS, sgn::launch_col_basis_eg(g, ctx->W, ctx->V, ctx->vstride, it + 1, ctx->st, ctx->E,
                                                         ctx->G, ctx->partials, s));
  return SGN_OK;
}

// RK4 stage `stage` after its solve: fluxes, Bernoulli function and the
// stage combine (stage input (ih, ivx, ivy); the step's state h, vx, vy).
int enqueue_stage_flux(sgn_ctx* ctx, int stage, double dt, void* h, void* vx, void* vy, const void* ih,
                       const void* ivx, const void* ivy, bool spec = false) {
  const sgn::Geom& g = ctx->g;
  hipStream_t s = ctx->stream;
  sgn::RkStage rk;
  if (stage < 3) {
    rk.mode = 1;
    rk.first = stage == 0;
    rk.wacc = stage == 0 ? 1.0 / 6.0 : 1.0 / 3.0;
    rk.cnext = stage == 2 ? dt : 0.5 * dt;
  } else {
    rk.mode = 2;
    rk.first = 0;
    rk.wacc = 1.0 / 6.0;
    rk.cnext = 0.0;
  }
  rk.dt = dt;
  rk.pred = spec ? &ctx->st->st : nullptr;
  const bool last = stage == 3;
  sgn::RkField fvx{vx, ctx->acc_vx, last ? vx : ctx->vxs};
  sgn::RkField fh{h, ctx->acc_h, last ? h : ctx->hs};
  sgn::RkField fvy{vy, ctx->acc_vy, last ? vy : ctx->vys};
  TIMED(SGN_KERNEL_ROW_FLUX, sgn::launch_row_flux(g, ctx->E, ctx->G, ih, ivx, ivy, ctx->P, ctx->Q, ctx->R1, rk, fvx, s));
  TIMED(SGN_KERNEL_COL_FLUX, sgn::launch_col_flux(g, ctx->P, ctx->Q, ctx->R1, rk, fh, fvy, s));
  return SGN_OK;
}

// The per-step spectral filter (Krasny, two-thirds rule) of h, vx, vy.
int enqueue_step_filter(sgn_ctx* ctx, void* h, void* vx, void* vy) {
  if (!step_filter_on(ctx->cfg)) return SGN_OK;
  const sgn::Geom& g = ctx->g;
  hipStream_t s = ctx->stream;
  // the three fields in one launch of each pass; scratch (free between
  // solves): P, Q, R1 for the x-half spectra, R2, W, Z for the filtered ones
  void* fl[3] = {ctx->R2, ctx->W, ctx->Z};
  HIPCK(sgn::launch_row_r2c3(g, sgn::Trio{{h, vx, vy}, {ctx->P, ctx->Q, ctx->R1}}, s));
  HIPCK(sgn::launch_col_filter3(g, sgn::Trio{{ctx->P, ctx->Q, ctx->R1}, {fl[0], fl[1], fl[2]}},
                                step_filter_op(ctx->cfg), ctx->cfg.krasny, s));
  HIPCK(sgn::launch_row_c2r3(g, sgn::Trio{{fl[0], fl[1], fl[2]}, {h, vx, vy}}, s));
  return SGN_OK;
}

double cycle_timed_bytes(const sgn_ctx* ctx, int jd);
int run_solve_members(sgn_ctx* ctx, int mode, const void* h, const void* vx, const void* vy, SolveResult* res,
                      int slot, void* D);

// Restarted GMRES for L_h sigma = b with the warm start held in (SIG, E, G).
// mode 1: b = -div v from (vx, vy); mode 2: b given (passed as vx).
// On return (SIG, E, G) hold the solution.
// slot: which history predicts the iteration count (the RK stage, or 4).
// post (may be null): enqueues the caller's work that follows the solve.
// With it, every batch of Arnoldi steps is followed, before the host waits
// for the status, by the solution update and post(true), all predicated on
// the solve having converged: the GPU goes on with them while the host reads
// the status.  res->post_done tells the caller that they did run.
int run_solve(sgn_ctx* ctx, int mode, const void* h, const void* vx, const void* vy, SolveResult* res,
              int slot = 4, void* D = nullptr, const std::function<int(bool)>* post = nullptr) {
  if (members(ctx) > 1) return run_solve_members(ctx, mode, h, vx, vy, res, slot, D);
  const sgn::Geom& g = ctx->g;
  hipStream_t s = ctx->stream;
  const int m = ctx->cfg.gmres_restart;
  const int maxit = ctx->cfg.gmres_max_iters;
  int need_b = 1, flags = 1;
  int total = 0;
  res->restarts = 0;
  res->converged = 0;
  res->post_done = false;
  if (post && !ctx->stat_ev) HIPCK(hipEventCreateWithFlags(&ctx->stat_ev, hipEventDisableTiming));
  for (;;) {
    int rc0 = enqueue_residual(ctx, mode, h, vx, vy, need_b, flags);
    if (rc0) return rc0;
    need_b = 0;
    flags = 0;
    int j = 0;
    // speculative batch: as many steps as this slot's previous solve needed
    // (plus batch_margin; 0 measured fastest at every size tried)
    int batch = (res->restarts == 0 ? ctx->last_iters[slot] : m) + ctx->batch_margin;
    if (batch < 1) batch = 1;
    for (;;) {
      int nrun = batch;
      if (nrun > m - j) nrun = m - j;
      if (nrun > maxit - total - j) nrun = maxit - total - j;
      if (nrun <= 0) break;  // the device sets done at the cycle or iteration cap
      for (int it = j; it < j + nrun; ++it) {
        int rc1 = enqueue_arnoldi(ctx, h, it);
        if (rc1) return rc1;
      }
      j += nrun;
      if (post) {
        HIPCK(hipMemcpyAsync(ctx->hstat, &ctx->st->st, sizeof(sgn::GmresStatus), hipMemcpyDeviceToHost, s));
        HIPCK(hipEventRecord(ctx->stat_ev, s));
        HIPCK(sgn::launch_col_update_eg(g, ctx->SIG, ctx->V, ctx->vstride, ctx->st, ctx->E, ctx->G, D, 1, s));
        int rc = (*post)(true);
        if (rc) return rc;
        HIPCK(hipEventSynchronize(ctx->stat_ev));
        res->post_done = ctx->hstat->done == 1;
      } else {
        int rc = read_status(ctx);
        if (rc) return rc;
      }
      if (ctx->hstat->done) break;
      batch = 2;
    }
    const sgn::GmresStatus& st = *ctx->hstat;
    if (ctx->timed_kind >= 0) {
      const bool ran = !(st.done == 1 && st.jdone == 0 && st.total_iters == total);
      if (ran) ctx->timed_bytes += cycle_timed_bytes(ctx, st.jdone);
    }
    total = st.total_iters;
    // sigma_hat += V y, and E, G of the new sigma (already enqueued when a
    // predicated update ran)
    if (!res->post_done)
      HIPCK(sgn::launch_col_update_eg(g, ctx->SIG, ctx->V, ctx->vstride, ctx->st, ctx->E, ctx->G, D, 0, s));
    res->rel_resid = st.beta0 > 0 ? st.resid / st.beta0 : 0.0;
    if (st.done == 1) {
      res->converged = 1;
      break;
    }
    if (total >= maxit) break;
    res->restarts += 1;
  }
  res->iters = total;
  ctx->last_iters[slot] = total < m ? total : m;
  return SGN_OK;
}

// Algorithmic bytes of one cycle's launches that did work (fields of fb
// bytes read or written once) for the timed kernel class: a cycle of jd
// Arnoldi steps that ran (not converged at its start).  Three-kernel step j:
// A (j+4), B 5, C (j+5), with A's pass for 1 <= j < jd (A_jd stops the cycle
// before its pass; step 0's A is part of the residual pass) and B's
// transforms for j < jd.  Four-kernel step j: basis (j+4), x part 5,
// projections (j+4), update (j+3).
double cycle_timed_bytes(const sgn_ctx* ctx, int jd) {
  const sgn::Geom& g = ctx->g;
  const double fb = (g.fp32 ? 4.0 : 8.0) * (double)g.nx * (double)g.ny;
  double b = 0.0;
  if (ctx->timed_kind == SGN_KERNEL_ROW_MATVEC) b += 5.0 * jd * fb;
  if (ctx->arnoldi == 2) {
    if (ctx->timed_kind == SGN_KERNEL_COL_PRECOND_DOT)
      for (int jj = 0; jj < jd; ++jj) b += (jj + 5) * fb;
    if (ctx->timed_kind == SGN_KERNEL_COL_BASIS)
      for (int jj = 1; jj < jd; ++jj) b += (jj + 4) * fb;
  } else {
    for (int jj = 0; jj < jd; ++jj) {
      if (ctx->timed_kind == SGN_KERNEL_COL_BASIS || ctx->timed_kind == SGN_KERNEL_COL_PRECOND_DOT)
        b += (jj + 4) * fb;
      if (ctx->timed_kind == SGN_KERNEL_GS_UPDATE) b += (jj + 3) * fb;
    }
  }
  return b;
}

// run_solve for a context of several ensemble members: every launch covers
// all members, each member's kernels exit once its own status says done.
// Cycle round 0 starts every member; a later round restarts only the members
// whose cycle filled up (their residual passes test that on the device), and
// the solution update of a round runs only for the members that ran a cycle
// in it.  The host reads all members' status words once per batch of
// Arnoldi steps and goes on until every member has stopped.
int run_solve_members(sgn_ctx* ctx, int mode, const void* h, const void* vx, const void* vy, SolveResult* res,
                      int slot, void* D) {
  const sgn::Geom& g = ctx->g;
  hipStream_t s = ctx->stream;
  const int M = members(ctx);
  const int m = ctx->cfg.gmres_restart;
  const int maxit = ctx->cfg.gmres_max_iters;
  std::vector<int> before(M, 0);
  for (int k = 0; k < M; ++k) res[k] = SolveResult{};
  int most = 0;
  for (int round = 0;; ++round) {
    int rc0 = enqueue_residual(ctx, mode, h, vx, vy, round == 0 ? 1 : 0, round == 0 ? 1 : (4 | (round << 8)));
    if (rc0) return rc0;
    int j = 0;
    int batch = (round == 0 ? ctx->last_iters[slot] : m) + ctx->batch_margin;
    if (batch < 1) batch = 1;
    for (;;) {
      int nrun = batch;
      if (nrun > m - j) nrun = m - j;
      if (nrun <= 0) break;  // the device stops every member at its cycle or iteration cap
      for (int it = j; it < j + nrun; ++it) {
        int rc1 = enqueue_arnoldi(ctx, h, it);
        if (rc1) return rc1;
      }
      j += nrun;
      int rc = read_status(ctx);
      if (rc) return rc;
      bool all = true;
      for (int k = 0; k < M; ++k) all = all && ctx->hstat[k].done != 0;
      if (all) break;
      batch = 2;
    }
    HIPCK(sgn::launch_col_update_eg(g, ctx->SIG, ctx->V, ctx->vstride, ctx->st, ctx->E, ctx->G, D,
                                    2 | (round << 8), s));
    bool again = false;
    for (int k = 0; k < M; ++k) {
      const sgn::GmresStatus& st = ctx->hstat[k];
      if (st.cyc != round) continue;  // stopped in an earlier round
      if (ctx->timed_kind >= 0) {
        const bool ran = !(st.done == 1 && st.jdone == 0 && st.total_iters == before[k]);
        if (ran) ctx->timed_bytes += cycle_timed_bytes(ctx, st.jdone);
      }
      before[k] = st.total_iters;
      res[k].iters = st.total_iters;
      res[k].rel_resid = st.beta0 > 0 ? st.resid / st.beta0 : 0.0;
      res[k].converged = st.done == 1;
      if (st.done == 2 && st.total_iters < maxit) {
        res[k].restarts += 1;
        again = true;
      }
      most = std::max(most, std::min(st.total_iters, m));
    }
    if (!again) break;
  }
  ctx->last_iters[slot] = most;
  return SGN_OK;
}

bool all_converged(const std::vector<SolveResult>& r) {
  for (const SolveResult& x : r)
    if (!x.converged) return false;
  return true;
}

// The stage-increment guess starts every call from zero increments.
int clear_guess(sgn_ctx* ctx) {
  if (!ctx->D) return SGN_OK;
  if (members(ctx) == 1)
    HIPCK(hipMemsetAsync(ctx->D, 0, 4 * ctx->field_bytes, ctx->stream));
  else
    HIPCK(hipMemset2DAsync(ctx->D, ctx->ws_stride, 0, 4 * ctx->field_bytes, members(ctx), ctx->stream));
  return SGN_OK;
}

// ---- the learned initial guess

// Start of a solve with the learned guess or the recorder: r0 = b - L sigma_prev
// and M^-1 r0 from the GMRES start kernels, their scale |r0| (RMS, in the
// device state), the network input (into the recorder's slot when recording)
// and, with use_net, sigma_prev replaced by sigma_prev + |r0| net(input).
// Scratch: V_0, V_1, V_2 (physical r0, M^-1 r0, the guess; the solve
// overwrites them afterwards), R1, R2 (x-half spectra) and the first
// checkpoint field (sigma_prev, kept for the recorder's target).
int learned_start(sgn_ctx* ctx, const void* h, const void* vx, const void* vy, float** slot, bool use_net) {
  const sgn::Geom& g = ctx->g;
  hipStream_t s = ctx->stream;
  const size_t n = (size_t)g.nx * g.ny;
  char* V = static_cast<char*>(ctx->V);
  void* r0 = V;
  void* mr0 = V + ctx->field_bytes;
  void* sg = V + 2 * ctx->field_bytes;
  void* sp = ctx->ckpt;
  HIPCK(sgn::launch_row_op(g, 1, ctx->E, ctx->G, h, vx, vy, ctx->P, ctx->Q, ctx->R1, ctx->R2, 1, 0, ctx->st, s));
  HIPCK(sgn::launch_col_resid(g, ctx->P, ctx->Q, ctx->R1, ctx->R2, 1, 1, ctx->st, ctx->W, ctx->partials, nullptr,
                              nullptr, s));
  HIPCK(sgn::launch_col_learn(g, ctx->W, ctx->R1, ctx->R2, s));
  HIPCK(sgn::launch_row_c2r(g, ctx->R1, r0, s));
  HIPCK(sgn::launch_row_c2r(g, ctx->R2, mr0, s));
  HIPCK(sgn::launch_row_c2r(g, ctx->E, sp, s));
  HIPCK(sgn::launch_learn_norm(g, r0, n, ctx->st, ctx->partials, s));
  float* in3;
  if (ctx->learn_rec) {
    *slot = ctx->learn_rec + (size_t)(ctx->learn_count % ctx->learn_cap) * 4 * n;
    in3 = *slot;
  } else {
    in3 = sgn_cnn_in3_buffer(ctx->learn_net);
  }
  HIPCK(sgn::launch_learn_pack(g, r0, mr0, h, n, ctx->st, in3, s));
  if (!use_net) return SGN_OK;
  float* out = sgn_cnn_out_buffer(ctx->learn_net);
  if (sgn_cnn_forward_on(ctx->learn_net, in3, out, s) != SGN_OK) {
    ctx->err = "learned guess: network forward pass failed";
    return SGN_ERR_HIP;
  }
  HIPCK(sgn::launch_learn_apply(g, sp, out, ctx->st, sg, n, s));
  return load_sigma(ctx, sg);
}

// After the solve: the recorder's target (sigma - sigma_prev) / |r0|.
int learned_finish(sgn_ctx* ctx, float* slot) {
  const sgn::Geom& g = ctx->g;
  const size_t n = (size_t)g.nx * g.ny;
  void* snew = ctx->ckpt + ctx->field_bytes;
  HIPCK(sgn::launch_row_c2r(g, ctx->E, snew, ctx->stream));
  HIPCK(sgn::launch_learn_target(g, snew, ctx->ckpt, ctx->st, slot + 3 * n, n, ctx->stream));
  ctx->learn_count += 1;
  return SGN_OK;
}

// ---- the captured RK4 step

// One RK4 step for capture: the solve of stage s is a single GMRES cycle of
// budget[s] Arnoldi steps, all predicated on the device status, with the
// device's iteration cap at budget[s] (so the device closes the cycle at
// convergence or there): the caller sets budget[0] before the first replay,
// and each solve's update kernel counts the solve and sets the cap of the
// next (stage 3's that of the next step's stage 0).  kind 0: first step of a call (sigma itself is
// the guess); kind 1: later steps (stage-increment guess, if on).
int enqueue_graph_step(sgn_ctx* ctx, int kind, void* h, void* vx, void* vy, double dt, const int* budget) {
  const sgn::Geom& g = ctx->g;
  hipStream_t s = ctx->stream;
  int rc;
  for (int stage = 0; stage < 4; ++stage) {
    const void* ih = stage == 0 ? h : ctx->hs;
    const void* ivx = stage == 0 ? vx : ctx->vxs;
    const void* ivy = stage == 0 ? vy : ctx->vys;
    void* Dst = ctx->D ? ctx->D + (size_t)stage * ctx->field_bytes : nullptr;
    if (Dst && kind == 1) HIPCK(sgn::launch_col_guess_eg(g, ctx->SIG, Dst, ctx->E, ctx->G, s));
    if ((rc = enqueue_residual(ctx, 1, ih, ivx, ivy, 1, 1))) return rc;
    for (int it = 0; it < budget[stage]; ++it)
      if ((rc = enqueue_arnoldi(ctx, ih, it))) return rc;
    HIPCK(sgn::launch_col_update_eg(g, ctx->SIG, ctx->V, ctx->vstride, ctx->st, ctx->E, ctx->G, Dst,
                                    4 | (budget[(stage + 1) & 3] << 16), s));
    if ((rc = enqueue_stage_flux(ctx, stage, dt, h, vx, vy, ih, ivx, ivy))) return rc;
  }
  return enqueue_step_filter(ctx, h, vx, vy);
}

// Instantiated graph of one step of this kind, captured on ctx->stream (the
// private stream) unless the cached one has the same fields, dt and budgets.
int graph_for(sgn_ctx* ctx, int kind, void* h, void* vx, void* vy, double dt, const int* budget) {
  sgn_ctx::GraphKey key;
  key.h = h;
  key.vx = vx;
  key.vy = vy;
  key.dt = dt;
  std::copy(budget, budget + 4, key.budget);
  key.arnoldi = ctx->arnoldi;
  key.tile_blocks = ctx->g.tile_blocks;
  key.row_threads = ctx->g.row_threads;
  if (ctx->gexec[kind] && ctx->gkey[kind] == key) return SGN_OK;
  if (ctx->gexec[kind]) {
    HIPCK(hipGraphExecDestroy(ctx->gexec[kind]));
    ctx->gexec[kind] = nullptr;
  }
  const int timed = ctx->timed_kind;  // no timing events inside a graph
  ctx->timed_kind = -1;
  HIPCK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed));
  ctx->g.status_first = ctx->graph_status_first;
  const int rc = enqueue_graph_step(ctx, kind, h, vx, vy, dt, budget);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(ctx->stream, &graph);
  ctx->timed_kind = timed;
  ctx->g.status_first = 0;
  if (rc || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc ? rc : fail(ctx, e, "hipStreamEndCapture");
  }
  hipGraphExec_t x = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&x, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) return fail(ctx, e2, "hipGraphInstantiate");
  ctx->gexec[kind] = x;
  ctx->gkey[kind] = key;
  return SGN_OK;
}

// Runs a captured call on the context's private stream, ordered after the
// work already on the caller's stream and before the work enqueued there
// later.
struct PrivateStream {
  sgn_ctx* ctx;
  hipStream_t user;
  bool ok = false;
  explicit PrivateStream(sgn_ctx* c) : ctx(c), user(c->stream) {
    if (!c->gstream) {
      if (hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess) {
        c->gstream = nullptr;
        return;
      }
      for (hipEvent_t& e : c->gev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return;
    }
    if (hipEventRecord(c->gev[0], user) != hipSuccess) return;
    if (hipStreamWaitEvent(c->gstream, c->gev[0], 0) != hipSuccess) return;
    c->stream = c->gstream;
    ok = true;
  }
  ~PrivateStream() {
    if (!ok) return;
    (void)hipEventRecord(ctx->gev[1], ctx->gstream);
    (void)hipStreamWaitEvent(user, ctx->gev[1], 0);
    ctx->stream = user;
  }
};

}  // namespace

extern "C" {

void sgn_config_default(sgn_config* cfg, int32_t nx, int32_t ny, double Lx, double Ly) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof *cfg);
  cfg->nx = nx;
  cfg->ny = ny;
  cfg->Lx = Lx;
  cfg->Ly = Ly;
  cfg->g = 1.0;
  cfg->h_inf = 1.0;
  cfg->precision = SGN_FP64;
  cfg->gmres_restart = 20;
  cfg->gmres_tol = 1e-10;
  cfg->gmres_max_iters = 200;
  cfg->batch = 1;
  cfg->krasny = 0.0;
  cfg->invariants_tol = 1e-13;
}

size_t sgn_workspace_bytes(const sgn_config* cfg) {
  if (check_config(cfg) != SGN_OK) return 0;
  return layout(cfg).total;
}

int sgn_init(const sgn_config* cfg, void* ws, size_t ws_bytes, void* hip_stream, sgn_ctx** out) {
  if (!out) return SGN_ERR_INVALID_ARG;
  *out = nullptr;
  int rc = check_config(cfg);
  if (rc) return rc;
  const Layout L = layout(cfg);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0 || ws_bytes < L.total) return SGN_ERR_INVALID_ARG;
  sgn_ctx* ctx = new sgn_ctx();
  ctx->cfg = *cfg;
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    return SGN_ERR_HIP;
  }
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  ctx->ws = static_cast<char*>(ws);
  ctx->ws_bytes = ws_bytes;
  for (int& li : ctx->last_iters) li = cfg->gmres_restart / 2;
  // SGN_ARNOLDI_KERNELS = fused | chained | serial selects the Arnoldi
  // kernels (a tuning and testing switch; all compute the same quantities)
  const char* ak = std::getenv("SGN_ARNOLDI_KERNELS");
  // default: the three-kernel step; for columns of 2048 points and more the
  // four-kernel step with one transform chain per block measured faster
  ctx->arnoldi = cfg->ny >= 2048 ? 0 : 2;
  if (ak && std::strcmp(ak, "fused") == 0) ctx->arnoldi = 2;
  if (ak && std::strcmp(ak, "chained") == 0) ctx->arnoldi = 1;
  if (ak && std::strcmp(ak, "serial") == 0) ctx->arnoldi = 0;
  const int nx = cfg->nx, ny = cfg->ny;
  sgn::Geom& g = ctx->g;
  sgn::geom_init(*cfg, g);
  // SGN_BATCH_MARGIN (0..4): Arnoldi steps enqueued beyond the previous
  // solve's count before the host reads the status
  if (const char* bm = std::getenv("SGN_BATCH_MARGIN")) {
    const int v = std::atoi(bm);
    if (v >= 0 && v <= 4) ctx->batch_margin = v;
  }
  // SGN_GRAPH_MARGIN (0..4): Arnoldi steps a captured solve runs beyond the
  // most its stage needed in the host-driven steps seen
  if (const char* gm = std::getenv("SGN_GRAPH_MARGIN")) {
    const int v = std::atoi(gm);
    if (v >= 0 && v <= 4) ctx->graph_margin = v;
  }
  if (const char* gs = std::getenv("SGN_GRAPH_STATUS_FIRST")) ctx->graph_status_first = std::atoi(gs) != 0;
  if (!sgn::chained_ok(g)) ctx->arnoldi = 0;
  char* base = ctx->ws;
  const int M = cfg->batch;
  g.members = M;
  // members test the GMRES status before their loads: members that have
  // converged skip the loads of the launches for the others' further steps
  // (SGN_MEMBER_STATUS_FIRST=0: after, as a single grid does)
  if (M > 1) {
    g.status_first = 1;
    if (const char* sf = std::getenv("SGN_MEMBER_STATUS_FIRST")) g.status_first = std::atoi(sf) != 0;
  }
  g.ws_lo = reinterpret_cast<uintptr_t>(base);
  g.ws_span = g.ws_stride = L.member;
  g.f_stride = (size_t)nx * ny * (g.fp32 ? sizeof(float) : sizeof(double));
  ctx->ws_stride = L.member;
  cplx* tw = reinterpret_cast<cplx*>(base + L.tw);
  float2* tw32 = reinterpret_cast<float2*>(base + L.tw + align_up((size_t)(nx + ny) * sizeof(double2)));
  g.twx = tw;
  g.twy = tw + nx;
  g.twx32 = tw32;
  g.twy32 = tw32 + nx;
  ctx->st = reinterpret_cast<sgn::GmresState*>(base + L.st);
  ctx->partials = reinterpret_cast<double*>(base + L.partials);
  ctx->partials2 = reinterpret_cast<double*>(base + L.partials2);
  ctx->field_bytes = L.field_bytes;
  ctx->vstride = L.field_bytes / (g.fp32 ? sizeof(float2) : sizeof(double2));
  char* f = base + L.fields;
  auto next = [&]() {
    char* p = f;
    f += L.field_bytes;
    return p;
  };
  ctx->V = f;
  f += (size_t)(cfg->gmres_restart + 1) * L.field_bytes;
  ctx->Z = f;
  f += L.field_bytes;
  ctx->W = next();
  ctx->E = next();
  ctx->G = next();
  ctx->P = next();
  ctx->Q = next();
  ctx->R1 = next();
  ctx->R2 = next();
  ctx->SIG = next();
  ctx->hs = next();
  ctx->vxs = next();
  ctx->vys = next();
  ctx->acc_h = next();
  ctx->acc_vx = next();
  ctx->acc_vy = next();
  ctx->ckpt = f;
  f += (size_t)ckpt_fields(cfg) * L.field_bytes;
  ctx->D = nullptr;
  if (cfg->guess == SGN_GUESS_STAGE_INCREMENT) {
    ctx->D = f;
    f += 4 * L.field_bytes;
  }

  // FP64 twiddles exp(-2 pi i k / n), from the symmetric angle to keep the
  // table accurate to a rounding of the exact value
  std::vector<cplx> htw((size_t)nx + ny);
  auto fill = [&](cplx* dst, int n) {
    for (int k = 0; k < n; ++k) {
      const double a = 2.0 * M_PI * (double)k / (double)n;
      dst[k] = make_double2(std::cos(a), -std::sin(a));
    }
  };
  fill(htw.data(), nx);
  fill(htw.data() + nx, ny);
  // the same tables rounded to FP32 for the mixed-precision kernels
  std::vector<float2> htw32(htw.size());
  for (size_t k = 0; k < htw.size(); ++k) htw32[k] = make_float2((float)htw[k].x, (float)htw[k].y);
  sgn::GmresState hst;
  std::memset(&hst, 0, sizeof hst);
  hst.tol = effective_tol(*cfg, cfg->gmres_tol);
  hst.m = cfg->gmres_restart;
  hst.maxit = cfg->gmres_max_iters;
  hipError_t e = hipMemcpyAsync(tw, htw.data(), htw.size() * sizeof(cplx), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(tw32, htw32.data(), htw32.size() * sizeof(float2), hipMemcpyHostToDevice, ctx->stream);
  for (int k = 0; k < M && e == hipSuccess; ++k)
    e = hipMemcpyAsync(base + (size_t)k * L.member + L.st, &hst, sizeof hst, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&ctx->hstat), (size_t)M * sizeof(sgn::GmresStatus), 0);
  if (e != hipSuccess) {
    delete ctx;
    return SGN_ERR_HIP;
  }
  *out = ctx;
  return SGN_OK;
}

int sgn_destroy(sgn_ctx* ctx) {
  if (!ctx) return SGN_ERR_INVALID_ARG;
  (void)drain_timing(ctx);
  for (hipEvent_t e : ctx->ev_free) (void)hipEventDestroy(e);
  for (hipGraphExec_t x : ctx->gexec)
    if (x) (void)hipGraphExecDestroy(x);
  for (hipEvent_t e : ctx->gev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
  if (ctx->stat_ev) (void)hipEventDestroy(ctx->stat_ev);
  if (ctx->hstat) (void)hipHostFree(ctx->hstat);
  delete ctx;
  return SGN_OK;
}

int sgn_elliptic_solve(sgn_ctx* ctx, const void* h, const void* b, void* sigma, sgn_solve_info* info) {
  if (!ctx || !aligned(h) || !aligned(b) || !aligned(sigma)) return SGN_ERR_INVALID_ARG;
  int rc = check_state(ctx, h, b, b);
  if (rc) return rc;
  rc = load_sigma(ctx, sigma);
  if (rc) return rc;
  std::vector<SolveResult> res(members(ctx));
  rc = run_solve(ctx, 2, h, b, nullptr, res.data());
  if (rc) return rc;
  HIPCK(sgn::launch_row_c2r(ctx->g, ctx->E, sigma, ctx->stream));
  if (info) {
    // ||b - L sigma|| from the final (E, G)
    HIPCK(sgn::launch_row_op(ctx->g, 2, ctx->E, ctx->G, h, b, nullptr, ctx->P, ctx->Q, ctx->R1, ctx->R2, 0, 0,
                             ctx->st, ctx->stream));
    HIPCK(sgn::launch_col_resid(ctx->g, ctx->P, ctx->Q, nullptr, nullptr, 0, 2, ctx->st, nullptr, ctx->partials,
                                nullptr, nullptr, ctx->stream));
    rc = read_status(ctx);
    if (rc) return rc;
    for (int k = 0; k < members(ctx); ++k) {
      info[k].iters = res[k].iters;
      info[k].restarts = res[k].restarts;
      info[k].converged = res[k].converged;
      info[k].rel_resid_precond = res[k].rel_resid;
      const double bn = ctx->hstat[k].bnorm;
      info[k].rel_resid_true = bn > 0 ? std::sqrt(ctx->hstat[k].true_resid2) / bn : 0.0;
    }
  } else {
    HIPCK(hipStreamSynchronize(ctx->stream));
  }
  return all_converged(res) ? SGN_OK : SGN_ERR_NOT_CONVERGED;
}

int sgn_elliptic_solve_refined(sgn_ctx* c64, sgn_ctx* c32, const double* h, const double* b, double* sigma,
                               double tol, int32_t max_rounds, sgn_refine_info* info) {
  if (!c64 || !c32 || c64 == c32 || !aligned(h) || !aligned(b) || !aligned(sigma) || !(tol > 0.0) ||
      !std::isfinite(tol) || max_rounds < 1)
    return SGN_ERR_INVALID_ARG;
  const sgn_config &a = c64->cfg, &q = c32->cfg;
  if (a.precision != SGN_FP64 || q.precision != SGN_FP32_MIXED || a.batch != 1 || q.batch != 1)
    return SGN_ERR_UNSUPPORTED;
  if (a.nx != q.nx || a.ny != q.ny || a.Lx != q.Lx || a.Ly != q.Ly || a.g != q.g || a.h_inf != q.h_inf ||
      c64->device != c32->device)
    return SGN_ERR_INVALID_ARG;
  sgn_ctx* ctx = c64;  // for HIPCK
  const size_t n = (size_t)a.nx * a.ny;
  const size_t fb = c64->field_bytes;  // >= 8 n bytes
  double* r64 = reinterpret_cast<double*>(c64->ckpt);
  float* h32 = reinterpret_cast<float*>(c64->ckpt + fb);
  float* r32 = reinterpret_cast<float*>(c64->ckpt + 2 * fb);
  float* d32 = reinterpret_cast<float*>(c64->ckpt + 3 * fb);
  hipStream_t s = c64->stream;
  int nb = (int)((n + 255) / 256);
  if (nb > 1024) nb = 1024;
  std::vector<double> hp(2 * (size_t)nb);
  HIPCK(sgn::launch_to_f32(h, h32, n, s));
  sgn_refine_info inf{};
  int rc = SGN_OK;
  for (int round = 0;; ++round) {
    // r = b - L sigma in FP64, and its norm
    if ((rc = sgn_apply_operator(c64, h, sigma, r64, 0))) return rc;
    HIPCK(sgn::launch_refine_resid(b, r64, r32, n, c64->partials, nb, s));
    HIPCK(hipMemcpyAsync(hp.data(), c64->partials, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    double rr = 0.0, bb = 0.0;
    for (int i = 0; i < nb; ++i) {
      rr += hp[2 * (size_t)i];
      bb += hp[2 * (size_t)i + 1];
    }
    const double rel = bb > 0.0 ? std::sqrt(rr / bb) : std::sqrt(rr);
    if (round == 0) inf.rel_resid_first = rel;
    inf.rel_resid_true = rel;
    if (rel <= tol) break;
    if (round == max_rounds) {
      rc = SGN_ERR_NOT_CONVERGED;
      break;
    }
    // L d = r in the mixed-precision mode, d from 0
    HIPCK(hipMemsetAsync(d32, 0, n * sizeof(float), s));
    HIPCK(hipStreamSynchronize(s));
    sgn_solve_info si{};
    const int rs = sgn_elliptic_solve(c32, h32, r32, d32, &si);
    if (rs != SGN_OK && rs != SGN_ERR_NOT_CONVERGED) return rs;
    inf.rounds += 1;
    inf.inner_iters += si.iters;
    HIPCK(sgn::launch_refine_update(sigma, d32, n, s));
  }
  if (info) *info = inf;
  return rc;
}

int sgn_rk4_step_refined(sgn_ctx* c64, sgn_ctx* c32, double* h, double* vx, double* vy, double* sigma, double dt,
                         int32_t nsteps, double tol, int32_t max_rounds, sgn_refined_step_info* info) {
  if (!c64 || !c32 || c64 == c32 || !aligned(h) || !aligned(vx) || !aligned(vy) || !aligned(sigma) || nsteps < 0 ||
      !std::isfinite(dt) || !(tol > 0.0) || !std::isfinite(tol) || max_rounds < 1)
    return SGN_ERR_INVALID_ARG;
  const sgn_config &a = c64->cfg, &q = c32->cfg;
  if (a.precision != SGN_FP64 || q.precision != SGN_FP32_MIXED || a.batch != 1 || q.batch != 1)
    return SGN_ERR_UNSUPPORTED;
  if (a.nx != q.nx || a.ny != q.ny || a.Lx != q.Lx || a.Ly != q.Ly || a.g != q.g || a.h_inf != q.h_inf ||
      c64->device != c32->device)
    return SGN_ERR_INVALID_ARG;
  if (c64->learn_net || c64->learn_rec) return SGN_ERR_UNSUPPORTED;
  sgn_ctx* ctx = c64;  // for HIPCK
  const sgn::Geom& g = c64->g;
  hipStream_t s = c64->stream;
  const size_t n = (size_t)g.nx * g.ny;
  int rc = check_state(c64, h, vx, vy);
  if (rc) return rc;
  // scratch in c64's Krylov basis, which this call never fills: the
  // divergence terms and b (V_0 .. V_2) and the warm-start chain of sigma (V_3)
  char* V = static_cast<char*>(c64->V);
  const size_t fb = c64->field_bytes;
  double* t1 = reinterpret_cast<double*>(V);
  double* t2 = reinterpret_cast<double*>(V + fb);
  double* b = reinterpret_cast<double*>(V + 2 * fb);
  double* sg = reinterpret_cast<double*>(V + 3 * fb);
  HIPCK(hipMemcpyAsync(sg, sigma, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  sgn_refined_step_info inf{};
  inf.max_rel_resid = 0.0;
  bool unconv = false;
  for (int step = 0; step < nsteps; ++step) {
    for (int stage = 0; stage < 4; ++stage) {
      const double* ih = stage == 0 ? h : static_cast<const double*>(c64->hs);
      const double* ivx = stage == 0 ? vx : static_cast<const double*>(c64->vxs);
      const double* ivy = stage == 0 ? vy : static_cast<const double*>(c64->vys);
      // b = -div v in FP64
      HIPCK(sgn::launch_row_dx(g, ivx, t1, s));
      HIPCK(sgn::launch_col_dy(g, ivy, t2, s));
      HIPCK(sgn::launch_neg_sum(t1, t2, b, n, s));
      // sigma from the previous stage's, refined to tol in the FP64 residual
      sgn_refine_info ri{};
      rc = sgn_elliptic_solve_refined(c64, c32, ih, b, sg, tol, max_rounds, &ri);
      if (rc && rc != SGN_ERR_NOT_CONVERGED) return rc;
      unconv = unconv || rc == SGN_ERR_NOT_CONVERGED;
      inf.solves += 1;
      inf.rounds += ri.rounds;
      inf.inner_iters += ri.inner_iters;
      inf.max_rounds_per_solve = std::max(inf.max_rounds_per_solve, ri.rounds);
      inf.max_rel_resid = std::max(inf.max_rel_resid, ri.rel_resid_true);
      // fluxes, Bernoulli function and the stage combine in FP64 from sigma
      if ((rc = load_sigma(c64, sg))) return rc;
      if ((rc = enqueue_stage_flux(c64, stage, dt, h, vx, vy, ih, ivx, ivy))) return rc;
    }
    if ((rc = enqueue_step_filter(c64, h, vx, vy))) return rc;
  }
  HIPCK(hipMemcpyAsync(sigma, sg, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCK(sgn::launch_field_stats(g, h, vx, vy, n, c64->st, c64->partials, s));
  if ((rc = read_status(c64))) return rc;
  inf.min_h = c64->hstat->stat_minh;
  if (info) *info = inf;
  if (c64->hstat->stat_nonfinite) return SGN_ERR_NONFINITE;
  if (!(c64->hstat->stat_minh > 0.0)) return SGN_ERR_CAVITATION;
  return unconv ? SGN_ERR_NOT_CONVERGED : SGN_OK;
}

int sgn_rhs(sgn_ctx* ctx, const void* h, const void* vx, const void* vy, void* sigma, void* dh, void* dvx,
            void* dvy, sgn_solve_info* info) {
  if (!ctx || !aligned(h) || !aligned(vx) || !aligned(vy) || !aligned(sigma) || !aligned(dh) || !aligned(dvx) ||
      !aligned(dvy))
    return SGN_ERR_INVALID_ARG;
  int rc = check_state(ctx, h, vx, vy);
  if (rc) return rc;
  rc = load_sigma(ctx, sigma);
  if (rc) return rc;
  std::vector<SolveResult> res(members(ctx));
  rc = run_solve(ctx, 1, h, vx, vy, res.data());
  if (rc) return rc;
  sgn::RkStage rk{0, 0, 0.0, 0.0, 0.0};
  void* dhp = ctx->P;
  void* qy = ctx->Q;
  void* B = ctx->R1;
  HIPCK(sgn::launch_row_flux(ctx->g, ctx->E, ctx->G, h, vx, vy, dhp, qy, B, rk, sgn::RkField{nullptr, nullptr, dvx},
                             ctx->stream));
  HIPCK(sgn::launch_col_flux(ctx->g, dhp, qy, B, rk, sgn::RkField{nullptr, nullptr, dh},
                             sgn::RkField{nullptr, nullptr, dvy}, ctx->stream));
  HIPCK(sgn::launch_row_c2r(ctx->g, ctx->E, sigma, ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));
  if (info) {
    for (int k = 0; k < members(ctx); ++k) {
      info[k].iters = res[k].iters;
      info[k].restarts = res[k].restarts;
      info[k].converged = res[k].converged;
      info[k].rel_resid_precond = res[k].rel_resid;
      info[k].rel_resid_true = -1.0;
    }
  }
  return all_converged(res) ? SGN_OK : SGN_ERR_NOT_CONVERGED;
}

namespace {

// Per-member totals of the steps of one call.
struct StepTally {
  std::vector<int64_t> total;
  std::vector<int> maxper, unconv;
  int solves = 0;
  explicit StepTally(int M) : total(M, 0), maxper(M, 0), unconv(M, 0) {}
};

// Steps [first, first + n) of a call, host-driven, continuing from the
// carried state as it stands (SIG, E, G and, with the stage-increment guess,
// D).  Records the most iterations of each stage in ctx->stage_max (member 0).
int rk4_host_steps(sgn_ctx* ctx, void* h, void* vx, void* vy, double dt, int first, int n, StepTally& t) {
  const sgn::Geom& g = ctx->g;
  hipStream_t s = ctx->stream;
  const int M = members(ctx);
  int rc;
  std::vector<SolveResult> res(M);
  for (int step = first; step < first + n; ++step) {
    for (int stage = 0; stage < 4; ++stage) {
      const void* ih = stage == 0 ? h : ctx->hs;
      const void* ivx = stage == 0 ? vx : ctx->vxs;
      const void* ivy = stage == 0 ? vy : ctx->vys;
      void* Dst = ctx->D ? ctx->D + (size_t)stage * ctx->field_bytes : nullptr;
      if (Dst && step > 0) HIPCK(sgn::launch_col_guess_eg(g, ctx->SIG, Dst, ctx->E, ctx->G, s));
      float* slot = nullptr;
      const bool use_net = ctx->learn_net && ((ctx->learn_stages >> stage) & 1);
      if ((use_net || ctx->learn_rec) && (rc = learned_start(ctx, ih, ivx, ivy, &slot, use_net))) return rc;
      // the stage's fluxes follow each batch of Arnoldi steps speculatively
      // (not with the learned guess, whose finish comes between, nor for
      // ensemble members, which finish their solves at different steps)
      const std::function<int(bool)> post = [&](bool spec) {
        return enqueue_stage_flux(ctx, stage, dt, h, vx, vy, ih, ivx, ivy, spec);
      };
      rc = run_solve(ctx, 1, ih, ivx, ivy, res.data(), stage, Dst, slot ? nullptr : &post);
      if (rc) return rc;
      if (slot && (rc = learned_finish(ctx, slot))) return rc;
      for (int k = 0; k < M; ++k) {
        t.total[k] += res[k].iters;
        t.maxper[k] = std::max(t.maxper[k], res[k].iters);
        t.unconv[k] |= !res[k].converged;
      }
      ctx->stage_max[stage] = std::max(ctx->stage_max[stage], res[0].iters);
      t.solves += 1;
      if (!res[0].post_done && (rc = enqueue_stage_flux(ctx, stage, dt, h, vx, vy, ih, ivx, ivy))) return rc;
    }
    if ((rc = enqueue_step_filter(ctx, h, vx, vy))) return rc;
  }
  return SGN_OK;
}

// The checkpoint of a chunk of captured steps (save) or its restoration:
// the caller's h, vx, vy and the carried solver state SIG, E, G (and D_0..D_3).
int chunk_checkpoint(sgn_ctx* ctx, void* h, void* vx, void* vy, bool save) {
  const sgn::Geom& g = ctx->g;
  const size_t nb = (size_t)g.nx * g.ny * (g.fp32 ? sizeof(float) : sizeof(double));
  std::vector<void*> f = {h, vx, vy, ctx->SIG, ctx->E, ctx->G};
  if (ctx->D)
    for (int k = 0; k < 4; ++k) f.push_back(ctx->D + (size_t)k * ctx->field_bytes);
  for (size_t i = 0; i < f.size(); ++i) {
    void* c = ctx->ckpt + i * ctx->field_bytes;
    HIPCK(hipMemcpyAsync(save ? c : f[i], save ? f[i] : c, nb, hipMemcpyDeviceToDevice, ctx->stream));
  }
  return SGN_OK;
}

// Status words, outputs and return code of a call of K steps.
int finish_call(sgn_ctx* ctx, void* h, void* vx, void* vy, void* sigma, const StepTally& t, sgn_step_info* info) {
  const sgn::Geom& g = ctx->g;
  const int M = members(ctx);
  HIPCK(sgn::launch_row_c2r(g, ctx->E, sigma, ctx->stream));
  HIPCK(sgn::launch_field_stats(g, h, vx, vy, (size_t)g.nx * g.ny, ctx->st, ctx->partials, ctx->stream));
  int rc = read_status(ctx);
  if (rc) return rc;
  bool any_unconv = false, nonfinite = false, cavit = false;
  for (int k = 0; k < M; ++k) {
    if (info) {
      info[k].total_iters = t.total[k];
      info[k].max_iters_per_solve = t.maxper[k];
      info[k].solves = t.solves;
      info[k].min_h = ctx->hstat[k].stat_minh;
      info[k].any_unconverged = t.unconv[k];
    }
    any_unconv = any_unconv || t.unconv[k];
    nonfinite = nonfinite || ctx->hstat[k].stat_nonfinite;
    cavit = cavit || !(ctx->hstat[k].stat_minh > 0.0);
  }
  if (nonfinite) return SGN_ERR_NONFINITE;
  if (cavit) return SGN_ERR_CAVITATION;
  return any_unconv ? SGN_ERR_NOT_CONVERGED : SGN_OK;
}

constexpr int kGraphChunk = 16;  // captured steps between status reads (and checkpoints)

}  // namespace

int sgn_rk4_step(sgn_ctx* ctx, void* h, void* vx, void* vy, void* sigma, double dt, int32_t nsteps,
                 sgn_step_info* info) {
  if (!ctx || !aligned(h) || !aligned(vx) || !aligned(vy) || !aligned(sigma) || nsteps < 0 || !std::isfinite(dt))
    return SGN_ERR_INVALID_ARG;
  int rc = check_state(ctx, h, vx, vy);
  if (rc) return rc;
  rc = load_sigma(ctx, sigma);
  if (rc) return rc;
  // stage-increment guess: the increments start at zero in every call, so the
  // first step starts each stage from the previous stage's sigma
  if ((rc = clear_guess(ctx))) return rc;
  StepTally t(members(ctx));
  if ((rc = rk4_host_steps(ctx, h, vx, vy, dt, 0, nsteps, t))) return rc;
  return finish_call(ctx, h, vx, vy, sigma, t, info);
}

// Captured steps: after a host-driven calibration step (automatic budgets),
// chunks of kGraphChunk graph replays, each from a checkpoint of the fields
// and the carried state, followed by one status read.  A chunk in which a
// solve needed more than its stage's budget is restored and redone
// host-driven (continuing exactly where the replays started, so the call ends
// bit for bit where sgn_rk4_step does), and the budgets grow to what the
// redone steps needed.
int sgn_rk4_step_graph(sgn_ctx* ctx, void* h, void* vx, void* vy, void* sigma, double dt, int32_t nsteps,
                       int32_t iter_budget, sgn_step_info* info, int32_t* replayed) {
  if (replayed) *replayed = 0;
  if (!ctx || !aligned(h) || !aligned(vx) || !aligned(vy) || !aligned(sigma) || nsteps < 0 || !std::isfinite(dt) ||
      iter_budget > ctx->cfg.gmres_restart)
    return SGN_ERR_INVALID_ARG;
  if (members(ctx) > 1) {
    ctx->err = "the captured step runs one grid per context (batch = 1)";
    return SGN_ERR_UNSUPPORTED;
  }
  if (nsteps == 0) return sgn_rk4_step(ctx, h, vx, vy, sigma, dt, 0, info);
  if (ctx->learn_net || ctx->learn_rec) {
    ctx->err = "the captured step does not run the learned guess";
    return SGN_ERR_UNSUPPORTED;
  }
  PrivateStream ps(ctx);
  if (!ps.ok) return fail(ctx, hipErrorInvalidValue, "private stream for the captured step");
  hipStream_t s = ctx->stream;
  int rc = check_state(ctx, h, vx, vy);
  if (rc) return rc;
  if ((rc = load_sigma(ctx, sigma))) return rc;
  if ((rc = clear_guess(ctx))) return rc;
  const int m = ctx->cfg.gmres_restart;
  const int cap = m < ctx->cfg.gmres_max_iters ? m : ctx->cfg.gmres_max_iters;
  const bool fixed = iter_budget > 0;
  StepTally t(1);
  int step = 0;
  int budget[4];
  auto from_stage_max = [&]() {
    for (int k = 0; k < 4; ++k) {
      const int b = std::min(std::max(ctx->stage_max[k] + ctx->graph_margin, 1), cap);
      ctx->graph_budgets[k] = std::max(ctx->graph_budgets[k], b);
    }
  };
  if (fixed) {
    for (int k = 0; k < 4; ++k) budget[k] = std::min(iter_budget, cap);
  } else {
    if (ctx->graph_budgets[0] <= 0) {
      // calibration: the first two steps host-driven (the second is the first
      // that starts from the stage-increment guess, if on)
      const int nc = std::min(nsteps, 2);
      std::fill(ctx->stage_max, ctx->stage_max + 4, 0);
      if ((rc = rk4_host_steps(ctx, h, vx, vy, dt, 0, nc, t))) return rc;
      from_stage_max();
      step = nc;
    }
    std::copy(ctx->graph_budgets, ctx->graph_budgets + 4, budget);
  }
  // solves that need restarts stay host-driven
  bool host_only = t.unconv[0] != 0;
  const bool two = ctx->D != nullptr;
  int32_t nrep = 0;
  while (step < nsteps) {
    const int n = std::min(kGraphChunk, nsteps - step);
    if (host_only) {
      if ((rc = rk4_host_steps(ctx, h, vx, vy, dt, step, nsteps - step, t))) return rc;
      break;
    }
    // with the stage-increment guess the first step of a call differs
    if ((!two || step == 0) && (rc = graph_for(ctx, 0, h, vx, vy, dt, budget))) return rc;
    if (two && step + n > 1 && (rc = graph_for(ctx, 1, h, vx, vy, dt, budget))) return rc;
    if ((rc = chunk_checkpoint(ctx, h, vx, vy, true))) return rc;
    HIPCK(hipMemsetAsync(&ctx->st->st.g_fail, 0, 2 * sizeof(int32_t) + sizeof(int64_t), s));
    if ((rc = set_state_scalar(ctx, &ctx->st->maxit, budget[0]))) return rc;
    for (int k = step; k < step + n; ++k) HIPCK(hipGraphLaunch(ctx->gexec[two && k > 0 ? 1 : 0], s));
    if ((rc = set_state_scalar(ctx, &ctx->st->maxit, ctx->cfg.gmres_max_iters))) return rc;
    if ((rc = read_status(ctx))) return rc;
    if (ctx->hstat->g_fail == 0) {
      t.total[0] += ctx->hstat->g_total;
      t.maxper[0] = std::max(t.maxper[0], (int)ctx->hstat->g_max);
      t.solves += 4 * n;
      nrep += n;
    } else {
      // a solve needed more than its budget: redo the chunk host-driven
      if ((rc = chunk_checkpoint(ctx, h, vx, vy, false))) return rc;
      std::fill(ctx->stage_max, ctx->stage_max + 4, 0);
      if ((rc = rk4_host_steps(ctx, h, vx, vy, dt, step, n, t))) return rc;
      host_only = t.unconv[0] != 0;
      if (!fixed) {
        from_stage_max();
        std::copy(ctx->graph_budgets, ctx->graph_budgets + 4, budget);
      }
    }
    step += n;
  }
  if (replayed) *replayed = nrep;
  return finish_call(ctx, h, vx, vy, sigma, t, info);
}

int sgn_learned_guess_attach(sgn_ctx* ctx, sgn_cnn* net, float* record, int32_t capacity) {
  if (!ctx || capacity < 0 || (record && capacity == 0) || (reinterpret_cast<uintptr_t>(record) & 15) != 0)
    return SGN_ERR_INVALID_ARG;
  if (net) {
    int H = 0, W = 0;
    sgn_cnn_grid(net, &H, &W);
    if (H != ctx->cfg.ny || W != ctx->cfg.nx) {
      ctx->err = "network grid differs from the solver grid";
      return SGN_ERR_INVALID_ARG;
    }
  }
  if ((net || record) && members(ctx) > 1) {
    ctx->err = "the learned guess runs one grid per context (batch = 1)";
    return SGN_ERR_UNSUPPORTED;
  }
  if ((net || record) && ctx->cfg.guess != SGN_GUESS_PREVIOUS) {
    ctx->err = "the learned guess replaces the warm start; it does not combine with the stage-increment guess";
    return SGN_ERR_UNSUPPORTED;
  }
  ctx->learn_net = net;
  ctx->learn_rec = record;
  ctx->learn_cap = record ? capacity : 0;
  ctx->learn_count = 0;
  return SGN_OK;
}

namespace {

// L_h applied to a physical FP64 field (the launches of sgn_apply_operator,
// without its synchronisation).  Scratch: E, R1, G, P, Q, W, R2.
int fg_apply_L(sgn_ctx* ctx, const void* h, const void* x, void* out) {
  const sgn::Geom& g = ctx->g;
  hipStream_t s = ctx->stream;
  HIPCK(sgn::launch_row_r2c(g, x, ctx->E, s));
  HIPCK(sgn::launch_col_fwd_eg(g, ctx->E, ctx->R1, ctx->G, s));
  HIPCK(sgn::launch_row_op(g, 0, ctx->E, ctx->G, h, nullptr, nullptr, ctx->P, ctx->Q, nullptr, nullptr, 0, 0, ctx->st,
                           s));
  HIPCK(sgn::launch_col_apply(g, ctx->P, ctx->Q, 0, ctx->W, s));
  HIPCK(sgn::launch_col_inv(g, ctx->W, ctx->R2, s));
  HIPCK(sgn::launch_row_c2r(g, ctx->R2, out, s));
  return SGN_OK;
}

// Inner products <V_k, w>, k < nv (fixed-order sums of the block partials).
int fg_dots(sgn_ctx* ctx, const double* V, size_t vstride, int nv, const double* w, double* out) {
  const size_t n = (size_t)ctx->g.nx * ctx->g.ny;
  const int nb = sgn::fg_blocks(n);
  HIPCK(sgn::launch_fg_dots(V, vstride, nv, w, n, ctx->partials2, ctx->stream));
  std::vector<double> part((size_t)nb * nv);
  HIPCK(hipMemcpyAsync(part.data(), ctx->partials2, part.size() * sizeof(double), hipMemcpyDeviceToHost,
                       ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < nv; ++k) {
    double a = 0.0;
    for (int bl = 0; bl < nb; ++bl) a += part[(size_t)bl * nv + k];
    out[k] = a;
  }
  return SGN_OK;
}

}  // namespace

int sgn_elliptic_solve_fgmres(sgn_ctx* ctx, sgn_cnn* net, const void* h, const void* b, void* sigma,
                              int32_t max_iters, sgn_fgmres_info* info) {
  if (!ctx || !net || !aligned(h) || !aligned(b) || !aligned(sigma) || max_iters < 0 || sigma == b || sigma == h)
    return SGN_ERR_INVALID_ARG;
  if (ctx->g.fp32 || members(ctx) > 1) {
    ctx->err = "the flexible GMRES solve runs FP64 contexts with batch = 1";
    return SGN_ERR_UNSUPPORTED;
  }
  int H = 0, W = 0;
  sgn_cnn_grid(net, &H, &W);
  if (H != ctx->cfg.ny || W != ctx->cfg.nx) {
    ctx->err = "network grid differs from the solver grid";
    return SGN_ERR_INVALID_ARG;
  }
  int rc = check_state(ctx, h, b, b);
  if (rc) return rc;
  const sgn::Geom& g = ctx->g;
  hipStream_t s = ctx->stream;
  const size_t n = (size_t)g.nx * g.ny;
  const size_t vs = ctx->field_bytes / sizeof(double);  // field stride in doubles
  const int m = std::min(ctx->cfg.gmres_restart / 2, sgn::kFgMaxVecs - 1);
  if (m < 1) {
    ctx->err = "the flexible GMRES solve needs gmres_restart >= 2";
    return SGN_ERR_UNSUPPORTED;
  }
  // V_0..V_m and Z_0..Z_{m-1} in the Krylov fields (restart + 1 >= 2 m + 1)
  double* V = static_cast<double*>(ctx->V);
  double* Z = V + (size_t)(m + 1) * vs;
  double* w = static_cast<double*>(ctx->Z);
  double* mr = static_cast<double*>(ctx->acc_h);
  double* zero = static_cast<double*>(ctx->acc_vx);
  double* lx = static_cast<double*>(ctx->acc_vy);
  double* sg = static_cast<double*>(sigma);
  const double* bb = static_cast<const double*>(b);
  HIPCK(hipMemsetAsync(zero, 0, n * sizeof(double), s));
  float* in3 = sgn_cnn_in3_buffer(net);
  float* nout = sgn_cnn_out_buffer(net);
  const sgn::FgCoefs none{};
  double bn2 = 0.0;
  if ((rc = fg_dots(ctx, bb, 0, 1, bb, &bn2))) return rc;
  const double bnorm = std::sqrt(bn2);
  const double tol = ctx->cfg.gmres_tol;
  int total = 0, cycles = 0;
  double rel = 0.0;
  bool stalled = false;
  std::vector<double> Hm((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), y(m);
  while (bnorm > 0.0) {
    // r = b - L sigma into V_0
    if ((rc = fg_apply_L(ctx, h, sg, lx))) return rc;
    HIPCK(sgn::launch_fg_combine(V, lx, -1.0, bb, 1.0, nullptr, 0, 0, none, n, s));
    double beta2 = 0.0;
    if ((rc = fg_dots(ctx, V, 0, 1, V, &beta2))) return rc;
    const double beta = std::sqrt(beta2);
    rel = beta / bnorm;
    if (rel <= tol || total >= max_iters || stalled) break;
    HIPCK(sgn::launch_fg_combine(V, V, 1.0 / beta, nullptr, 0.0, nullptr, 0, 0, none, n, s));
    std::fill(Hm.begin(), Hm.end(), 0.0);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int jd = 0;
    for (int j = 0; j < m && total < max_iters; ++j) {
      double* vj = V + (size_t)j * vs;
      double* zj = Z + (size_t)j * vs;
      // z_j = s net(v_j / s, M^-1 v_j / s, h - h_inf), s = RMS of v_j
      HIPCK(sgn::launch_learn_norm(g, vj, n, ctx->st, ctx->partials, s));
      HIPCK(sgn::launch_row_r2c(g, vj, ctx->E, s));
      HIPCK(sgn::launch_col_filter(g, ctx->E, 0, 0.0, ctx->P, s));
      HIPCK(sgn::launch_row_c2r(g, ctx->P, mr, s));
      HIPCK(sgn::launch_learn_pack(g, vj, mr, h, n, ctx->st, in3, s));
      if (sgn_cnn_forward_on(net, in3, nout, s) != SGN_OK) {
        ctx->err = "flexible GMRES: network forward pass failed";
        return SGN_ERR_HIP;
      }
      HIPCK(sgn::launch_learn_apply(g, zero, nout, ctx->st, zj, n, s));
      // w = L z_j, orthogonalised against V_0..V_j (two classical passes)
      if ((rc = fg_apply_L(ctx, h, zj, w))) return rc;
      double hc[sgn::kFgMaxVecs] = {}, h2[sgn::kFgMaxVecs];
      for (int pass = 0; pass < 2; ++pass) {
        if ((rc = fg_dots(ctx, V, vs, j + 1, w, h2))) return rc;
        sgn::FgCoefs c{};
        for (int i = 0; i <= j; ++i) {
          c.c[i] = -h2[i];
          hc[i] += h2[i];
        }
        HIPCK(sgn::launch_fg_combine(w, w, 1.0, nullptr, 0.0, V, vs, j + 1, c, n, s));
      }
      double hn2 = 0.0;
      if ((rc = fg_dots(ctx, w, 0, 1, w, &hn2))) return rc;
      const double hn = std::sqrt(hn2);
      total += 1;
      for (int i = 0; i <= j; ++i) Hm[(size_t)i * m + j] = hc[i];
      Hm[(size_t)(j + 1) * m + j] = hn;
      // Givens rotations of the column
      for (int i = 0; i < j; ++i) {
        const double a = Hm[(size_t)i * m + j], c2 = Hm[(size_t)(i + 1) * m + j];
        Hm[(size_t)i * m + j] = cs[i] * a + sn[i] * c2;
        Hm[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c2;
      }
      const double a = Hm[(size_t)j * m + j], c2 = Hm[(size_t)(j + 1) * m + j];
      const double r = std::hypot(a, c2);
      // a direction that adds nothing (zero network output): stop here
      if (!(r > 1e-14 * beta)) {
        stalled = true;
        break;
      }
      cs[j] = a / r;
      sn[j] = c2 / r;
      Hm[(size_t)j * m + j] = r;
      Hm[(size_t)(j + 1) * m + j] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      jd = j + 1;
      if (std::fabs(gv[j + 1]) <= tol * bnorm || !(hn > 0.0)) break;
      HIPCK(sgn::launch_fg_combine(V + (size_t)(j + 1) * vs, w, 1.0 / hn, nullptr, 0.0, nullptr, 0, 0, none, n, s));
    }
    if (jd > 0) {
      // sigma += Z y, R y = g
      for (int i = jd - 1; i >= 0; --i) {
        double t = gv[i];
        for (int k = i + 1; k < jd; ++k) t -= Hm[(size_t)i * m + k] * y[k];
        y[i] = t / Hm[(size_t)i * m + i];
      }
      sgn::FgCoefs c{};
      for (int i = 0; i < jd; ++i) c.c[i] = y[i];
      HIPCK(sgn::launch_fg_combine(sg, sg, 1.0, nullptr, 0.0, Z, vs, jd, c, n, s));
    }
    cycles += 1;
    if (jd == 0) break;
  }
  // plain GMRES from the result: the fallback and the judge
  sgn_solve_info ji{};
  const int jrc = sgn_elliptic_solve(ctx, h, b, sigma, &ji);
  if (jrc && jrc != SGN_ERR_NOT_CONVERGED) return jrc;
  if (info) {
    info->fgmres_iters = total;
    info->fgmres_cycles = cycles;
    info->gmres_iters = ji.iters;
    info->converged = ji.converged;
    info->fgmres_rel_resid = rel;
    info->rel_resid_true = ji.rel_resid_true;
  }
  return jrc;
}

int sgn_learned_guess_stages(sgn_ctx* ctx, int32_t stage_mask) {
  if (!ctx || stage_mask < 0 || stage_mask > 0xF) return SGN_ERR_INVALID_ARG;
  ctx->learn_stages = stage_mask;
  return SGN_OK;
}

int sgn_learned_guess_recorded(sgn_ctx* ctx, int64_t* count) {
  if (!ctx || !count) return SGN_ERR_INVALID_ARG;
  *count = ctx->learn_count;
  return SGN_OK;
}

int sgn_invariants(sgn_ctx* ctx, const void* h, const void* vx, const void* vy, void* sigma,
                   sgn_invariants_out* out) {
  if (!ctx || !out || !aligned(h) || !aligned(vx) || !aligned(vy) || !aligned(sigma)) return SGN_ERR_INVALID_ARG;
  int rc = check_state(ctx, h, vx, vy);
  if (rc) return rc;
  rc = set_tol(ctx, ctx->cfg.invariants_tol);
  if (rc) return rc;
  rc = load_sigma(ctx, sigma);
  std::vector<SolveResult> res(members(ctx));
  if (!rc) rc = run_solve(ctx, 1, h, vx, vy, res.data());
  const int rc2 = set_tol(ctx, ctx->cfg.gmres_tol);
  if (rc) return rc;
  if (rc2) return rc2;
  const sgn::Geom& g = ctx->g;
  void* dyvx = ctx->R2;
  HIPCK(sgn::launch_col_dy(g, vx, dyvx, ctx->stream));
  HIPCK(sgn::launch_row_invariants(g, ctx->E, ctx->G, h, vx, vy, dyvx, ctx->partials, ctx->st, ctx->stream));
  HIPCK(sgn::launch_row_r2c(g, h, ctx->P, ctx->stream));
  HIPCK(sgn::launch_col_tail(g, ctx->P, ctx->st, ctx->partials, ctx->stream));
  HIPCK(sgn::launch_row_c2r(g, ctx->E, sigma, ctx->stream));
  rc = read_status(ctx);
  if (rc) return rc;
  for (int k = 0; k < members(ctx); ++k) {
    const double* r = ctx->hstat[k].red;
    out[k].mass = r[0];
    out[k].px = r[1];
    out[k].py = r[2];
    out[k].energy = r[3];
    out[k].curl_l2 = r[4];
    out[k].min_h = r[5];
    out[k].max_h = r[6];
    out[k].spectral_tail = r[7];
  }
  return all_converged(res) ? SGN_OK : SGN_ERR_NOT_CONVERGED;
}

int sgn_derivative(sgn_ctx* ctx, int32_t axis, const void* f, void* out) {
  if (!ctx || !aligned(f) || !aligned(out) || f == out || (axis != 0 && axis != 1)) return SGN_ERR_INVALID_ARG;
  if (axis == 0)
    HIPCK(sgn::launch_row_dx(ctx->g, f, out, ctx->stream));
  else
    HIPCK(sgn::launch_col_dy(ctx->g, f, out, ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));
  return SGN_OK;
}

int sgn_apply_operator(sgn_ctx* ctx, const void* h, const void* s, void* out, int32_t precondition) {
  if (!ctx || !aligned(h) || !aligned(s) || !aligned(out) || out == s || out == h) return SGN_ERR_INVALID_ARG;
  const sgn::Geom& g = ctx->g;
  hipStream_t st = ctx->stream;
  HIPCK(sgn::launch_row_r2c(g, s, ctx->E, st));
  HIPCK(sgn::launch_col_fwd_eg(g, ctx->E, ctx->R1, ctx->G, st));
  HIPCK(sgn::launch_row_op(g, 0, ctx->E, ctx->G, h, nullptr, nullptr, ctx->P, ctx->Q, nullptr, nullptr, 0, 0, ctx->st,
                           st));
  HIPCK(sgn::launch_col_apply(g, ctx->P, ctx->Q, precondition ? 1 : 0, ctx->W, st));
  HIPCK(sgn::launch_col_inv(g, ctx->W, ctx->R2, st));
  HIPCK(sgn::launch_row_c2r(g, ctx->R2, out, st));
  HIPCK(hipStreamSynchronize(st));
  return SGN_OK;
}

int sgn_apply_precond(sgn_ctx* ctx, const void* r, void* out) {
  if (!ctx || !aligned(r) || !aligned(out) || out == r) return SGN_ERR_INVALID_ARG;
  const sgn::Geom& g = ctx->g;
  HIPCK(sgn::launch_row_r2c(g, r, ctx->E, ctx->stream));
  HIPCK(sgn::launch_col_filter(g, ctx->E, 0, 0.0, ctx->P, ctx->stream));
  HIPCK(sgn::launch_row_c2r(g, ctx->P, out, ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));
  return SGN_OK;
}

int sgn_krasny_filter(sgn_ctx* ctx, void* f) {
  if (!ctx || !aligned(f)) return SGN_ERR_INVALID_ARG;
  const sgn::Geom& g = ctx->g;
  HIPCK(sgn::launch_row_r2c(g, f, ctx->E, ctx->stream));
  HIPCK(sgn::launch_col_filter(g, ctx->E, step_filter_op(ctx->cfg), ctx->cfg.krasny, ctx->P, ctx->stream));
  HIPCK(sgn::launch_row_c2r(g, ctx->P, f, ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));
  return SGN_OK;
}

namespace {
// Members on host threads of their own; graphs: each member's steps as
// captured-graph replays (sgn_rk4_step_graph, automatic budget).
int run_ensemble(int32_t n, sgn_ctx* const* ctxs, void* const* h, void* const* vx, void* const* vy,
                 void* const* sigma, const double* dt, int32_t nsteps, sgn_step_info* infos, bool graphs) {
  if (n < 0 || (n > 0 && (!ctxs || !h || !vx || !vy || !sigma || !dt)) || nsteps < 0) return SGN_ERR_INVALID_ARG;
  // infos of context i: members(ctxs[i]) entries after those of the earlier contexts
  std::vector<int> off(n > 0 ? n : 1, 0);
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return SGN_ERR_INVALID_ARG;
    if (graphs && members(ctxs[i]) > 1) return SGN_ERR_UNSUPPORTED;  // the captured step runs single grids
    for (int k = 0; k < i; ++k)
      if (ctxs[k] == ctxs[i]) return SGN_ERR_INVALID_ARG;  // a context is not thread-safe
    if (i + 1 < n) off[i + 1] = off[i] + members(ctxs[i]);
  }
  std::vector<int> rc(n, SGN_OK);
  std::vector<std::thread> threads;
  threads.reserve(n);
  for (int i = 0; i < n; ++i) {
    threads.emplace_back([&, i]() {
      if (hipSetDevice(ctxs[i]->device) != hipSuccess) {
        rc[i] = SGN_ERR_HIP;
        return;
      }
      sgn_step_info* inf = infos ? &infos[off[i]] : nullptr;
      rc[i] = graphs ? sgn_rk4_step_graph(ctxs[i], h[i], vx[i], vy[i], sigma[i], dt[i], nsteps, 0, inf, nullptr)
                     : sgn_rk4_step(ctxs[i], h[i], vx[i], vy[i], sigma[i], dt[i], nsteps, inf);
    });
  }
  for (auto& t : threads) t.join();
  for (int i = 0; i < n; ++i)
    if (rc[i] != SGN_OK) return rc[i];
  return SGN_OK;
}
}  // namespace

int sgn_rk4_step_ensemble(int32_t n, sgn_ctx* const* ctxs, void* const* h, void* const* vx, void* const* vy,
                          void* const* sigma, const double* dt, int32_t nsteps, sgn_step_info* infos) {
  return run_ensemble(n, ctxs, h, vx, vy, sigma, dt, nsteps, infos, false);
}

int sgn_rk4_step_ensemble_graph(int32_t n, sgn_ctx* const* ctxs, void* const* h, void* const* vx, void* const* vy,
                                void* const* sigma, const double* dt, int32_t nsteps, sgn_step_info* infos) {
  return run_ensemble(n, ctxs, h, vx, vy, sigma, dt, nsteps, infos, true);
}

namespace {
std::mutex g_tune_mutex;
struct TuneChoice {
  int arnoldi, tile_blocks, row_threads;
  int row_radix = 0;  // values per thread of the members' two-chain row kernel (0: default)
};
// (nx, ny, precision, restart, members, device)
std::map<std::tuple<int, int, int, int, int, int>, TuneChoice> g_tune_cache;
}  // namespace

int sgn_autotune(sgn_ctx* ctx, int32_t* chosen) {
  if (!ctx) return SGN_ERR_INVALID_ARG;
  const sgn_config& c = ctx->cfg;
  const int M = members(ctx);
  const auto key = std::make_tuple(c.nx, c.ny, c.precision, c.gmres_restart, M, ctx->device);
  {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      ctx->arnoldi = it->second.arnoldi;
      ctx->g.tile_blocks = it->second.tile_blocks;
      ctx->g.row_threads = it->second.row_threads;
      ctx->g.row_radix = it->second.row_radix;
      if (chosen) *chosen = it->second.arnoldi;
      return SGN_OK;
    }
  }
  sgn::Geom& g = ctx->g;
  hipStream_t s = ctx->stream;
  // synthetic smooth problem in the workspace's RK4 stage buffers: depth
  // h = 1 + 0.3 sin(x) cos(2y), right-hand side b = cos(3x + y), zero guess
  const size_t npts = (size_t)c.nx * c.ny;
  std::vector<double> hh(npts), bb(npts);
  for (int y = 0; y < c.ny; ++y)
    for (int x = 0; x < c.nx; ++x) {
      const double X = -M_PI + 2.0 * M_PI * x / c.nx, Y = -M_PI + 2.0 * M_PI * y / c.ny;
      hh[(size_t)y * c.nx + x] = 1.0 + 0.3 * std::sin(X) * std::cos(2.0 * Y);
      bb[(size_t)y * c.nx + x] = std::cos(3.0 * X + Y);
    }
  // every member gets the same problem (its stage buffers, at the member stride)
  auto upload = [&](void* dst, const std::vector<double>& src) -> hipError_t {
    hipError_t e = hipSuccess;
    std::vector<float> f;
    if (g.fp32) f.assign(src.begin(), src.end());
    for (int k = 0; k < M && e == hipSuccess; ++k) {
      char* d = static_cast<char*>(dst) + (size_t)k * ctx->ws_stride;
      e = g.fp32 ? hipMemcpyAsync(d, f.data(), npts * sizeof(float), hipMemcpyHostToDevice, s)
                 : hipMemcpyAsync(d, src.data(), npts * sizeof(double), hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // f is a host local
    return e;
  };
  HIPCK(upload(ctx->hs, hh));
  HIPCK(upload(ctx->vxs, bb));
  if (M == 1)
    HIPCK(hipMemsetAsync(ctx->vys, 0, ctx->field_bytes, s));
  else
    HIPCK(hipMemset2DAsync(ctx->vys, ctx->ws_stride, 0, ctx->field_bytes, M, s));
  HIPCK(hipStreamSynchronize(s));
  hipEvent_t e0, e1;
  HIPCK(hipEventCreate(&e0));
  HIPCK(hipEventCreate(&e1));
  const TuneChoice saved{ctx->arnoldi, g.tile_blocks, g.row_threads, g.row_radix};
  int rc = SGN_OK;
  // time one candidate: three solves from zero after a warm-up solve
  auto time_it = [&](const TuneChoice& t, float* out) {
    ctx->arnoldi = t.arnoldi;
    g.tile_blocks = t.tile_blocks;
    g.row_threads = t.row_threads;
    g.row_radix = t.row_radix;
    float total = 0.0f;
    for (int rep = 0; rep < 4 && rc == SGN_OK; ++rep) {  // rep 0 warms up
      rc = load_sigma(ctx, ctx->vys);
      if (rc) break;
      if (hipEventRecord(e0, s) != hipSuccess) rc = SGN_ERR_HIP;
      std::vector<SolveResult> res(M);
      if (!rc) rc = run_solve(ctx, 2, ctx->hs, ctx->vxs, nullptr, res.data());
      if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = SGN_ERR_HIP;
      if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = SGN_ERR_HIP;
      float ms = 0.0f;
      if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = SGN_ERR_HIP;
      if (rep > 0) total += ms;
    }
    *out = total;
  };
  // 1. the Arnoldi schedules at the default launch shapes
  std::vector<int> sched = {0};
  if (sgn::chained_ok(g)) {
    sched.push_back(1);
    sched.push_back(2);
  }
  TuneChoice best = saved;
  float best_ms = 1e30f;
  for (int v : sched) {
    if (rc) break;
    const TuneChoice t{v, saved.tile_blocks, saved.row_threads, saved.row_radix};
    float ms;
    time_it(t, &ms);
    if (!rc && ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  // 2. for that schedule, the column tile widths and rows per row block that
  // give launch shapes not yet timed
  std::vector<std::array<int, 4>> seen;
  auto shape_of = [&](const TuneChoice& t) {
    sgn::Geom q = g;
    q.tile_blocks = t.tile_blocks;
    q.row_threads = t.row_threads;
    std::array<int, 4> a{};
    sgn::launch_shape(q, a.data());
    return a;
  };
  seen.push_back(shape_of(best));
  const TuneChoice base = best;
  for (int tb : {128, 256, 512, 1024}) {
    for (int rt : {64, 128, 256}) {
      if (rc) break;
      const TuneChoice t{base.arnoldi, tb, rt, base.row_radix};
      const auto a = shape_of(t);
      if (std::find(seen.begin(), seen.end(), a) != seen.end()) continue;
      seen.push_back(a);
      float ms;
      time_it(t, &ms);
      if (!rc && ms < best_ms) {
        best_ms = ms;
        best = t;
      }
    }
  }
  // 3. with several members on the three-kernel step, the radix of the
  // two-chain row kernel's transforms (4 or 8 values per thread)
  if (!rc && M > 1 && best.arnoldi == 2 && g.row_split && (c.nx == 512 || c.nx == 1024)) {
    for (int rr : {0, 8}) {
      if (rc || rr == best.row_radix) continue;
      TuneChoice t = best;
      t.row_radix = rr;
      float ms;
      time_it(t, &ms);
      if (!rc && ms < best_ms) {
        best_ms = ms;
        best = t;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const TuneChoice use = rc ? saved : best;
  ctx->arnoldi = use.arnoldi;
  g.tile_blocks = use.tile_blocks;
  g.row_threads = use.row_threads;
  g.row_radix = use.row_radix;
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_cache[key] = best;
  }
  if (chosen) *chosen = best.arnoldi;
  return SGN_OK;
}

int sgn_launch_shape(const sgn_ctx* ctx, int32_t* out) {
  if (!ctx || !out) return SGN_ERR_INVALID_ARG;
  int a[4];
  sgn::launch_shape(ctx->g, a);
  out[0] = ctx->arnoldi;
  out[1] = ctx->g.tile_blocks;
  out[2] = ctx->g.row_threads;
  for (int i = 0; i < 4; ++i) out[3 + i] = a[i];
  out[7] = ctx->g.row_radix;
  return SGN_OK;
}

int sgn_kernel_timing(sgn_ctx* ctx, int32_t kind, int32_t enable) {
  if (!ctx || kind < 0 || kind >= SGN_KERNEL_COUNT) return SGN_ERR_INVALID_ARG;
  int rc = drain_timing(ctx);
  if (rc) return rc;
  if (enable < 0) return SGN_ERR_INVALID_ARG;
  if (enable) {
    ctx->timed_kind = kind;
    ctx->timed_launches = 0;
    ctx->timed_all = 0;
    ctx->timed_period = enable;
    ctx->timed_ms = 0.0;
    ctx->timed_bytes = 0.0;
    // create the events now so that the timed launches make no runtime
    // allocation calls (they would stall the host and starve the GPU)
    while (ctx->ev_free.size() < 2 * 4096) {
      hipEvent_t e = nullptr;
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return fail(ctx, hipErrorOutOfMemory, "hipEventCreate");
      ctx->ev_free.push_back(e);
    }
  } else if (ctx->timed_kind == kind) {
    ctx->timed_kind = -1;
  }
  return SGN_OK;
}

int sgn_kernel_time(sgn_ctx* ctx, int32_t kind, int64_t* launches, double* total_ms, double* algo_bytes) {
  if (!ctx || !launches || !total_ms || kind < 0 || kind >= SGN_KERNEL_COUNT) return SGN_ERR_INVALID_ARG;
  int rc = drain_timing(ctx);
  if (rc) return rc;
  const bool mine = ctx->timed_kind == kind;
  // with sampling, the summed duration is scaled from the launches that
  // carried events to all launches of the class
  *launches = mine ? ctx->timed_all : 0;
  *total_ms = mine && ctx->timed_launches > 0
                  ? ctx->timed_ms * (double)ctx->timed_all / (double)ctx->timed_launches
                  : 0.0;
  if (algo_bytes) *algo_bytes = mine ? ctx->timed_bytes : 0.0;
  return SGN_OK;
}

const char* sgn_status_string(int status) {
  switch (status) {
    case SGN_OK: return "ok";
    case SGN_ERR_INVALID_ARG: return "invalid argument";
    case SGN_ERR_UNSUPPORTED: return "unsupported configuration";
    case SGN_ERR_HIP: return "HIP runtime error";
    case SGN_ERR_NOT_CONVERGED: return "GMRES did not converge";
    case SGN_ERR_CAVITATION: return "cavitation (min h <= 0)";
    case SGN_ERR_NONFINITE: return "non-finite value";
    default: return "unknown status";
  }
}

const char* sgn_last_error(const sgn_ctx* ctx) { return ctx ? ctx->err.c_str() : sgn::global_error(); }

}  // extern "C"

// Internal definitions shared by the kernels and the host runtime of libsgn.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace sgn {

constexpr int kMaxRestart = 64;     // largest GMRES restart length m
constexpr int kPartialStride = 136;  // doubles per block in the reduction scratch (>= 2 (m_max + 1))
constexpr int kMaxPartialBlocks = 4096;

// Grid geometry and spectral constants, passed by value to every kernel.
struct Geom {
  int nx, ny, nh;          // nh = nx / 2 complex columns of a half spectrum
  double inv_Lx, inv_Ly;   // wavenumber k = m / L
  double inv_nx, inv_ny, inv_n;
  double g, h_inf;
  double m0, m1;           // preconditioner symbol M = m0 + m1 (kx^2 + ky^2)
  double dA;               // cell area dx * dy
  const double2* twx;      // exp(-2 pi i k / nx), k < nx
  const double2* twy;      // exp(-2 pi i k / ny), k < ny
  const float2* twx32;     // the same tables rounded to FP32 (mixed-precision mode)
  const float2* twy32;
  int fp32;                // 1: fields, spectra and transforms in FP32; reductions stay FP64
  int m;                   // GMRES restart length (sizes the back-substitution scratch)
  int tile_blocks;         // column passes: the widest tiles that still give this many blocks (256)
  int row_threads;         // row passes: row pairs per block for at least this many threads (64)
  int status_first;        // 1: kernels test the GMRES status before their loads (captured graphs,
                           // whose fixed budgets launch many steps after convergence); 0: after
  // ensemble members of one context, one per blockIdx.z of every launch:
  // member m's workspace is member 0's [ws_lo, ws_lo + ws_span) moved by
  // m * ws_stride bytes, its caller fields are member 0's moved by m * f_stride
  int members;             // 1 for a single grid
  int row_split;           // 1: with several members, the Arnoldi row kernel in blocks of two chains
  int row_radix;           // that kernel's values per thread: 0 the engine's default, 8 radix-8 (512, 1024 points)
  uintptr_t ws_lo;
  size_t ws_span, ws_stride, f_stride;
};

// GMRES state kept in device memory.  Written only by the single "last
// block" of the reduction kernels; read by the following kernels and,
// through GmresStatus, by the host.
struct GmresStatus {
  int32_t done;         // 0 running, 1 converged, 2 cycle full (restart), 3 iteration cap
  int32_t jdone;        // Arnoldi steps completed in the current cycle
  int32_t total_iters;  // Arnoldi steps over the whole solve
  int32_t zero;         // b == 0: the solution is exactly 0
  double resid;         // current |g_{j+1}| (preconditioned residual estimate)
  double beta0;         // ||M^-1 b||
  double bnorm;         // ||b||
  double true_resid2;   // ||b - L x||^2 when requested
  double red[8];        // invariants: mass, Px, Py, energy, |curl v|, min h, max h, tail
  double stat_minh;     // min h of the last field check
  int32_t stat_nonfinite;
  int32_t cyc;          // host round of the current GMRES cycle (set by the residual pass)
  // solves of a captured RK4 step (one GMRES cycle each, no host reads):
  int32_t g_fail;   // solves that stopped at the iteration budget unconverged
  int32_t g_max;    // largest Arnoldi step count of one solve
  int64_t g_total;  // Arnoldi steps summed over the solves
};

struct GmresState {
  GmresStatus st;
  double tol;
  int32_t m;            // restart length
  int32_t maxit;        // total Arnoldi steps allowed per solve
  double beta;          // norm of the newest (not yet normalised) Krylov vector
  int32_t cycle_base;   // Arnoldi steps of the solve before the current cycle
  int32_t pad2;
  double learn_scale;   // learned guess: RMS of the warm start's residual r0
  double H[(kMaxRestart + 1) * kMaxRestart];  // H[i + j*(m_max+1)]
  double cs[kMaxRestart], sn[kMaxRestart];
  double gv[kMaxRestart + 1];  // g_j before rotation j (written when step j - 1 finishes)
  double gr[kMaxRestart];      // g_j after rotation j
  double y[kMaxRestart];
  double s[kMaxRestart + 1];   // first projection coefficients
  double s2[kMaxRestart + 1];  // second projection coefficients
  double cproj[kMaxRestart + 1];  // Gram-corrected projection coefficients (2I - G) s
  double G[(kMaxRestart + 1) * (kMaxRestart + 1)];  // Gram matrix <V_i, V_k> of the cycle
  // last-block ticket counters: [0] over groups, [32 (1 + g)] within group g
  // of kTicketGroup blocks (one 128-byte line each); reset by their last user
  uint32_t ctr[32 * (1 + kMaxPartialBlocks / 16)];
};

constexpr int kTicketGroup = 16;

__host__ __device__ inline int hidx(int i, int j) { return i + j * (kMaxRestart + 1); }

// One RK4 stage combine, fused into the flux passes.
//   mode 0: write k (the right-hand side) to `out`
//   mode 1: acc = (first ? 0 : acc) + wacc k; out = yn + cnext k
//   mode 2 (last stage): yn = yn + dt (acc + wacc k)
struct RkStage {
  int mode;
  int first;
  double wacc;
  double cnext;
  double dt;
  // non-null: a launch enqueued before the host knew that the solve had
  // converged; the kernel does nothing unless pred->done == 1
  const GmresStatus* pred = nullptr;
};

// Up to three independent fields for one launch of a pass (blockIdx.y picks
// one): in[i] is read, out[i] written.
struct Trio {
  const void* in[3];
  void* out[3];
};

// Field pointers of the working precision (double or float arrays).
struct RkField {
  const void* yn;   // state at the start of the step
  void* acc;        // accumulator of weighted stage derivatives
  void* out;        // next stage input (mode 1), k (mode 0) or yn itself (mode 2)
};

}  // namespace sgn

// Host-side launchers of the SGN kernels.
//
// The kernels are compiled once per precision (sgn_kernels.hip with
// SGN_PREC=64 into namespace sgn::p64, with SGN_PREC=32 into sgn::p32); the
// launchers of namespace sgn dispatch on Geom::fp32.  Field and spectrum
// pointers are untyped: FP64 arrays (double, double2) in FP64 mode, FP32
// arrays (float, float2) in the mixed-precision mode.  Reduction scratch and
// the GMRES state are FP64 in both.
#pragma once
#include "sgn_internal.hpp"

// X(name, parameter list, argument list)
#define SGN_LAUNCHERS(X)                                                                                        \
  X(row_r2c, (const Geom& g, const void* f, void* S, hipStream_t s), (g, f, S, s))                             \
  X(row_c2r, (const Geom& g, const void* S, void* f, hipStream_t s), (g, S, f, s))                             \
  X(row_r2c3, (const Geom& g, Trio io, hipStream_t s), (g, io, s))                                              \
  X(row_c2r3, (const Geom& g, Trio io, hipStream_t s), (g, io, s))                                              \
  X(col_filter3, (const Geom& g, Trio io, int op, double thr, hipStream_t s), (g, io, op, thr, s))              \
  X(row_dx, (const Geom& g, const void* f, void* o, hipStream_t s), (g, f, o, s))                              \
  X(row_op,                                                                                                     \
    (const Geom& g, int mode, const void* E, const void* G, const void* h, const void* vx, const void* vy,      \
     void* P, void* Q, void* R1, void* R2, int need_b, int pred, const GmresState* st, hipStream_t s),           \
    (g, mode, E, G, h, vx, vy, P, Q, R1, R2, need_b, pred, st, s))                                              \
  X(row_flux,                                                                                                   \
    (const Geom& g, const void* E, const void* G, const void* h, const void* vx, const void* vy, void* dhp,     \
     void* qy, void* B, RkStage rk, RkField fvx, hipStream_t s),                                                \
    (g, E, G, h, vx, vy, dhp, qy, B, rk, fvx, s))                                                               \
  X(row_invariants,                                                                                             \
    (const Geom& g, const void* E, const void* G, const void* h, const void* vx, const void* vy,                \
     const void* dyvx, double* partials, GmresState* st, hipStream_t s),                                        \
    (g, E, G, h, vx, vy, dyvx, partials, st, s))                                                                \
  X(row_matvec3,                                                                                                \
    (const Geom& g, const void* E, const void* G, const void* h, void* P, void* Q, const GmresState* st,        \
     hipStream_t s),                                                                                            \
    (g, E, G, h, P, Q, st, s))                                                                                  \
  X(col_fwd_eg, (const Geom& g, const void* Ein, void* SIG, void* Go, hipStream_t s), (g, Ein, SIG, Go, s))    \
  X(col_basis_eg,                                                                                               \
    (const Geom& g, const void* W, void* V, size_t vs, int j, GmresState* st, void* Eo, void* Go,               \
     const double* pin, hipStream_t s),                                                                         \
    (g, W, V, vs, j, st, Eo, Go, pin, s))                                                                       \
  X(col_basis2,                                                                                                 \
    (const Geom& g, const void* W, void* V, size_t vs, int j, GmresState* st, void* Eo, void* Go,               \
     const double* pin, hipStream_t s),                                                                         \
    (g, W, V, vs, j, st, Eo, Go, pin, s))                                                                       \
  X(col_update_eg,                                                                                              \
    (const Geom& g, void* SIG, const void* V, size_t vs, GmresState* st, void* Eo, void* Go, void* D,           \
     int spec, hipStream_t s),                                                                                  \
    (g, SIG, V, vs, st, Eo, Go, D, spec, s))                                                                    \
  X(col_guess_eg, (const Geom& g, void* SIG, const void* D, void* Eo, void* Go, hipStream_t s),                \
    (g, SIG, D, Eo, Go, s))                                                                                     \
  X(col_precond_dot,                                                                                            \
    (const Geom& g, const void* P, const void* Q, const void* V, size_t vs, int j, GmresState* st, void* W,     \
     double* partials, hipStream_t s),                                                                          \
    (g, P, Q, V, vs, j, st, W, partials, s))                                                                    \
  X(col_precond_dot2,                                                                                           \
    (const Geom& g, const void* P, const void* Q, const void* V, size_t vs, int j, GmresState* st, void* W,     \
     double* partials, hipStream_t s),                                                                          \
    (g, P, Q, V, vs, j, st, W, partials, s))                                                                    \
  X(col_proj,                                                                                                   \
    (const Geom& g, const void* win, void* W, const void* V, size_t vs, int j, GmresState* st, void* Eo,        \
     void* Go, const double* pin, hipStream_t s),                                                               \
    (g, win, W, V, vs, j, st, Eo, Go, pin, s))                                                                  \
  X(col_precond_new,                                                                                            \
    (const Geom& g, const void* P, const void* Q, const void* W, void* V, void* Z, size_t vs, int j,            \
     GmresState* st, double* partials, hipStream_t s),                                                          \
    (g, P, Q, W, V, Z, vs, j, st, partials, s))                                                                 \
  X(col_resid,                                                                                                  \
    (const Geom& g, const void* P, const void* Q, const void* R1, const void* R2, int need_b, int flags,        \
     GmresState* st, void* W, double* partials, void* Eo, void* Go, hipStream_t s),                             \
    (g, P, Q, R1, R2, need_b, flags, st, W, partials, Eo, Go, s))                                               \
  X(col_inv, (const Geom& g, const void* S, void* o, hipStream_t s), (g, S, o, s))                             \
  X(col_apply, (const Geom& g, const void* P, const void* Q, int precond, void* o, hipStream_t s),             \
    (g, P, Q, precond, o, s))                                                                                   \
  X(col_filter, (const Geom& g, const void* Sx, int op, double thr, void* o, hipStream_t s),                   \
    (g, Sx, op, thr, o, s))                                                                                     \
  X(col_tail, (const Geom& g, const void* Sx, GmresState* st, double* partials, hipStream_t s),                 \
    (g, Sx, st, partials, s))                                                                                   \
  X(col_dy, (const Geom& g, const void* f, void* o, hipStream_t s), (g, f, o, s))                              \
  X(col_flux,                                                                                                   \
    (const Geom& g, const void* dhp, const void* qy, const void* B, RkStage rk, RkField fh, RkField fvy,        \
     hipStream_t s),                                                                                            \
    (g, dhp, qy, B, rk, fh, fvy, s))                                                                            \
  X(upd, (const Geom& g, void* W, const void* V, size_t vs, int j, GmresState* st, double* partials,           \
          const double* pin, int chained, hipStream_t s),                                                       \
    (g, W, V, vs, j, st, partials, pin, chained, s))                                                            \
  X(col_learn, (const Geom& g, const void* W, void* out_r, void* out_m, hipStream_t s), (g, W, out_r, out_m, s))   \
  X(learn_norm, (const Geom& g, const void* r0, size_t n, GmresState* st, double* partials, hipStream_t s),       \
    (g, r0, n, st, partials, s))                                                                                \
  X(learn_pack,                                                                                                 \
    (const Geom& g, const void* r0, const void* mr0, const void* h, size_t n, const GmresState* st, float* in3, \
     hipStream_t s),                                                                                            \
    (g, r0, mr0, h, n, st, in3, s))                                                                             \
  X(learn_apply,                                                                                                \
    (const Geom& g, const void* sig_prev, const float* out, const GmresState* st, void* sig_guess, size_t n,    \
     hipStream_t s),                                                                                            \
    (g, sig_prev, out, st, sig_guess, n, s))                                                                    \
  X(learn_target,                                                                                               \
    (const Geom& g, const void* sig_new, const void* sig_prev, const GmresState* st, float* target, size_t n,   \
     hipStream_t s),                                                                                            \
    (g, sig_new, sig_prev, st, target, n, s))                                                                   \
  X(field_stats,                                                                                                \
    (const Geom& g, const void* h, const void* vx, const void* vy, size_t n, GmresState* st, double* partials,  \
     hipStream_t s),                                                                                            \
    (g, h, vx, vy, n, st, partials, s))

// Meaning of the launchers (all stream-ordered; none allocates):
//   row_r2c / row_c2r: physical <-> x-half spectra; row_dx: d/dx;
//   row_op: x part of the elliptic operator (mode 0), or of the residual with
//     b = -div v (mode 1) or an explicit b (mode 2);
//   row_matvec3: mode 0 of row_op with three concurrent transform chains;
//     with pin (three-kernel step jb) every block first finishes step jb - 1
//     from the block partials kernel A left in pin;
//   row_flux / col_flux: fluxes, Bernoulli function and the RK4 combine;
//   row_invariants / col_tail: invariant densities and the spectral tail;
//   col_fwd_eg: sigma's 2D spectrum and the inverse y-transforms E, G;
//   col_basis_eg / col_basis2 / col_precond_dot / col_precond_dot2 / upd: the
//     four-kernel Arnoldi step (one- and two-chain variants); upd reduces the
//     projection kernel's partials (pin; chained: which variant wrote them)
//     and the basis kernel of step j + 1 finishes step j from upd's;
//   col_proj / col_precond_new (with row_matvec3): the three-kernel step; each
//     leaves block partials that the next kernel of the step reduces (col_proj
//     reads those of col_precond_new from pin, so the two need distinct
//     partials buffers);
//   col_update_eg: sigma_hat += V y (and the guess increment D; in captured
//     steps also the solve counters and the next solve's iteration cap);
//   col_guess_eg: sigma_hat += D; col_resid: start of a GMRES cycle;
//   col_inv / col_apply / col_filter / col_dy: building blocks;
//   col_learn / learn_norm / learn_pack / learn_apply / learn_target: the
//     learned guess (r0 and M^-1 r0 from the GMRES start, their scale, the
//     network input, the corrected sigma, the training target);
//   field_stats: min h and a non-finite flag over the state.

namespace sgn {

#define SGN_DECLARE_LAUNCHER(name, params, args) hipError_t launch_##name params;
SGN_LAUNCHERS(SGN_DECLARE_LAUNCHER)

// Iterative refinement passes (sgn_refine.hip; FP64 residuals, FP32
// corrections): out = (float) in; r = b - r with r32 = (float) r and per-block
// partials (sum r^2, sum b^2) in partials[2 block], nblocks <= 1024;
// sigma += (double) d.
hipError_t launch_to_f32(const double* in, float* out, size_t n, hipStream_t s);
hipError_t launch_refine_resid(const double* b, double* r, float* r32, size_t n, double* partials, int nblocks,
                               hipStream_t s);
hipError_t launch_refine_update(double* sigma, const float* d, size_t n, hipStream_t s);
// out = -(a + c), n points (FP64).
hipError_t launch_neg_sum(const double* a, const double* c, double* out, size_t n, hipStream_t s);

// Flexible GMRES vector work (FP64 physical fields, n points): block partials
// of the inner products of w with V_0..V_{nv-1} (fields vstride doubles apart)
// into partials[block * nv + k] over fg_blocks(n) blocks; and
// out = a y + bx x + sum_k c_k V_k (y, x may be null; out may alias y).
constexpr int kFgMaxVecs = 16;  // basis fields per call (restart + 1 at most)
constexpr int kFgBlocks = 512;
struct FgCoefs {
  double c[kFgMaxVecs];
};
int fg_blocks(size_t n);
hipError_t launch_fg_dots(const double* V, size_t vstride, int nv, const double* w, size_t n, double* partials,
                          hipStream_t s);
hipError_t launch_fg_combine(double* out, const double* y, double a, const double* x, double bx, const double* V,
                             size_t vstride, int nv, const FgCoefs& c, size_t n, hipStream_t s);

// Largest number of blocks any reduction kernel launches for this grid.
int max_partial_blocks(const Geom& g);
// Whether this grid can use the chain-parallel Arnoldi passes.
bool chained_ok(const Geom& g);
// Launch shape of the grid's passes: row pairs per block of the single-chain
// and three-chain row kernels, columns per tile of the single-chain and
// two-chain column kernels (0: no such kernel for this size).
void launch_shape(const Geom& g, int* out4);
// The next kernel launch records these events at its start and end (null: none).
void set_launch_events(hipEvent_t start, hipEvent_t stop);
// Events for the next launch (consumed by it); shared by both precisions.
extern thread_local hipEvent_t t_ev_start, t_ev_stop;
// Ensemble members of the launch being dispatched (gridDim.z).
extern thread_local unsigned t_members;

namespace p64 {
SGN_LAUNCHERS(SGN_DECLARE_LAUNCHER)
int max_partial_blocks(const Geom& g);
bool chained_ok(const Geom& g);
void launch_shape(const Geom& g, int* out4);
}  // namespace p64
namespace p32 {
SGN_LAUNCHERS(SGN_DECLARE_LAUNCHER)
int max_partial_blocks(const Geom& g);
bool chained_ok(const Geom& g);
void launch_shape(const Geom& g, int* out4);
}  // namespace p32

}  // namespace sgn

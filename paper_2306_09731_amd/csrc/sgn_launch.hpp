// Host-side launchers of the SGN kernels (defined in sgn_kernels.hip).
#pragma once
#include "sgn_internal.hpp"

namespace sgn {

typedef double2 cplx;

hipError_t launch_row_r2c(const Geom& g, const double* f, cplx* S, hipStream_t s);
hipError_t launch_row_c2r(const Geom& g, const cplx* S, double* f, hipStream_t s);
hipError_t launch_row_dx(const Geom& g, const double* f, double* o, hipStream_t s);
hipError_t launch_row_op(const Geom& g, int mode, const cplx* E, const cplx* G, const double* h, const double* vx,
                         const double* vy, cplx* P, cplx* Q, cplx* R1, cplx* R2, int need_b, int pred,
                         const GmresState* st, hipStream_t s);
hipError_t launch_row_flux(const Geom& g, const cplx* E, const cplx* G, const double* h, const double* vx,
                           const double* vy, double* dhp, double* qy, double* B, RkStage rk, RkField fvx,
                           hipStream_t s);
hipError_t launch_row_invariants(const Geom& g, const cplx* E, const cplx* G, const double* h, const double* vx,
                                 const double* vy, const double* dyvx, double* partials, GmresState* st,
                                 hipStream_t s);
hipError_t launch_col_fwd_eg(const Geom& g, const cplx* Ein, cplx* SIG, cplx* Go, hipStream_t s);
hipError_t launch_col_basis_eg(const Geom& g, const cplx* W, cplx* V, size_t vs, int j, const GmresState* st,
                               cplx* Eo, cplx* Go, hipStream_t s);
// D (may be null): D += (updated - previous) sigma_hat, the guess increment
hipError_t launch_col_update_eg(const Geom& g, cplx* SIG, const cplx* V, size_t vs, const GmresState* st, cplx* Eo,
                                cplx* Go, cplx* D, hipStream_t s);
// SIG += D, then E, G of SIG (extrapolated initial guess of an RK stage)
hipError_t launch_col_guess_eg(const Geom& g, cplx* SIG, const cplx* D, cplx* Eo, cplx* Go, hipStream_t s);
hipError_t launch_col_precond_dot(const Geom& g, const cplx* P, const cplx* Q, const cplx* V, size_t vs, int j,
                                  GmresState* st, cplx* W, double* partials, hipStream_t s);
hipError_t launch_col_resid(const Geom& g, const cplx* P, const cplx* Q, const cplx* R1, const cplx* R2, int need_b,
                            int flags, GmresState* st, cplx* W, double* partials, hipStream_t s);
hipError_t launch_col_inv(const Geom& g, const cplx* S, cplx* o, hipStream_t s);
hipError_t launch_col_apply(const Geom& g, const cplx* P, const cplx* Q, int precond, cplx* o, hipStream_t s);
hipError_t launch_col_filter(const Geom& g, const cplx* Sx, int op, double thr, cplx* o, hipStream_t s);
hipError_t launch_col_tail(const Geom& g, const cplx* Sx, GmresState* st, double* partials, hipStream_t s);
hipError_t launch_col_dy(const Geom& g, const double* f, double* o, hipStream_t s);
hipError_t launch_col_flux(const Geom& g, const double* dhp, const double* qy, const double* B, RkStage rk, RkField fh,
                           RkField fvy, hipStream_t s);
hipError_t launch_upd(const Geom& g, cplx* W, const cplx* V, size_t vs, int j, GmresState* st, double* partials,
                      hipStream_t s);
hipError_t launch_field_stats(const double* h, const double* vx, const double* vy, size_t n, GmresState* st,
                              double* partials, hipStream_t s);
int max_partial_blocks(const Geom& g);
// The next kernel launch records these events at its start and end (null: none).
void set_launch_events(hipEvent_t start, hipEvent_t stop);
// chain-parallel Arnoldi passes (same results as row_op mode 0, col_basis_eg,
// col_precond_dot); chained_ok tells whether this grid can use them
bool chained_ok(const Geom& g);
hipError_t launch_row_matvec3(const Geom& g, const cplx* E, const cplx* G, const double* h, cplx* P, cplx* Q,
                              const GmresState* st, hipStream_t s);
hipError_t launch_col_basis2(const Geom& g, const cplx* W, cplx* V, size_t vs, int j, const GmresState* st, cplx* Eo,
                             cplx* Go, hipStream_t s);
hipError_t launch_col_proj(const Geom& g, const cplx* win, cplx* W, const cplx* V, size_t vs, int j, GmresState* st,
                           cplx* Eo, cplx* Go, double* partials, hipStream_t s);
hipError_t launch_col_precond_new(const Geom& g, const cplx* P, const cplx* Q, const cplx* W, cplx* V, cplx* Z,
                                  size_t vs, int j, GmresState* st, double* partials, hipStream_t s);
hipError_t launch_col_precond_dot2(const Geom& g, const cplx* P, const cplx* Q, const cplx* V, size_t vs, int j,
                                   GmresState* st, cplx* W, double* partials, hipStream_t s);

}  // namespace sgn

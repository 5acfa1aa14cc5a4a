// HIP kernels of the SGN hot path for gfx950 (FP64).
//
// Data layout (one field = ny x nx doubles, row-major, x contiguous):
//   physical fields     f[y][x]
//   x-half spectra      S[y][c], c < nx/2, complex: the x-DFT of row y; slot
//                       c = 0 holds DC + i * Nyquist (both real for a real row)
//   2D spectra          the y-DFT of the x-half spectra (same layout), i.e.
//                       the 2D DFT at (kx = c, ky); column 0 packs kx = 0 and
//                       kx = nx/2, which every operator here treats alike
//                       because the Nyquist wavenumber is set to zero.
// Row passes transform two adjacent real rows as one complex row; column
// passes transform tc adjacent complex columns per block (loads of tc*16
// contiguous bytes per row), two real columns per complex column for physical
// data.
//
// This file is compiled once per working precision: SGN_PREC=64 (namespace
// sgn::p64, double fields) and SGN_PREC=32 (namespace sgn::p32, float fields
// and transforms).  Reductions, inner products, norms, the GMRES state and
// every scalar coefficient are FP64 in both.
#include <hip/hip_ext.h>

#ifndef SGN_PREC
#define SGN_PREC 64
#endif
#if SGN_PREC == 32
#define SGN_NS p32
#define SGN_REAL float
#define SGN_CPLX float2
#define TWX(g) ((g).twx32)
#define TWY(g) ((g).twy32)
#elif SGN_PREC == 64
#define SGN_NS p64
#define SGN_REAL double
#define SGN_CPLX double2
#define TWX(g) ((g).twx)
#define TWY(g) ((g).twy)
#else
#error "SGN_PREC must be 32 or 64"
#endif

#include "sgn_internal.hpp"
#include "sgn_launch.hpp"
#include "sgn_fft.hpp"

namespace sgn {
namespace SGN_NS {

// ----------------------------------------------------------------------------
// Ensemble members in one launch: member m = blockIdx.z works on the member
// m copy of every array.  Member workspaces sit at a fixed stride from member
// 0's (Geom::ws_lo, ws_span, ws_stride), the caller's fields at another
// (Geom::f_stride); an address inside member 0's workspace moves by the
// first, any other by the second.  Member 0 (and a single grid) uses the
// pointers as given.
// ----------------------------------------------------------------------------

template <class T>
__device__ __forceinline__ T* mshift(const Geom& g, T* p) {
  const size_t m = blockIdx.z;
  if (m == 0 || p == nullptr) return p;
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  const size_t stride = (a - g.ws_lo < g.ws_span) ? g.ws_stride : g.f_stride;
  return reinterpret_cast<T*>(a + m * stride);
}

__device__ __forceinline__ RkField mshift_field(const Geom& g, RkField f) {
  f.yn = mshift(g, f.yn); f.acc = mshift(g, f.acc); f.out = mshift(g, f.out);
  return f;
}

// ----------------------------------------------------------------------------
// Reductions (deterministic: fixed-order trees, no floating-point atomics)
// ----------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ double wave_min(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o, 64));
  return x;
}
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

__constant__ int kKindsInvariants[7] = {0, 0, 0, 0, 0, 1, 2};
__constant__ int kKindsMax[1] = {2};
__constant__ int kKindsStats[2] = {1, 2};

__device__ __forceinline__ int flat_tid() { return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z); }
__device__ __forceinline__ int block_threads() { return blockDim.x * blockDim.y * blockDim.z; }

// Partials travel through device-scope atomic stores and loads, which are
// performed at the device coherence point (not in an XCD-private L2), so the
// last-block protocol needs no cache-wide write-back or invalidate.
__device__ __forceinline__ void partial_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double partial_load(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The GMRES stop code where a block of the same launch may store it (kernels
// that finish an Arnoldi step: block 0 stores the step while later blocks of
// the launch may still be starting).  Every block derives the same stop code
// from the same inputs, and block 0 stores either the value the others read
// before (0) or the one they compute themselves, so a block that sees the new
// value exits exactly where it would have exited on its own.  The load and
// the store are relaxed agent-scope atomics so that this benign race is
// well-defined; the ordering it needs comes from the kernel boundaries.
__device__ __forceinline__ int status_load(const GmresState* st) {
  return __hip_atomic_load(const_cast<int32_t*>(&st->st.done), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void status_store(GmresState* st, int v) {
  __hip_atomic_store(&st->st.done, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Ensemble launches that start a restarted cycle run only for the members
// whose last cycle filled up below the iteration cap (the host enqueues them
// for every member once any member needs one).
__device__ __forceinline__ bool restart_due(const GmresState* st) {
  return st->st.done == 2 && st->st.total_iters < st->maxit;
}

__device__ __forceinline__ uint32_t ticket(uint32_t* c) {
  return __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void reset_counter(uint32_t* c) {
  __hip_atomic_store(c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every block calls this once after writing its partials with partial_store.
// Returns true in exactly one block (the last to arrive).  Each thread first
// waits for its own partial stores to complete.  The ordering of the partial
// stores before the ticket rests on gfx950 behaviour, not on the HIP memory
// model: an agent-scope store is acknowledged (s_waitcnt) only once it has
// reached the device coherence point, and the ticket is taken after every
// thread of the block has waited for its acknowledgements.  A release/acquire
// pair would make this formal but compiles to an L2 write-back and invalidate
// in every block, which cost 5-10x in the kernels that finish reductions.  Tickets are taken in two
// levels (groups of kTicketGroup blocks, then groups) so that no counter sees
// more than max(kTicketGroup, #groups) same-address atomics.
__device__ bool last_block_arrive(uint32_t* ctr, int nblocks) {
  __shared__ int s_last;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (flat_tid() == 0) {
    const int grp = blockIdx.x / kTicketGroup;
    const int ngroups = (nblocks + kTicketGroup - 1) / kTicketGroup;
    const int gsize = min(kTicketGroup, nblocks - grp * kTicketGroup);
    uint32_t* gc = ctr + 32 * (1 + grp);
    int last = 0;
    if (ticket(gc) == (uint32_t)(gsize - 1)) {
      reset_counter(gc);
      if (ticket(ctr) == (uint32_t)(ngroups - 1)) {
        reset_counter(ctr);
        last = 1;
      }
    }
    s_last = last;
  }
  __syncthreads();
  return s_last != 0;
}

// Reduce-scatter of eight values over a wave: on return lane l holds the
// wave sum of value (l >> 3) & 7.  The first three butterfly levels halve the
// values each lane carries (4, 2, 1 shuffles), the last three finish one
// value: 10 shuffles instead of 6 per value.
__device__ __forceinline__ double wave_sum8_scatter(const double (&a)[8]) {
  const int lane = flat_tid() & 63;
  const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
  double b[4], c[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) b[i] = (h5 ? a[4 + i] : a[i]) + __shfl_xor(h5 ? a[i] : a[4 + i], 32, 64);
#pragma unroll
  for (int i = 0; i < 2; ++i) c[i] = (h4 ? b[2 + i] : b[i]) + __shfl_xor(h4 ? b[i] : b[2 + i], 16, 64);
  double d = (h3 ? c[1] : c[0]) + __shfl_xor(h3 ? c[0] : c[1], 8, 64);
  d += __shfl_xor(d, 4, 64);
  d += __shfl_xor(d, 2, 64);
  d += __shfl_xor(d, 1, 64);
  return d;
}

// The same for four values a[0..3]: the sum of a[i] over the wave ends in
// lanes 16 i .. 16 i + 15.
__device__ __forceinline__ double wave_sum4_scatter(const double (&a)[8]) {
  const int lane = flat_tid() & 63;
  const bool h5 = lane & 32, h4 = lane & 16;
  double b[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) b[i] = (h5 ? a[2 + i] : a[i]) + __shfl_xor(h5 ? a[i] : a[2 + i], 32, 64);
  double d = (h4 ? b[1] : b[0]) + __shfl_xor(h4 ? b[0] : b[1], 16, 64);
  d += __shfl_xor(d, 8, 64);
  d += __shfl_xor(d, 4, 64);
  d += __shfl_xor(d, 2, 64);
  d += __shfl_xor(d, 1, 64);
  return d;
}

// kind: 0 sum, 1 min, 2 max.  out[k] (LDS) = reduction over blocks of
// partials[b * kPartialStride + k], in a fixed order.
// kAtomic = false: the partials were written by an earlier kernel on the
// stream (visible to plain loads after the kernel boundary).
// VW: values per wave in a sum (8, or 4 for a caller that holds other loads
// in registers meanwhile).
template <bool kAtomic = true, int VW = 8>
__device__ void reduce_partials(const double* partials, int nblocks, int nvals, const int* kind,
                                double* out) {
  static_assert(VW == 8 || VW == 4, "eight or four values per wave");
  const int tid = flat_tid();
  const int lane = tid & 63, wave = tid >> 6, nw = block_threads() >> 6;
  if (!kind) {
    // sums: each wave takes VW values and keeps the loads of 256 blocks in
    // flight together
    for (int k0 = VW * wave; k0 < nvals; k0 += VW * nw) {
      double a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = 0.0;
      for (int b0 = 0; b0 < nblocks; b0 += 256) {
        double x[4][VW];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int b = b0 + 64 * u + lane;
#pragma unroll
          for (int q = 0; q < VW; ++q)
            x[u][q] = (b < nblocks && k0 + q < nvals)
                          ? (kAtomic ? partial_load(&partials[(size_t)b * kPartialStride + k0 + q])
                                     : partials[(size_t)b * kPartialStride + k0 + q])
                          : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int q = 0; q < VW; ++q) a[q] += x[u][q];
      }
      if constexpr (VW == 8) {
        const double r = wave_sum8_scatter(a);
        if ((lane & 7) == 0 && k0 + (lane >> 3) < nvals) out[k0 + (lane >> 3)] = r;
      } else {
        const double r = wave_sum4_scatter(a);
        if ((lane & 15) == 0 && k0 + (lane >> 4) < nvals) out[k0 + (lane >> 4)] = r;
      }
    }
    __syncthreads();
    return;
  }
  for (int k = wave; k < nvals; k += nw) {
    const int kd = kind ? kind[k] : 0;
    const double id = kd == 0 ? 0.0 : (kd == 1 ? 1e300 : -1e300);
    double s = id;
    for (int b0 = 0; b0 < nblocks; b0 += 64 * 8) {
      double x[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int b = b0 + lane + 64 * q;
        x[q] = b < nblocks ? partial_load(&partials[(size_t)b * kPartialStride + k]) : id;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) s = kd == 0 ? s + x[q] : (kd == 1 ? fmin(s, x[q]) : fmax(s, x[q]));
    }
    s = kd == 0 ? wave_sum(s) : (kd == 1 ? wave_min(s) : wave_max(s));
    if (lane == 0) out[k] = s;
  }
  __syncthreads();
}

// Block-level: wave partial of value k goes to red[k * nw + wave].
__device__ __forceinline__ void wave_partial(double x, double* red, int k) {
  const int tid = flat_tid();
  const double s = wave_sum(x);
  if ((tid & 63) == 0) red[k * (block_threads() >> 6) + (tid >> 6)] = s;
}

// Eight values at once (one reduce-scatter): a[q] is the thread's
// contribution to value k0 + q; wave sums go to red[k * nw + wave], k < nvals.
__device__ __forceinline__ void wave_partials8(double (&a)[8], double* red, int k0, int nvals) {
  const double s = wave_sum8_scatter(a);
  const int tid = flat_tid(), lane = tid & 63;
  if ((lane & 7) == 0 && k0 + (lane >> 3) < nvals) red[(k0 + (lane >> 3)) * (block_threads() >> 6) + (tid >> 6)] = s;
}

__device__ __forceinline__ void block_partials_out(const double* red, int nvals, double* partials,
                                                   const int* kind) {
  __syncthreads();
  const int tid = flat_tid(), nw = block_threads() >> 6;
  for (int k = tid; k < nvals; k += block_threads()) {
    const int kd = kind ? kind[k] : 0;
    double s = red[k * nw];
    for (int w = 1; w < nw; ++w) {
      const double x = red[k * nw + w];
      s = kd == 0 ? s + x : (kd == 1 ? fmin(s, x) : fmax(s, x));
    }
    partial_store(&partials[(size_t)blockIdx.x * kPartialStride + k], s);
  }
}

// ----------------------------------------------------------------------------
// GMRES scalar work (one thread of a block, from LDS copies)
// ----------------------------------------------------------------------------

// The state that finishing Arnoldi step j reads, loaded into registers at
// the start of a kernel so that these loads wait together with those of the
// block partials instead of after them: thread i < j holds rotation i,
// thread i <= j (with_cj) the projection coefficient i, thread 0 the scalars.
struct FinishPre {
  double cs, sn, cj;
  double gvj, tol, beta0;
  int cycle_base, m, maxit;
};

__device__ __forceinline__ FinishPre finish_prefetch(const GmresState* st, int j, bool with_cj) {
  FinishPre p{};
  const int tid = flat_tid();
  if (tid < j) {
    p.cs = st->cs[tid];
    p.sn = st->sn[tid];
  }
  if (with_cj && tid <= j) p.cj = st->cproj[tid];
  if (tid == 0 && j >= 0) {
    p.gvj = st->gv[j];
    p.tol = st->tol;
    p.beta0 = st->st.beta0;
    p.cycle_base = st->cycle_base;
    p.m = st->m;
    p.maxit = st->maxit;
  }
  return p;
}

__device__ int gmres_finish_column(GmresState* st, int j, const double* cj, double beta, const double* s2,
                                   bool write, const FinishPre* pre = nullptr, bool restart_now = false);

// Finish CGS2 Arnoldi step j in a block of the kernel that follows the
// update kernel, from its nb block partials (value 0: ||w1||^2; 1 + i:
// s2_i = <V_i, w1>): H(:, j) = s + s2 and H(j+1, j) = ||w1 - V s2|| =
// sqrt(||w1||^2 - |s2|^2), then the Givens update and test of
// gmres_finish_column (write: this block stores the step).  Leaves s2 in the
// caller's LDS array and H(j+1, j) in beta; returns the stop code.
__device__ int cgs2_finish(const Geom& g, GmresState* st, int j, const double* pin, int nb, double* s2, double& beta,
                           bool write) {
  __shared__ double outv[kMaxRestart + 2];
  __shared__ double colv[kMaxRestart + 1];
  __shared__ double sh_beta;
  const int tid = flat_tid(), nt = block_threads();
  reduce_partials<false>(pin, nb, j + 2, nullptr, outv);
  for (int i = tid; i <= j; i += nt) {
    s2[i] = outv[1 + i] * g.inv_n;
    colv[i] = st->s[i] + s2[i];
  }
  if (tid == 0) {
    double sum2 = 0.0;
    for (int i = 0; i <= j; ++i) {
      const double x = outv[1 + i] * g.inv_n;
      sum2 += x * x;
    }
    const double b2 = outv[0] * g.inv_n - sum2;
    sh_beta = b2 > 0.0 ? sqrt(b2) : 0.0;
  }
  __syncthreads();
  beta = sh_beta;
  return gmres_finish_column(st, j, colv, sh_beta, s2, write);
}

// Finish Arnoldi step j given its Hessenberg column cj[0..j] and
// H(j+1, j) = beta: apply the previous Givens rotations and a new one,
// update the residual estimate and test it.  Returns the stop code (0 go on,
// 1 converged, 2 cycle full, 3 iteration cap) in every thread of the block.
// write: this block stores the step (column j of R, rotation j, g_j after
// and g_{j+1} before rotation, beta, the status, s2 and, when stopping, the
// back-substituted y).  Several blocks of one kernel may evaluate the same
// step, one of them writing: the others read only state that the step leaves
// unchanged (rotations below j, g_j before rotation, the cycle's iteration
// base), so each takes the writer's decision.
__device__ int gmres_finish_column(GmresState* st, int j, const double* cj, double beta, const double* s2,
                                   bool write, const FinishPre* pre, bool restart_now) {
  __shared__ double sh_col[kMaxRestart + 1];
  __shared__ double sh_cs[kMaxRestart], sh_sn[kMaxRestart];
  __shared__ double sh_gj, sh_gn, sh_resid;
  __shared__ int sh_stop, sh_total;
  const int tid = flat_tid(), nt = block_threads();
  const int ld = kMaxRestart + 1;
  const FinishPre p = pre ? *pre : finish_prefetch(st, j, false);
  if (tid < j) {
    sh_cs[tid] = p.cs;
    sh_sn[tid] = p.sn;
  }
  for (int i = tid; i <= j; i += nt) sh_col[i] = cj[i];
  __syncthreads();
  if (tid == 0) {
    double* col = sh_col;  // column j, rotated in place
    col[j + 1] = beta;
    for (int i = 0; i < j; ++i) {
      const double a = col[i], b = col[i + 1];
      col[i] = sh_cs[i] * a + sh_sn[i] * b;
      col[i + 1] = -sh_sn[i] * a + sh_cs[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double rho = hypot(a, b);
    double c = 1.0, sn = 0.0;
    if (rho > 0.0) {
      c = a / rho;
      sn = b / rho;
    }
    col[j] = rho;
    col[j + 1] = 0.0;
    sh_cs[j] = c;
    sh_sn[j] = sn;
    const double gj = p.gvj;
    sh_gj = c * gj;
    sh_gn = -sn * gj;
    const double resid = fabs(sh_gn);
    const int total = p.cycle_base + j + 1;
    int done = 0;
    if (restart_now)
      done = total >= p.maxit ? 3 : 2;
    else if (resid <= p.tol * p.beta0 || beta == 0.0)
      done = 1;
    else if (j + 1 >= p.m)
      done = 2;
    else if (total >= p.maxit)
      done = 3;
    sh_resid = resid;
    sh_total = total;
    sh_stop = done;
  }
  __syncthreads();
  const int stop = sh_stop;
  if (!write) return stop;
  for (int i = tid; i <= j + 1; i += nt) st->H[j * ld + i] = sh_col[i];
  if (s2)
    for (int i = tid; i <= j; i += nt) st->s2[i] = s2[i];
  if (stop) {
    // back substitution R y = g on the (j+1) x (j+1) triangle (columns below
    // j of R and the rotated g below j from earlier steps); R is staged in
    // the kernel's dynamic LDS (launched with at least m^2 doubles), which
    // the block does not use otherwise once it stops
    extern __shared__ double dyn_lds[];
    double* sh_R = dyn_lds;
    const int lr = j + 1;
    __shared__ double sh_g[kMaxRestart + 1], sh_y[kMaxRestart];
    for (int e = tid; e < j * lr; e += nt) sh_R[e] = st->H[(e / lr) * ld + e % lr];
    for (int i = tid; i <= j; i += nt) sh_R[j * lr + i] = sh_col[i];
    for (int i = tid; i < j; i += nt) sh_g[i] = st->gr[i];
    if (tid == 0) sh_g[j] = sh_gj;
    __syncthreads();
    if (tid == 0) {
      for (int i = j; i >= 0; --i) {
        double acc = sh_g[i];
        for (int l = i + 1; l <= j; ++l) acc -= sh_R[l * lr + i] * sh_y[l];
        const double d = sh_R[i * lr + i];
        sh_y[i] = d != 0.0 ? acc / d : 0.0;
      }
    }
    __syncthreads();
    for (int i = tid; i <= j; i += nt) st->y[i] = sh_y[i];
  }
  if (tid == 0) {
    st->cs[j] = sh_cs[j];
    st->sn[j] = sh_sn[j];
    st->gr[j] = sh_gj;
    st->gv[j + 1] = sh_gn;
    st->beta = beta;
    st->st.jdone = j + 1;
    st->st.total_iters = sh_total;
    st->st.resid = sh_resid;
    status_store(st, stop);
  }
  return stop;
}

// ----------------------------------------------------------------------------
// Row passes
// ----------------------------------------------------------------------------

// EE: values per thread of the row transforms (the engine's default, or
// another radix a kernel is instantiated for).
template <int N, int EE = FftShape<N>::E>
struct Row {
  static constexpr int E = EE;
  static constexpr int TPF = N / EE;
  static constexpr int LDS = RowMap::size(N);  // cplx per row pair
};

template <int N, int EE = FftShape<N>::E>
__device__ __forceinline__ void load_phys_pair(cplx* v, const real* __restrict__ f, int ya, int t) {
  const real* a = f + (size_t)ya * N;
  const real* b = a + N;
#pragma unroll
  for (int r = 0; r < Row<N, EE>::E; ++r) {
    const int p = t + r * Row<N, EE>::TPF;
    v[r] = make_cplx(a[p], b[p]);
  }
}

template <int N>
__device__ __forceinline__ void store_phys_pair(const cplx* v, real* __restrict__ f, int ya, int t) {
  real* a = f + (size_t)ya * N;
  real* b = a + N;
#pragma unroll
  for (int r = 0; r < Row<N>::E; ++r) {
    const int p = t + r * Row<N>::TPF;
    a[p] = v[r].x;
    b[p] = v[r].y;
  }
}

// Full spectrum of (row ya) + i (row ya+1) from their x-half spectra, times s.
template <int N, int EE = FftShape<N>::E>
__device__ __forceinline__ void load_spec_pair(cplx* v, const cplx* __restrict__ S, int ya, int t, double s) {
  constexpr int H = N / 2;
  const cplx* A = S + (size_t)ya * H;
  const cplx* B = A + H;
  // one unconditional load pair per value, all issued before any is used,
  // so that they are in flight together
  cplx la[Row<N, EE>::E], lb[Row<N, EE>::E];
#pragma unroll
  for (int r = 0; r < Row<N, EE>::E; ++r) {
    const int p = t + r * Row<N, EE>::TPF;
    const int q = (p == 0 || p == H) ? 0 : (p < H ? p : N - p);
    la[r] = A[q];
    lb[r] = B[q];
  }
#pragma unroll
  for (int r = 0; r < Row<N, EE>::E; ++r) {
    const int p = t + r * Row<N, EE>::TPF;
    const cplx a = la[r], b = lb[r];
    cplx z;
    if (p == 0)
      z = make_cplx(a.x, b.x);
    else if (p == H)
      z = make_cplx(a.y, b.y);
    else if (p < H)
      z = make_cplx(a.x - b.y, a.y + b.x);
    else
      z = make_cplx(a.x + b.y, b.x - a.y);
    v[r] = cscale(z, s);
  }
}

// Split the full spectrum of a packed row pair into the two half spectra.
template <int N>
__device__ __forceinline__ void store_spec_pair(const cplx* v, cplx* __restrict__ S, int ya, int t, cplx* buf) {
  const RowMap M;
  constexpr int H = N / 2;
#pragma unroll
  for (int r = 0; r < Row<N>::E; ++r) buf[M.at(t + r * Row<N>::TPF)] = v[r];
  __syncthreads();
  cplx* A = S + (size_t)ya * H;
  cplx* B = A + H;
#pragma unroll
  for (int r = 0; r < Row<N>::E / 2; ++r) {
    const int k = t + r * Row<N>::TPF;
    if (k == 0) {
      const cplx z0 = buf[M.at(0)], zn = buf[M.at(H)];
      A[0] = make_cplx(z0.x, zn.x);
      B[0] = make_cplx(z0.y, zn.y);
    } else {
      const cplx z = buf[M.at(k)], zc = buf[M.at(N - k)];
      A[k] = make_cplx(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));
      B[k] = make_cplx(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));
    }
  }
  __syncthreads();
}

#define ROW_SETUP(N)                                   \
  constexpr int E = Row<N>::E;                         \
  constexpr int TPF = Row<N>::TPF;                     \
  const RowMap map;                                    \
  extern __shared__ cplx lds[];                        \
  const int t = threadIdx.x;                           \
  const int ya = 2 * (blockIdx.x * blockDim.y + threadIdx.y); \
  cplx* buf = lds + threadIdx.y * Row<N>::LDS;         \
  TwiddleSet<N> twx;                                   \
  gather_twiddles<N>(twx, t, TWX(g));                   \
  (void)TPF;

// physical f -> x-half spectra S
template <int N>
__global__ void __launch_bounds__(512) k_row_r2c(Geom g, Trio io) {
  const real* __restrict__ f = mshift(g, static_cast<const real*>(io.in[blockIdx.y]));
  cplx* __restrict__ S = mshift(g, static_cast<cplx*>(io.out[blockIdx.y]));
  ROW_SETUP(N)
  cplx v[E];
  load_phys_pair<N>(v, f, ya, t);
  fft<N, false, decltype(map)>(v, buf, t, twx, map);
  store_spec_pair<N>(v, S, ya, t, buf);
}

// x-half spectra S -> physical f
template <int N>
__global__ void __launch_bounds__(512) k_row_c2r(Geom g, Trio io) {
  const cplx* __restrict__ S = mshift(g, static_cast<const cplx*>(io.in[blockIdx.y]));
  real* __restrict__ f = mshift(g, static_cast<real*>(io.out[blockIdx.y]));
  ROW_SETUP(N)
  cplx v[E];
  load_spec_pair<N>(v, S, ya, t, g.inv_nx);
  fft<N, true, decltype(map)>(v, buf, t, twx, map);
  store_phys_pair<N>(v, f, ya, t);
}

// out = d/dx f
template <int N>
__global__ void __launch_bounds__(512) k_row_dx(Geom g, const real* __restrict__ f, real* __restrict__ out) {
  f = mshift(g, f); out = mshift(g, out);
  ROW_SETUP(N)
  cplx v[E];
  load_phys_pair<N>(v, f, ya, t);
  fft<N, false, decltype(map)>(v, buf, t, twx, map);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = mul_ik(v[r], wavenumber(t + r * TPF, N, g.inv_Lx) * g.inv_nx);
  fft<N, true, decltype(map)>(v, buf, t, twx, map);
  store_phys_pair<N>(v, out, ya, t);
}

#ifndef SGN_FAST_RECIP
#define SGN_FAST_RECIP 1
#endif
// 1 / x for a positive normal x (the depth h, which the field checks keep
// positive, and the preconditioner symbol, at least m0 = 3 / h_inf^3): the
// hardware reciprocal estimate refined by two Newton steps, within an ulp of
// the quotient, instead of the full division sequence (scaling and fix-up for
// zeros, infinities and denormals, which these operands never are; a depth
// or symbol beyond the normal range would give a non-finite result, which the
// field checks report)
__device__ __forceinline__ double recip_pos(double x) {
#if SGN_FAST_RECIP
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
#else
  return 1.0 / x;
#endif
}

// Elliptic operator, x part, in x-spectral form.  From E = F_x sigma and
// G = F_x d_y sigma (x-half spectra) and the depth h:
//   A1 = F_x(3 sigma / h^3) - i kx F_x(d_x sigma / h),   A2 = F_x(d_y sigma / h)
// so that F(L_h sigma) = F_y(A1) - i ky F_y(A2).
// MODE 0: P = A1, Q = A2 (the Arnoldi matvec; skipped once GMRES is done).
// MODE 1: residual with b = -div v:  B1 = -i kx F_x vx, B2 = F_x vy,
//         P = B1 - A1, Q = B2 - A2 (and R1 = B1, R2 = B2 if need_b).
// MODE 2: residual with an explicit b (passed in vx): B1 = F_x b, B2 = 0.
template <int N, int MODE, bool SF = false>
__global__ void __launch_bounds__(512) k_row_op(Geom g, const cplx* __restrict__ Es, const cplx* __restrict__ Gs,
                                                const real* __restrict__ h, const real* __restrict__ vx,
                                                const real* __restrict__ vy, cplx* __restrict__ P,
                                                cplx* __restrict__ Q, cplx* __restrict__ R1, cplx* __restrict__ R2,
                                                int need_b, int predicate, const GmresState* __restrict__ st) {
  Es = mshift(g, Es); Gs = mshift(g, Gs); h = mshift(g, h); vx = mshift(g, vx); vy = mshift(g, vy);
  P = mshift(g, P); Q = mshift(g, Q); R1 = mshift(g, R1); R2 = mshift(g, R2); st = mshift(g, st);
  if (MODE == 0 && predicate && SF && st->st.done) return;
  if (MODE != 0 && predicate == 2 && !restart_due(st)) return;  // ensemble restart: only members that restart
  ROW_SETUP(N)
  // every global load first, so their latencies overlap (the GMRES status
  // too: the loads are in bounds whatever it is)
  cplx v[E], u[E], w[E], hi[E], x[E], y[E];
  load_spec_pair<N>(v, Es, ya, t, g.inv_nx);
  load_spec_pair<N>(w, Gs, ya, t, g.inv_nx);
  load_phys_pair<N>(hi, h, ya, t);
  if constexpr (MODE != 0) load_phys_pair<N>(x, vx, ya, t);
  if constexpr (MODE == 1) load_phys_pair<N>(y, vy, ya, t);
  if (MODE == 0 && predicate && st->st.done) return;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    hi[r] = make_cplx(recip_pos(hi[r].x), recip_pos(hi[r].y));
    u[r] = mul_ik(v[r], wavenumber(t + r * TPF, N, g.inv_Lx));
  }
  fft<N, true, decltype(map)>(v, buf, t, twx, map);  // sigma
  fft<N, true, decltype(map)>(u, buf, t, twx, map);  // d_x sigma
  fft<N, true, decltype(map)>(w, buf, t, twx, map);  // d_y sigma
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const double ia = hi[r].x, ib = hi[r].y;
    v[r] = make_cplx(3.0 * v[r].x * ia * ia * ia, 3.0 * v[r].y * ib * ib * ib);
    u[r] = make_cplx(u[r].x * ia, u[r].y * ib);
    w[r] = make_cplx(w[r].x * ia, w[r].y * ib);
  }
  fft<N, false, decltype(map)>(v, buf, t, twx, map);
  fft<N, false, decltype(map)>(u, buf, t, twx, map);
  fft<N, false, decltype(map)>(w, buf, t, twx, map);  // A2
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = csub(v[r], mul_ik(u[r], wavenumber(t + r * TPF, N, g.inv_Lx)));  // A1
  if constexpr (MODE == 0) {
    store_spec_pair<N>(v, P, ya, t, buf);
    store_spec_pair<N>(w, Q, ya, t, buf);
  } else {
    fft<N, false, decltype(map)>(x, buf, t, twx, map);
    if constexpr (MODE == 1) {
#pragma unroll
      for (int r = 0; r < E; ++r) x[r] = mul_ik(x[r], -wavenumber(t + r * TPF, N, g.inv_Lx));
    }
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = csub(x[r], v[r]);
    store_spec_pair<N>(v, P, ya, t, buf);
    if (need_b) store_spec_pair<N>(x, R1, ya, t, buf);
    if constexpr (MODE == 1) {
      fft<N, false, decltype(map)>(y, buf, t, twx, map);
#pragma unroll
      for (int r = 0; r < E; ++r) w[r] = csub(y[r], w[r]);
      store_spec_pair<N>(w, Q, ya, t, buf);
      if (need_b) store_spec_pair<N>(y, R2, ya, t, buf);
    } else {
#pragma unroll
      for (int r = 0; r < E; ++r) w[r] = make_cplx(-w[r].x, -w[r].y);
      store_spec_pair<N>(w, Q, ya, t, buf);
    }
  }
}

// The Arnoldi matvec, x part (same result as k_row_op<N, 0>), with its three
// independent transform chains run concurrently by three thread groups of
// the block (threadIdx.y % 3):
//   chain 0: sigma -> 3 sigma / h^3 -> F_x
//   chain 1: d_x sigma -> / h -> F_x -> (-i kx)
//   chain 2: d_y sigma -> / h -> F_x                      (= A2)
// A1 = chain 0 + chain 1 and A2 are split into half spectra through LDS.
// Block: (TPF, 3 * rows-pairs-per-block).
template <int N, bool SF>
__global__ void __launch_bounds__(1024) k_row_matvec3(Geom g, const cplx* __restrict__ Es, const cplx* __restrict__ Gs,
                                                      const real* __restrict__ h, cplx* __restrict__ P,
                                                      cplx* __restrict__ Q, const GmresState* st) {
  Es = mshift(g, Es); Gs = mshift(g, Gs); h = mshift(g, h); P = mshift(g, P); Q = mshift(g, Q);
  st = mshift(g, st);
  if (SF && st->st.done) return;
  constexpr int E = Row<N>::E;
  constexpr int TPF = Row<N>::TPF;
  constexpr int H = N / 2;
  const RowMap map;
  extern __shared__ cplx lds[];
  const int t = threadIdx.x;
  const int slot = threadIdx.y / 3, chain = threadIdx.y % 3;
  const int ya = 2 * (blockIdx.x * (blockDim.y / 3) + slot);
  cplx* base = lds + slot * 3 * Row<N>::LDS;
  cplx* buf = base + chain * Row<N>::LDS;
  // the loads (in bounds whatever the state) are issued before the GMRES
  // status is tested, so that its round trip overlaps theirs
  TwiddleSet<N> twx;
  gather_twiddles<N>(twx, t, TWX(g));
  cplx v[E], hi[E];
  load_spec_pair<N>(v, chain == 2 ? Gs : Es, ya, t, g.inv_nx);
  load_phys_pair<N>(hi, h, ya, t);
  if (st->st.done) return;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    hi[r] = make_cplx(recip_pos(hi[r].x), recip_pos(hi[r].y));
    if (chain == 1) v[r] = mul_ik(v[r], wavenumber(t + r * TPF, N, g.inv_Lx));
  }
  fft<N, true, RowMap>(v, buf, t, twx, map);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const double ia = hi[r].x, ib = hi[r].y;
    if (chain == 0)
      v[r] = make_cplx(3.0 * v[r].x * ia * ia * ia, 3.0 * v[r].y * ib * ib * ib);
    else
      v[r] = make_cplx(v[r].x * ia, v[r].y * ib);
  }
  fft<N, false, RowMap>(v, buf, t, twx, map);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    if (chain == 1) v[r] = mul_ik(v[r], -wavenumber(t + r * TPF, N, g.inv_Lx));
    buf[map.at(t + r * TPF)] = v[r];
  }
  __syncthreads();
  // unpack: chains 0 and 1 share A1 = buf0 + buf1 (one k each), chain 2 does A2
  const cplx* b0 = base;
  const cplx* b1 = base + Row<N>::LDS;
  const cplx* b2 = base + 2 * Row<N>::LDS;
  auto at_A1 = [&](int k) { return cadd(b0[map.at(k)], b1[map.at(k)]); };
  auto emit = [&](cplx* S, int k, cplx z, cplx zc) {
    cplx* A = S + (size_t)ya * H;
    cplx* B = A + H;
    A[k] = make_cplx(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));
    B[k] = make_cplx(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));
  };
#pragma unroll
  for (int r = 0; r < E / 2; ++r) {
    if ((chain == 2) ? false : (r % 2 != chain)) continue;
    const int k = t + r * TPF;
    if (chain == 2) {
      if (k == 0) {
        const cplx z0 = b2[map.at(0)], zn = b2[map.at(H)];
        cplx* A = Q + (size_t)ya * H;
        A[0] = make_cplx(z0.x, zn.x);
        A[H] = make_cplx(z0.y, zn.y);
      } else {
        emit(Q, k, b2[map.at(k)], b2[map.at(N - k)]);
      }
    } else {
      if (k == 0) {
        const cplx z0 = at_A1(0), zn = at_A1(H);
        cplx* A = P + (size_t)ya * H;
        A[0] = make_cplx(z0.x, zn.x);
        A[H] = make_cplx(z0.y, zn.y);
      } else {
        emit(P, k, at_A1(k), at_A1(N - k));
      }
    }
  }
}

// The same result as k_row_matvec3 with the three chains spread over blocks
// of two chains (2 TPF threads), so that two blocks fit a CU where one
// three-chain block does (the kernel needs about 126 VGPRs in FP64: four
// waves per SIMD).  Blocks 0 .. npairs-1 run chains 0 and 1 of row pair
// blockIdx.x and form A1 = chain 0 + chain 1 through LDS; blocks npairs ..
// npairs + npairs/2 - 1 run chain 2 (A2) for two row pairs, one per thread
// group.  Block: (TPF, 2); grid.x = npairs + npairs / 2 (npairs even).
template <int N, bool SF, int EE = FftShape<N>::E>
__global__ void __launch_bounds__(512) k_row_matvec2(Geom g, const cplx* __restrict__ Es, const cplx* __restrict__ Gs,
                                                     const real* __restrict__ h, cplx* __restrict__ P,
                                                     cplx* __restrict__ Q, const GmresState* st) {
  Es = mshift(g, Es); Gs = mshift(g, Gs); h = mshift(g, h); P = mshift(g, P); Q = mshift(g, Q);
  st = mshift(g, st);
  if (SF && st->st.done) return;
  constexpr int E = Row<N, EE>::E;
  constexpr int TPF = Row<N, EE>::TPF;
  constexpr int H = N / 2;
  const RowMap map;
  extern __shared__ cplx lds[];
  const int t = threadIdx.x;
  const int npairs = g.ny / 2;
  // Blocks come in groups of three for two row pairs (chains 0 and 1 of each
  // pair, then chain 2 of both), which read the same h and E rows.  With
  // npairs a multiple of 16, a group's three blocks take consecutive slots of
  // one XCD (blocks are dealt to the eight XCDs by linear index), so the
  // second reads of h and E hit that XCD's L2; otherwise the first npairs
  // blocks take chains 0 and 1 and the rest chain 2.
  int role, grp;
  if ((npairs & 15) == 0) {
    const int b = blockIdx.x, slot = b >> 3;
    grp = (slot / 3) * 8 + (b & 7);
    role = slot % 3;
  } else if ((int)blockIdx.x < npairs) {
    grp = blockIdx.x >> 1;
    role = blockIdx.x & 1;
  } else {
    grp = blockIdx.x - npairs;
    role = 2;
  }
  const bool a1 = role < 2;  // chains 0 and 1 of one row pair, else chain 2 of two
  const int chain = a1 ? threadIdx.y : 2;
  const int ya = 2 * (2 * grp + (a1 ? role : threadIdx.y));
  cplx* buf = lds + threadIdx.y * Row<N>::LDS;
  TwiddleSet<N, EE> twx;
  gather_twiddles<N, EE>(twx, t, TWX(g));
  cplx v[E], hi[E];
  load_spec_pair<N, EE>(v, chain == 2 ? Gs : Es, ya, t, g.inv_nx);
  load_phys_pair<N, EE>(hi, h, ya, t);
  if (st->st.done) return;  // tested after the (in-bounds) loads are issued
#pragma unroll
  for (int r = 0; r < E; ++r) {
    hi[r] = make_cplx(recip_pos(hi[r].x), recip_pos(hi[r].y));
    if (chain == 1) v[r] = mul_ik(v[r], wavenumber(t + r * TPF, N, g.inv_Lx));
  }
  fft<N, true, RowMap>(v, buf, t, twx, map);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const double ia = hi[r].x, ib = hi[r].y;
    if (chain == 0)
      v[r] = make_cplx(3.0 * v[r].x * ia * ia * ia, 3.0 * v[r].y * ib * ib * ib);
    else
      v[r] = make_cplx(v[r].x * ia, v[r].y * ib);
  }
  fft<N, false, RowMap>(v, buf, t, twx, map);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    if (chain == 1) v[r] = mul_ik(v[r], -wavenumber(t + r * TPF, N, g.inv_Lx));
    buf[map.at(t + r * TPF)] = v[r];
  }
  __syncthreads();
  auto emit = [&](cplx* S, int k, cplx z, cplx zc) {
    cplx* A = S + (size_t)ya * H;
    cplx* B = A + H;
    A[k] = make_cplx(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));
    B[k] = make_cplx(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));
  };
  if (a1) {
    // A1 = chain 0 + chain 1, each group unpacking every other k
    const cplx* b0 = lds;
    const cplx* b1 = lds + Row<N>::LDS;
    auto at_A1 = [&](int k) { return cadd(b0[map.at(k)], b1[map.at(k)]); };
#pragma unroll
    for (int r = 0; r < E / 2; ++r) {
      if (r % 2 != (int)threadIdx.y) continue;
      const int k = t + r * TPF;
      if (k == 0) {
        const cplx z0 = at_A1(0), zn = at_A1(H);
        cplx* A = P + (size_t)ya * H;
        A[0] = make_cplx(z0.x, zn.x);
        A[H] = make_cplx(z0.y, zn.y);
      } else {
        emit(P, k, at_A1(k), at_A1(N - k));
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < E / 2; ++r) {
      const int k = t + r * TPF;
      if (k == 0) {
        const cplx z0 = buf[map.at(0)], zn = buf[map.at(H)];
        cplx* A = Q + (size_t)ya * H;
        A[0] = make_cplx(z0.x, zn.x);
        A[H] = make_cplx(z0.y, zn.y);
      } else {
        emit(Q, k, buf[map.at(k)], buf[map.at(N - k)]);
      }
    }
  }
}

__device__ __forceinline__ void rk_one(const RkStage& rk, const RkField& f, size_t i, double k) {
  real* out = static_cast<real*>(f.out);
  real* acc = static_cast<real*>(f.acc);
  const real* yn = static_cast<const real*>(f.yn);
  if (rk.mode == 0) {
    out[i] = k;
  } else if (rk.mode == 1) {
    const double a = rk.first ? 0.0 : (double)acc[i];
    acc[i] = a + rk.wacc * k;
    out[i] = yn[i] + rk.cnext * k;
  } else {
    out[i] = yn[i] + rk.dt * ((double)acc[i] + rk.wacc * k);
  }
}

// Fluxes, x part.  With sigma from (E, G), the stage state (h, vx, vy):
//   qx = h vx - d_x sigma,  qy = h vy - d_y sigma,
//   B  = (vx^2 + vy^2)/2 - |grad sigma|^2 / (2 h^2) + g h - 9/2 sigma^2 / h^4
// writes dhp = -d_x qx, qy, B and k_vx = -d_x B (through the RK combine).
template <int N>
__global__ void __launch_bounds__(512) k_row_flux(Geom g, const cplx* __restrict__ Es, const cplx* __restrict__ Gs,
                                                  const real* h, const real* vx, const real* vy,
                                                  real* __restrict__ dhp, real* __restrict__ qy,
                                                  real* __restrict__ Bo, RkStage rk, RkField fvx) {
  Es = mshift(g, Es); Gs = mshift(g, Gs); h = mshift(g, h); vx = mshift(g, vx); vy = mshift(g, vy);
  dhp = mshift(g, dhp); qy = mshift(g, qy); Bo = mshift(g, Bo); rk.pred = mshift(g, rk.pred);
  fvx = mshift_field(g, fvx);
  ROW_SETUP(N)
  cplx s[E], sx[E], sy[E], hh[E], ux[E], uy[E];
  load_spec_pair<N>(s, Es, ya, t, g.inv_nx);
  load_spec_pair<N>(sy, Gs, ya, t, g.inv_nx);
  load_phys_pair<N>(hh, h, ya, t);
  load_phys_pair<N>(ux, vx, ya, t);
  load_phys_pair<N>(uy, vy, ya, t);
  if (rk.pred && rk.pred->done != 1) return;  // tested after the (in-bounds) loads are issued
#pragma unroll
  for (int r = 0; r < E; ++r) sx[r] = mul_ik(s[r], wavenumber(t + r * TPF, N, g.inv_Lx));
  fft<N, true, decltype(map)>(s, buf, t, twx, map);   // sigma
  fft<N, true, decltype(map)>(sx, buf, t, twx, map);  // d_x sigma
  fft<N, true, decltype(map)>(sy, buf, t, twx, map);  // d_y sigma
  cplx B[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const double a = hh[r].x, b = hh[r].y;
    const double ia = recip_pos(a), ib = recip_pos(b);
    const double sa = s[r].x * ia * ia, sb = s[r].y * ib * ib;
    const double rxa = sx[r].x * ia, rxb = sx[r].y * ib, rya = sy[r].x * ia, ryb = sy[r].y * ib;
    B[r].x = 0.5 * (ux[r].x * ux[r].x + uy[r].x * uy[r].x) - 0.5 * (rxa * rxa + rya * rya) + g.g * a - 4.5 * sa * sa;
    B[r].y = 0.5 * (ux[r].y * ux[r].y + uy[r].y * uy[r].y) - 0.5 * (rxb * rxb + ryb * ryb) + g.g * b - 4.5 * sb * sb;
    sx[r] = make_cplx(a * ux[r].x - sx[r].x, b * ux[r].y - sx[r].y);  // qx
    sy[r] = make_cplx(a * uy[r].x - sy[r].x, b * uy[r].y - sy[r].y);  // qy
  }
  store_phys_pair<N>(sy, qy, ya, t);
  store_phys_pair<N>(B, Bo, ya, t);
  fft<N, false, decltype(map)>(sx, buf, t, twx, map);
  fft<N, false, decltype(map)>(B, buf, t, twx, map);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const double k = -wavenumber(t + r * TPF, N, g.inv_Lx) * g.inv_nx;
    sx[r] = mul_ik(sx[r], k);
    B[r] = mul_ik(B[r], k);
  }
  fft<N, true, decltype(map)>(sx, buf, t, twx, map);  // -d_x qx
  fft<N, true, decltype(map)>(B, buf, t, twx, map);   // k_vx = -d_x B
  store_phys_pair<N>(sx, dhp, ya, t);
  const size_t oa = (size_t)ya * N, ob = oa + N;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = t + r * TPF;
    rk_one(rk, fvx, oa + p, B[r].x);
    rk_one(rk, fvx, ob + p, B[r].y);
  }
}

// Invariant densities (Section 2.3) with sigma from (E, G); dyvx = d_y vx.
// Partial sums: mass, Px, Py, energy, |curl v|^2, min h, max h.
template <int N>
__global__ void __launch_bounds__(512) k_row_invariants(Geom g, const cplx* __restrict__ Es,
                                                        const cplx* __restrict__ Gs, const real* __restrict__ h,
                                                        const real* __restrict__ vx, const real* __restrict__ vy,
                                                        const real* __restrict__ dyvx, double* partials,
                                                        GmresState* st, int nblocks) {
  Es = mshift(g, Es); Gs = mshift(g, Gs); h = mshift(g, h); vx = mshift(g, vx); vy = mshift(g, vy);
  dyvx = mshift(g, dyvx); partials = mshift(g, partials); st = mshift(g, st);
  constexpr int E = Row<N>::E;
  constexpr int TPF = Row<N>::TPF;
  const RowMap map;
  extern __shared__ cplx lds[];
  const int t = threadIdx.x;
  // blocks hold at least one full wave; slots past the last row pair read a
  // valid row pair and contribute nothing
  const int ya_raw = 2 * (blockIdx.x * blockDim.y + threadIdx.y);
  const bool rvalid = ya_raw < g.ny;
  const int ya = rvalid ? ya_raw : g.ny - 2;
  cplx* buf = lds + threadIdx.y * Row<N>::LDS;
  TwiddleSet<N> twx;
  gather_twiddles<N>(twx, t, TWX(g));
  __shared__ double red[7 * 8];
  __shared__ double outv[8];
  const size_t oa = (size_t)ya * N, ob = oa + N;
  cplx s[E], d[E];
  double acc[5] = {0, 0, 0, 0, 0};
  double mn = 1e300, mx = -1e300;
  load_spec_pair<N>(s, Es, ya, t, g.inv_nx);
#pragma unroll
  for (int r = 0; r < E; ++r) d[r] = mul_ik(s[r], wavenumber(t + r * TPF, N, g.inv_Lx));
  fft<N, true, decltype(map)>(s, buf, t, twx, map);  // sigma
  fft<N, true, decltype(map)>(d, buf, t, twx, map);  // d_x sigma
  cplx e[E];
  load_spec_pair<N>(e, Gs, ya, t, g.inv_nx);
  fft<N, true, decltype(map)>(e, buf, t, twx, map);  // d_y sigma
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = t + r * TPF;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const size_t i = (half ? ob : oa) + p;
      const double hh = h[i], sg = half ? s[r].y : s[r].x;
      const double sx = half ? d[r].y : d[r].x, sy = half ? e[r].y : e[r].x;
      const double ux = vx[i] - sx / hh, uy = vy[i] - sy / hh;
      const double dh = hh - g.h_inf;
      const double on = rvalid ? 1.0 : 0.0;
      acc[0] += on * dh;
      acc[1] += on * hh * ux;
      acc[2] += on * hh * uy;
      acc[3] += on * (0.5 * hh * (ux * ux + uy * uy) + 1.5 * sg * sg / (hh * hh * hh) + 0.5 * g.g * dh * dh);
      if (rvalid) {
        mn = fmin(mn, hh);
        mx = fmax(mx, hh);
      }
    }
  }
  // curl v = d_x vy - d_y vx
  load_phys_pair<N>(d, vy, ya, t);
  fft<N, false, decltype(map)>(d, buf, t, twx, map);
#pragma unroll
  for (int r = 0; r < E; ++r) d[r] = mul_ik(d[r], wavenumber(t + r * TPF, N, g.inv_Lx) * g.inv_nx);
  fft<N, true, decltype(map)>(d, buf, t, twx, map);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = t + r * TPF;
    const double ca = d[r].x - dyvx[oa + p], cb = d[r].y - dyvx[ob + p];
    acc[4] += rvalid ? ca * ca + cb * cb : 0.0;
  }
  const int* kinds = kKindsInvariants;
#pragma unroll
  for (int k = 0; k < 5; ++k) wave_partial(acc[k], red, k);
  {
    const int tid = flat_tid();
    const double a = wave_min(mn), b = wave_max(mx);
    if ((tid & 63) == 0) {
      red[5 * (block_threads() >> 6) + (tid >> 6)] = a;
      red[6 * (block_threads() >> 6) + (tid >> 6)] = b;
    }
  }
  block_partials_out(red, 7, partials, kinds);
  if (last_block_arrive(st->ctr, nblocks)) {
    reduce_partials(partials, nblocks, 7, kinds, outv);
    if (flat_tid() == 0) {
      st->st.red[0] = outv[0] * g.dA;
      st->st.red[1] = outv[1] * g.dA;
      st->st.red[2] = outv[2] * g.dA;
      st->st.red[3] = outv[3] * g.dA;
      st->st.red[4] = sqrt(outv[4] * g.dA);
      st->st.red[5] = outv[5];
      st->st.red[6] = outv[6];
    }
  }
}

// ----------------------------------------------------------------------------
// Column passes
// ----------------------------------------------------------------------------

template <int N>
struct Col {
  static constexpr int E = FftShape<N>::E;
  static constexpr int TPF = FftShape<N>::TPF;
};

// Blocks are dealt to the 8 XCDs round-robin; map them so that the tiles one
// XCD works on are adjacent (tiles that share cache lines share an L2).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  return (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
}

__device__ __forceinline__ double inv_symbol(const Geom& g, double kx, double ky) {
  return recip_pos(g.m0 + g.m1 * (kx * kx + ky * ky));
}

// Weight of a half-spectrum column in a physical inner product:
// column 0 carries kx = 0 and the Nyquist column once, others stand for +-kx.
__device__ __forceinline__ double col_weight(int col) { return col == 0 ? 1.0 : 2.0; }

#define COL_SETUP(N)                                         \
  constexpr int E = Col<N>::E;                               \
  constexpr int TPF = Col<N>::TPF;                           \
  extern __shared__ cplx lds[];                              \
  const int c = threadIdx.x;                                 \
  const int t = threadIdx.y;                                 \
  const ColMap map{(int)blockDim.x};                         \
  const int col = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + c; \
  const bool valid = col < g.nh;                             \
  cplx* buf = lds + c;                                       \
  TwiddleSet<N> twy;                                         \
  gather_twiddles<N>(twy, t, TWY(g));                         \
  (void)valid;

// 2D spectra (the Krylov basis, sigma_hat, the residual and the guess
// increments) are only touched by column passes and are stored column-major,
// [nx/2][ny], so that a column pass reads and writes them contiguously; x-half
// spectra, which the row passes produce and consume, stay row-major [ny][nx/2].
__device__ __forceinline__ size_t sidx(const Geom& g, int p, int col) { return (size_t)col * g.ny + p; }

template <int N>
__device__ __forceinline__ void load_spec(cplx* v, const cplx* __restrict__ S, int col, int t, bool valid) {
#pragma unroll
  for (int r = 0; r < Col<N>::E; ++r)
    v[r] = valid ? S[(size_t)col * N + t + r * Col<N>::TPF] : make_cplx(0.0, 0.0);
}

template <int N>
__device__ __forceinline__ void store_spec(const cplx* v, cplx* __restrict__ S, int col, int t, bool valid) {
  if (!valid) return;
#pragma unroll
  for (int r = 0; r < Col<N>::E; ++r) S[(size_t)col * N + t + r * Col<N>::TPF] = v[r];
}

template <int N>
__device__ __forceinline__ void load_col(cplx* v, const cplx* __restrict__ S, int nh, int col, int t, bool valid) {
#pragma unroll
  for (int r = 0; r < Col<N>::E; ++r) {
    const int p = t + r * Col<N>::TPF;
    v[r] = valid ? S[(size_t)p * nh + col] : make_cplx(0.0, 0.0);
  }
}

template <int N>
__device__ __forceinline__ void store_col(const cplx* v, cplx* __restrict__ S, int nh, int col, int t, bool valid) {
  if (!valid) return;
#pragma unroll
  for (int r = 0; r < Col<N>::E; ++r) {
    const int p = t + r * Col<N>::TPF;
    S[(size_t)p * nh + col] = v[r];
  }
}

// x-half spectra Ein -> 2D spectrum SIG (forward y-DFT) and G = F_y^-1(i ky SIG)
template <int N>
__global__ void __launch_bounds__(512) k_col_fwd_eg(Geom g, const cplx* __restrict__ Ein, cplx* __restrict__ SIG,
                                                     cplx* __restrict__ Gout) {
  Ein = mshift(g, Ein); SIG = mshift(g, SIG); Gout = mshift(g, Gout);
  COL_SETUP(N)
  cplx v[E];
  load_col<N>(v, Ein, g.nh, col, t, valid);
  fft<N, false, decltype(map)>(v, buf, t, twy, map);
  store_spec<N>(v, SIG, col, t, valid);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = mul_ik(v[r], wavenumber(t + r * TPF, N, g.inv_Ly) * g.inv_ny);
  fft<N, true, decltype(map)>(v, buf, t, twy, map);
  store_col<N>(v, Gout, g.nh, col, t, valid);
}

// Inverse y-transforms of a 2D spectrum x: E = F_y^-1 x, G = F_y^-1 (i ky x).
template <int N>
__device__ __forceinline__ void col_emit_eg(Geom& g, cplx* v, cplx* buf, int t, int col, bool valid,
                                            cplx* __restrict__ Eo, cplx* __restrict__ Go, const TwiddleSet<N>& twy) {
  constexpr int E = Col<N>::E, TPF = Col<N>::TPF;
  const ColMap map{(int)blockDim.x};
  cplx u[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    u[r] = mul_ik(v[r], wavenumber(t + r * TPF, N, g.inv_Ly) * g.inv_ny);
    v[r] = cscale(v[r], g.inv_ny);
  }
  fft<N, true, decltype(map)>(v, buf, t, twy, map);
  store_col<N>(v, Eo, g.nh, col, t, valid);
  fft<N, true, decltype(map)>(u, buf, t, twy, map);
  store_col<N>(u, Go, g.nh, col, t, valid);
}

// Arnoldi: V_j = (W - sum_{i<j} s2_i V_i) / beta, then E, G of V_j.
template <int N>
__global__ void __launch_bounds__(512) k_col_basis_eg(Geom g, const cplx* __restrict__ W, cplx* __restrict__ V,
                                                       size_t vstride, int j, GmresState* st, cplx* __restrict__ Eo,
                                                       cplx* __restrict__ Go, const double* __restrict__ pin,
                                                       int nbin) {
  W = mshift(g, W); V = mshift(g, V); st = mshift(g, st); Eo = mshift(g, Eo); Go = mshift(g, Go);
  pin = mshift(g, pin);
  if (status_load(st)) return;
  __shared__ double coef[kMaxRestart + 1];
  double beta = st->beta;  // j = 0: the residual norm
  if (j > 0 && cgs2_finish(g, st, j - 1, pin, nbin, coef, beta, blockIdx.x == 0)) return;
  COL_SETUP(N)
  const double ib = 1.0 / beta;
  // V_j = (W - sum_i c_i V_i) / beta at all of the thread's points, KB basis
  // vectors at a time (for each point the terms are subtracted in the order
  // i = 0, 1, ...)
  constexpr int KB = N <= 512 ? 2 : 1;
  cplx v[E];
  size_t idx[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    idx[r] = sidx(g, t + r * TPF, col);
    v[r] = valid ? W[idx[r]] : make_cplx(0.0, 0.0);
  }
  if (valid) {
    for (int i0 = 0; i0 < j; i0 += KB) {
      cplx b[KB][E];
#pragma unroll
      for (int q = 0; q < KB; ++q)
#pragma unroll
        for (int r = 0; r < E; ++r)
          b[q][r] = i0 + q < j ? V[(i0 + q) * vstride + idx[r]] : make_cplx(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < KB; ++q) {
        const double c = i0 + q < j ? coef[i0 + q] : 0.0;
#pragma unroll
        for (int r = 0; r < E; ++r) {
          v[r].x -= c * b[q][r].x;
          v[r].y -= c * b[q][r].y;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
      v[r] = cscale(v[r], ib);
      V[j * vstride + idx[r]] = v[r];
    }
  }
  col_emit_eg<N>(g, v, buf, t, col, valid, Eo, Go, twy);
}

// Two-chain variants of the Arnoldi column passes: threadIdx.z selects the
// chain; each chain has its own LDS region of tc x N.
#define COL2_SETUP_NOTW(N)                                   \
  constexpr int E = Col<N>::E;                               \
  constexpr int TPF = Col<N>::TPF;                           \
  extern __shared__ cplx lds[];                              \
  const int c = threadIdx.x;                                 \
  const int t = threadIdx.y;                                 \
  const int chain = threadIdx.z;                             \
  const ColMap map{(int)blockDim.x};                         \
  const int col = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + c; \
  const bool valid = col < g.nh;                             \
  cplx* buf = lds + chain * (blockDim.x * N) + c;
#define COL2_SETUP(N)                                        \
  COL2_SETUP_NOTW(N)                                         \
  TwiddleSet<N> twy;                                         \
  gather_twiddles<N>(twy, t, TWY(g));

// Same result as k_col_basis_eg: V_j = (W - sum_{i<j} s2_i V_i) / beta and
// its inverse y-transforms E (chain 0) and G (chain 1) computed concurrently.
template <int N>
__global__ void __launch_bounds__(1024) k_col_basis2(Geom g, const cplx* __restrict__ W, cplx* __restrict__ V,
                                                     size_t vstride, int j, GmresState* st, cplx* __restrict__ Eo,
                                                     cplx* __restrict__ Go, const double* __restrict__ pin,
                                                     int nbin) {
  W = mshift(g, W); V = mshift(g, V); st = mshift(g, st); Eo = mshift(g, Eo); Go = mshift(g, Go);
  pin = mshift(g, pin);
  if (status_load(st)) return;
  __shared__ double coef[kMaxRestart + 1];
  double beta = st->beta;  // j = 0: the residual norm
  if (j > 0 && cgs2_finish(g, st, j - 1, pin, nbin, coef, beta, blockIdx.x == 0)) return;
  COL2_SETUP(N)
  const double ib = 1.0 / beta;
  cplx v[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = t + r * TPF;
    const size_t idx = sidx(g, p, col);
    cplx x = make_cplx(0.0, 0.0);
    if (valid) {
      x = W[idx];
      for (int i0 = 0; i0 < j; i0 += 4) {
        cplx b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) b[q] = i0 + q < j ? V[(i0 + q) * vstride + idx] : make_cplx(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double cf = i0 + q < j ? coef[i0 + q] : 0.0;
          x.x -= cf * b[q].x;
          x.y -= cf * b[q].y;
        }
      }
      x = cscale(x, ib);
      if (chain == 0) V[j * vstride + idx] = x;
    }
    v[r] = chain == 0 ? cscale(x, g.inv_ny) : mul_ik(x, wavenumber(p, N, g.inv_Ly) * g.inv_ny);
  }
  fft<N, true, ColMap>(v, buf, t, twy, map);
  store_col<N>(v, chain == 0 ? Eo : Go, g.nh, col, t, valid);
}

// Same result as k_col_precond_dot: chain 0 transforms P, chain 1 transforms
// Q (times -i ky); w = (sum) / M is formed through LDS and each chain then
// owns half of the thread's positions for the store and the projections.
template <int N, bool SF>
__global__ void __launch_bounds__(1024) k_col_precond_dot2(Geom g, const cplx* __restrict__ P,
                                                           const cplx* __restrict__ Q, const cplx* __restrict__ V,
                                                           size_t vstride, int j, const GmresState* st,
                                                           cplx* __restrict__ W, double* partials) {
  P = mshift(g, P); Q = mshift(g, Q); V = mshift(g, V); st = mshift(g, st); W = mshift(g, W);
  partials = mshift(g, partials);
  if (SF && st->st.done) return;
  COL2_SETUP(N)
  __shared__ double red[(kMaxRestart + 1) * 16];
  cplx v[E];
  load_col<N>(v, chain == 0 ? P : Q, g.nh, col, t, valid);
  if (st->st.done) return;  // tested after the (in-bounds) loads are issued
  fft<N, false, ColMap>(v, buf, t, twy, map);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    if (chain == 1) v[r] = mul_ik(v[r], -wavenumber(t + r * TPF, N, g.inv_Ly));
    buf[map.at(t + r * TPF)] = v[r];
  }
  __syncthreads();
  const cplx* b0 = lds + c;
  const cplx* b1 = lds + blockDim.x * N + c;
  const double kx = col * g.inv_Lx;
  constexpr int EH = E / 2;
  cplx w[EH];
#pragma unroll
  for (int q = 0; q < EH; ++q) {
    const int p = t + (chain * EH + q) * TPF;
    w[q] = cscale(cadd(b0[map.at(p)], b1[map.at(p)]), inv_symbol(g, kx, wavenumber(p, N, g.inv_Ly)));
    if (valid) W[sidx(g, p, col)] = w[q];
  }
  const double wt = valid ? col_weight(col) : 0.0;
  for (int i0 = 0; i0 <= j; i0 += 8) {
    double a[8];
#pragma unroll
    for (int q8 = 0; q8 < 8; ++q8) {
      double d = 0.0;
      if (valid && i0 + q8 <= j) {
#pragma unroll
        for (int q = 0; q < EH; ++q) {
          const int p = t + (chain * EH + q) * TPF;
          const cplx b = V[(i0 + q8) * vstride + sidx(g, p, col)];
          d += cdot(b, w[q]);
        }
      }
      a[q8] = wt * d;
    }
    wave_partials8(a, red, i0, j + 1);
  }
  block_partials_out(red, j + 1, partials, nullptr);  // reduced by the update kernel
}

// Three-kernel Arnoldi step (kernels A, B, C), one pass over the basis each.
// Orthogonalisation is classical Gram-Schmidt with the projection
// coefficients corrected by the Gram matrix of the stored basis,
// c = (2I - G) s with s = V^T w and G = V^T V (the first-order form of
// G^{-1} s); this removes the loss of orthogonality that a second CGS pass
// would remove, without a second pass over the basis.
//   A_j: c = (2I - G) s from the block partials of C_{j-1};
//        u_j = w_{j-1} - sum_{i<j} c_i V_i, partials of ||u_j||^2;
//        E = F_y^-1 u_j, G = F_y^-1 (i ky u_j)
//   B_j: finish step j-1 from the partials of A_j (H(:, j-1) = c,
//        H(j, j-1) = ||u_j||, Givens update, stop test); then the x part
//        of the operator on (E, G)                       (k_row_matvec3)
//   C_j: z = M^-1 F(L u_j);  V_j = u_j / beta_j,  w_j = z / beta_j;
//        partials of s_i = <V_i, w_j>, G_ij = <V_i, V_j>, i <= j.
// No kernel ends in a single-block reduction: the next kernel on the stream
// finishes it in every block (identically, in a fixed order), with block 0
// storing the result, so the serial reduction and the GMRES scalar work no
// longer idle the GPU at the end of a kernel.  (A single finishing block in B
// would let the other blocks run a useless transform on the stopping step,
// which costs more than the short prologue.)
// The same Krylov basis, Hessenberg matrix and iterates as modified or
// twice-iterated classical Gram-Schmidt, in exact arithmetic.

// Finish the projections of C_jc in a block of the following kernel A:
// s_i = <V_i, w_jc> and column jc of the Gram matrix from the nb block
// partials pin, then c = (2I - G) s into coef (LDS), i <= jc.  write: this
// block stores s, the new row and column of G and c.  The other blocks read
// only the Gram entries of earlier steps, which this step does not change.
__device__ bool cgs_coefficients(const Geom& g, GmresState* st, int jc, const double* pin, int nb, double* outv,
                                 double* coef, bool write, double& beta, int done) {
  const int tid = flat_tid(), nthr = block_threads();
  constexpr int ld = kMaxRestart + 1;
  // G_ik, i, k < jc, from earlier steps: for jc <= kPreG staged in LDS,
  // loaded before the partials so that both loads wait together
  constexpr int kPreG = 20;
  __shared__ double sG[kPreG * kPreG];
  const bool pre = jc <= kPreG;
  const int ng = pre ? jc * jc : 0;
  double gq[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = tid + u * nthr;
    gq[u] = e < ng ? st->G[(e / jc) * ld + e % jc] : 0.0;
  }
  reduce_partials<false, 4>(pin, nb, 2 * (jc + 1) + 1, nullptr, outv);
  // the GMRES status (read by the caller before these loads were issued,
  // uniform over the block): a stopped cycle writes nothing
  if (done) return false;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = tid + u * nthr;
    if (e < ng) sG[e] = gq[u];
  }
  for (int e = tid + 2 * nthr; e < ng; e += nthr) sG[e] = st->G[(e / jc) * ld + e % jc];
  for (int i = tid; i < 2 * (jc + 1) + 1; i += nthr) outv[i] *= g.inv_n;
  __syncthreads();
  // c_i = 2 s_i - sum_k G_ik s_k; G_ik, k < jc, from earlier steps, and
  // G_{i,jc} = <V_i, V_jc> from this reduction
  for (int i = tid; i <= jc; i += nthr) {
    double acc = 0.0;
    for (int k = 0; k < jc; ++k)
      acc += (i == jc ? outv[2 * k + 1] : (pre ? sG[i * jc + k] : st->G[i * ld + k])) * outv[2 * k];
    acc += outv[2 * i + 1] * outv[2 * jc];
    coef[i] = 2.0 * outv[2 * i] - acc;
  }
  __syncthreads();
  // H(jc+1, jc) = ||u|| with u = w - V c: ||u||^2 = ||w||^2 - 2 c.s + c^T G c
  // (G the Gram matrix of V_0..V_jc), without a pass over u
  __shared__ double gc[kMaxRestart + 1];
  __shared__ double sh_beta;
  for (int i = tid; i <= jc; i += nthr) {
    double acc = 0.0;
    for (int k = 0; k <= jc; ++k) {
      const double gik = k == jc ? outv[2 * i + 1]
                                 : (i == jc ? outv[2 * k + 1] : (pre ? sG[i * jc + k] : st->G[i * ld + k]));
      acc += gik * coef[k];
    }
    gc[i] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    const double w2 = outv[2 * (jc + 1)];
    double q = w2;
    for (int i = 0; i <= jc; ++i) q += coef[i] * (gc[i] - 2.0 * outv[2 * i]);
    // the identity cancels ||w||^2 down to ||u||^2, so its rounding error is
    // about eps ||w||^2 with the eps of the stored vectors; below kGramCut
    // ||w||^2 it no longer fixes ||u|| well enough (FP64: to 1e-6 relative
    // or better above 1e-10; FP32, where u is stored in float and differs
    // from the identity's u by about eps32 ||w||: to 6e-5 above 1e-6): -1
    // tells the caller so
    constexpr double kGramCut = SGN_PREC == 32 ? 1e-6 : 1e-10;
    sh_beta = q > kGramCut * w2 ? sqrt(q) : -1.0;
  }
  __syncthreads();
  beta = sh_beta;
  if (write) {
    for (int i = tid; i <= jc; i += nthr) {
      st->s[i] = outv[2 * i];
      st->G[i * ld + jc] = outv[2 * i + 1];
      st->G[jc * ld + i] = outv[2 * i + 1];
      st->cproj[i] = coef[i];
    }
  }
  return true;
}

// Kernel A's pass over the basis: vectors loaded per batch (BATCH; _E8 for
// transforms of eight values per thread, which hold twice the registers);
// waves per SIMD the kernel is compiled for at lengths <= 1024 (96 VGPRs at
// 5, two of them spilled at 512 points).  Measured on nine 1024x512
// members: batches of 4 and 8 take the same time; 5 waves 62.4 us per
// launch against 62.9 at 4.
#ifndef SGN_PROJ_BATCH
#define SGN_PROJ_BATCH 4
#endif
#ifndef SGN_PROJ_WAVES_SHORT
#define SGN_PROJ_WAVES_SHORT 5
#endif
#ifndef SGN_PROJ_BATCH_E8
#define SGN_PROJ_BATCH_E8 2
#endif

// Kernel A (j >= 1; the residual pass does step 0's).  win: w_{j-1}; u_j ->
// W.  pin: the block partials of C_{j-1} (same grid).  Every block first
// finishes Arnoldi step j - 1 from them (projection coefficients, H(j, j-1)
// by the Gram identity, Givens update and test; block 0 stores the step)
// and exits if the cycle stops there, so the last step costs no pass.
template <int N, bool SF>
__global__ void __launch_bounds__(1024, N <= 1024 ? SGN_PROJ_WAVES_SHORT : 4) k_col_proj(Geom g, const cplx* win, cplx* W, const cplx* __restrict__ V,
                                                   size_t vstride, int j, GmresState* st, cplx* __restrict__ Eo,
                                                   cplx* __restrict__ Go,
                                                   const double* __restrict__ pin) {
  win = mshift(g, win); W = mshift(g, W); V = mshift(g, V); st = mshift(g, st); Eo = mshift(g, Eo);
  Go = mshift(g, Go); pin = mshift(g, pin);
  if (SF && status_load(st)) return;
  // tested once the loads of the prologue are in flight; block 0 of this
  // launch may store it meanwhile (status_load)
  const int done = status_load(st);
  __shared__ double coef[kMaxRestart + 1];
  __shared__ double outv[2 * (kMaxRestart + 1) + 1];
  // w_{j-1} at this thread's points, loaded before the prologue (it does not
  // depend on the coefficients), so that its loads overlap the reduction
  constexpr int EH = Col<N>::E / 2;
  cplx u[EH];
  size_t uidx[EH];
  {
    const int col0 = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
#pragma unroll
    for (int q = 0; q < EH; ++q) {
      uidx[q] = sidx(g, threadIdx.y + (threadIdx.z * EH + q) * Col<N>::TPF, col0);
      u[q] = col0 < g.nh ? win[uidx[q]] : make_cplx(0.0, 0.0);
    }
  }
  {
    const FinishPre pre = finish_prefetch(st, j - 1, false);
    double beta;
    if (!cgs_coefficients(g, st, j - 1, pin, gridDim.x, outv, coef, blockIdx.x == 0, beta, done)) return;
    // a new direction too small for the Gram identity to measure: close the
    // cycle on the columns so far (H(j, j-1) = 0) and restart, so that
    // convergence is judged on a freshly computed residual
    const bool unsure = beta < 0.0;
    if (gmres_finish_column(st, j - 1, coef, unsure ? 0.0 : beta, nullptr, blockIdx.x == 0, &pre, unsure)) return;
  }
  COL2_SETUP_NOTW(N)
  // u_j = w_{j-1} - sum_i c_i V_i, KA basis vectors at a time at all of the
  // thread's points; the transform's twiddles are gathered after this pass,
  // so that their registers hold loads in flight during it
  constexpr int KA = E >= 8 ? SGN_PROJ_BATCH_E8 : SGN_PROJ_BATCH;
  if (valid) {
    for (int i0 = 0; i0 < j; i0 += KA) {
      cplx b[KA][EH];
#pragma unroll
      for (int k = 0; k < KA; ++k)
#pragma unroll
        for (int q = 0; q < EH; ++q)
          b[k][q] = i0 + k < j ? V[(i0 + k) * vstride + uidx[q]] : make_cplx(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < KA; ++k) {
        const double cf = i0 + k < j ? coef[i0 + k] : 0.0;
#pragma unroll
        for (int q = 0; q < EH; ++q) {
          u[q].x -= cf * b[k][q].x;
          u[q].y -= cf * b[k][q].y;
        }
      }
    }
  }
  TwiddleSet<N> twy;
  gather_twiddles<N>(twy, t, TWY(g));
  __syncthreads();  // every read of win (which may alias W) is done
#pragma unroll
  for (int q = 0; q < EH; ++q)
    if (valid) W[sidx(g, t + (chain * EH + q) * TPF, col)] = u[q];
  // gather all E positions of u for this chain's transform
  cplx* U = lds + c;  // chain 0's region, free until its transform
#pragma unroll
  for (int q = 0; q < EH; ++q) U[map.at(t + (chain * EH + q) * TPF)] = u[q];
  __syncthreads();
  cplx v[E];
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = U[map.at(t + r * TPF)];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < E; ++r)
    v[r] = chain == 0 ? cscale(v[r], g.inv_ny) : mul_ik(v[r], wavenumber(t + r * TPF, N, g.inv_Ly) * g.inv_ny);
  fft<N, true, ColMap>(v, buf, t, twy, map);
  store_col<N>(v, chain == 0 ? Eo : Go, g.nh, col, t, valid);
}

// Kernel C.  P, Q: x-part outputs of B_j for u_j; W: u_j; writes V_j and
// w_j (into Wn) and the block partials of the projections s and of the Gram
// column.
template <int N, bool SF>
__global__ void __launch_bounds__(1024) k_col_precond_new(Geom g, const cplx* __restrict__ P,
                                                          const cplx* __restrict__ Q, const cplx* __restrict__ W,
                                                          cplx* __restrict__ V, cplx* __restrict__ Wn, size_t vstride,
                                                          int j, const GmresState* st, double* partials) {
  P = mshift(g, P); Q = mshift(g, Q); W = mshift(g, W); V = mshift(g, V); Wn = mshift(g, Wn);
  st = mshift(g, st); partials = mshift(g, partials);
  if (SF && st->st.done) return;
  COL2_SETUP(N)
  __shared__ double red[(2 * (kMaxRestart + 1) + 1) * 16];
  cplx v[E];
  load_col<N>(v, chain == 0 ? P : Q, g.nh, col, t, valid);
  if (st->st.done) return;  // tested after the loads are issued (they are in bounds whatever the state)
  const double ib = 1.0 / st->beta;
  fft<N, false, ColMap>(v, buf, t, twy, map);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    if (chain == 1) v[r] = mul_ik(v[r], -wavenumber(t + r * TPF, N, g.inv_Ly));
    buf[map.at(t + r * TPF)] = v[r];
  }
  __syncthreads();
  const cplx* b0 = lds + c;
  const cplx* b1 = lds + blockDim.x * N + c;
  const double kx = col * g.inv_Lx;
  constexpr int EH = E / 2;
  cplx vj[EH], wj[EH];
#pragma unroll
  for (int q = 0; q < EH; ++q) {
    const int p = t + (chain * EH + q) * TPF;
    const size_t idx = sidx(g, p, col);
    const cplx z = cscale(cadd(b0[map.at(p)], b1[map.at(p)]), inv_symbol(g, kx, wavenumber(p, N, g.inv_Ly)));
    vj[q] = make_cplx(0.0, 0.0);
    wj[q] = make_cplx(0.0, 0.0);
    if (valid) {
      vj[q] = cscale(W[idx], ib);
      wj[q] = cscale(z, ib);
      V[j * vstride + idx] = vj[q];
      Wn[idx] = wj[q];
    }
  }
  // values 2i: <V_i, w_j>, 2i+1: <V_i, V_j>, i <= j (one pass over V)
  const double wt = valid ? col_weight(col) : 0.0;
  const int nv = 2 * (j + 1);
  double dsj = 0.0, dgj = 0.0;  // the i = j terms, from registers
#pragma unroll
  for (int q = 0; q < EH; ++q) {
    dsj += cdot(vj[q], wj[q]);
    dgj += cnorm2(vj[q]);
  }
  size_t pidx[EH];
#pragma unroll
  for (int q = 0; q < EH; ++q) pidx[q] = sidx(g, t + (chain * EH + q) * TPF, col);
  for (int i0 = 0; i0 <= j; i0 += 4) {
    double a[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = i0 + k;
      double ds = 0.0, dg = 0.0;
      if (valid && i < j) {
#pragma unroll
        for (int q = 0; q < EH; ++q) {
          const cplx b = V[i * vstride + pidx[q]];
          ds += cdot(b, wj[q]);
          dg += cdot(b, vj[q]);
        }
      } else if (i == j) {
        ds = dsj;
        dg = dgj;
      }
      a[2 * k] = wt * ds;
      a[2 * k + 1] = wt * dg;
    }
    wave_partials8(a, red, 2 * i0, nv);
  }
  // value 2 (j + 1): ||w_j||^2, for H(j+1, j) by the Gram identity
  double nw2 = 0.0;
#pragma unroll
  for (int q = 0; q < EH; ++q) nw2 += cnorm2(wj[q]);
  wave_partial(wt * nw2, red, nv);
  block_partials_out(red, nv + 1, partials, nullptr);  // finished by A_{j+1}
}

// sigma_hat += sum_{i<k} y_i V_i (or 0 when b == 0), then E, G of sigma_hat.
// D (optional): the stage increment of the extrapolated guess, D += (new -
// old sigma_hat), so that over a solve D collects sigma - guess.  spec & 1: a
// launch enqueued before the host knew the outcome of the solve; it does
// nothing unless the solve has converged.  spec & 4 (captured steps, one
// grid): thread 0 of block 0 adds the solve to the captured-step counters
// (anything but convergence counts as a failure: one GMRES cycle per solve
// there) and sets the iteration cap of the next solve to spec >> 16.
template <int N>
__global__ void __launch_bounds__(512) k_col_update_eg(Geom g, cplx* __restrict__ SIG, const cplx* __restrict__ V,
                                                        size_t vstride, GmresState* __restrict__ st,
                                                        cplx* __restrict__ Eo, cplx* __restrict__ Go,
                                                        cplx* __restrict__ D, int spec) {
  SIG = mshift(g, SIG); V = mshift(g, V); st = mshift(g, st); Eo = mshift(g, Eo); Go = mshift(g, Go);
  D = mshift(g, D);
  COL_SETUP(N)
  __shared__ double coef[kMaxRestart];
  const int tid = flat_tid();
  // the status, all the coefficient slots and sigma are loaded together (in
  // bounds whatever the status); the speculative launch's test follows
  const int done = st->st.done, k = st->st.jdone, zero = st->st.zero, cyc = st->st.cyc;
  for (int i = tid; i < kMaxRestart; i += block_threads()) coef[i] = st->y[i];
  if ((spec & 4) && blockIdx.x == 0 && tid == 0) {
    const int it = st->st.total_iters;
    st->st.g_total += it;
    if (it > st->st.g_max) st->st.g_max = it;
    if (done != 1) st->st.g_fail += 1;
    st->maxit = spec >> 16;
  }
  cplx sg[E];
#pragma unroll
  for (int r = 0; r < E; ++r) sg[r] = valid ? SIG[sidx(g, t + r * TPF, col)] : make_cplx(0.0, 0.0);
  if ((spec & 1) && done != 1) return;
  // spec & 2: an ensemble update after cycle round spec >> 8, for the members
  // that ran a cycle in that round only
  if ((spec & 2) && cyc != (spec >> 8)) return;
  __syncthreads();
  // sigma_hat + V y at all of the thread's points, KB basis vectors at a time
  // (for each point the terms are added in the order i = 0, 1, ...); one at a
  // time for longer columns, whose threads hold more points
  constexpr int KB = N <= 512 ? 2 : 1;
  cplx v[E], old[E];
  size_t idx[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    idx[r] = sidx(g, t + r * TPF, col);
    old[r] = (valid && (D || !zero)) ? sg[r] : make_cplx(0.0, 0.0);
    v[r] = (valid && !zero) ? old[r] : make_cplx(0.0, 0.0);
  }
  if (valid && !zero) {
    for (int i0 = 0; i0 < k; i0 += KB) {
      cplx b[KB][E];
#pragma unroll
      for (int q = 0; q < KB; ++q)
#pragma unroll
        for (int r = 0; r < E; ++r)
          b[q][r] = i0 + q < k ? V[(i0 + q) * vstride + idx[r]] : make_cplx(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < KB; ++q) {
        const double c = i0 + q < k ? coef[i0 + q] : 0.0;
#pragma unroll
        for (int r = 0; r < E; ++r) {
          v[r].x += c * b[q][r].x;
          v[r].y += c * b[q][r].y;
        }
      }
    }
  }
  if (valid) {
#pragma unroll
    for (int r = 0; r < E; ++r) {
      SIG[idx[r]] = v[r];
      if (D) D[idx[r]] = cadd(D[idx[r]], csub(v[r], old[r]));
    }
  }
  col_emit_eg<N>(g, v, buf, t, col, valid, Eo, Go, twy);
}

// Extrapolated initial guess of an RK stage: sigma_hat += D (the increment
// this stage had over the previous one in the last step), then E, G.
template <int N>
__global__ void __launch_bounds__(512) k_col_guess_eg(Geom g, cplx* __restrict__ SIG, const cplx* __restrict__ D,
                                                       cplx* __restrict__ Eo, cplx* __restrict__ Go) {
  SIG = mshift(g, SIG); D = mshift(g, D); Eo = mshift(g, Eo); Go = mshift(g, Go);
  COL_SETUP(N)
  cplx v[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const size_t idx = sidx(g, t + r * TPF, col);
    cplx x = make_cplx(0.0, 0.0);
    if (valid) {
      x = cadd(SIG[idx], D[idx]);
      SIG[idx] = x;
    }
    v[r] = x;
  }
  col_emit_eg<N>(g, v, buf, t, col, valid, Eo, Go, twy);
}

// F_y(P) - i ky F_y(Q) for the tile; P, Q are x-half spectra (Q may be null).
template <int N>
__device__ __forceinline__ void col_combine(Geom& g, cplx* v, cplx* buf, int t, int col, bool valid,
                                            const cplx* __restrict__ P, const cplx* __restrict__ Q,
                                            const TwiddleSet<N>& twy) {
  constexpr int E = Col<N>::E, TPF = Col<N>::TPF;
  const ColMap map{(int)blockDim.x};
  cplx u[E];
  load_col<N>(v, P, g.nh, col, t, valid);
  if (Q != nullptr) load_col<N>(u, Q, g.nh, col, t, valid);
  fft<N, false, decltype(map)>(v, buf, t, twy, map);
  if (Q == nullptr) return;  // second term absent (an explicit b has no y part)
  fft<N, false, decltype(map)>(u, buf, t, twy, map);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = csub(v[r], mul_ik(u[r], wavenumber(t + r * TPF, N, g.inv_Ly)));
}


// Arnoldi: w = M^-1 F(L V_j) (= (F_y P - i ky F_y Q) / M), s_i = <V_i, w>, i <= j.
template <int N>
__global__ void __launch_bounds__(512) k_col_precond_dot(Geom g, const cplx* __restrict__ P,
                                                          const cplx* __restrict__ Q, const cplx* __restrict__ V,
                                                          size_t vstride, int j, const GmresState* st,
                                                          cplx* __restrict__ W, double* partials) {
  P = mshift(g, P); Q = mshift(g, Q); V = mshift(g, V); st = mshift(g, st); W = mshift(g, W);
  partials = mshift(g, partials);
  if (st->st.done) return;
  COL_SETUP(N)
  __shared__ double red[(kMaxRestart + 1) * 16];
  cplx v[E];
  col_combine<N>(g, v, buf, t, col, valid, P, Q, twy);
  const double kx = col * g.inv_Lx;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = t + r * TPF;
    v[r] = cscale(v[r], inv_symbol(g, kx, wavenumber(p, N, g.inv_Ly)));
  }
  store_spec<N>(v, W, col, t, valid);
  const double wt = valid ? col_weight(col) : 0.0;
  for (int i0 = 0; i0 <= j; i0 += 8) {
    double a[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double d = 0.0;
      if (valid && i0 + q <= j) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const int p = t + r * TPF;
          const cplx b = V[(i0 + q) * vstride + sidx(g, p, col)];
          d += cdot(b, v[r]);
        }
      }
      a[q] = wt * d;
    }
    wave_partials8(a, red, i0, j + 1);
  }
  block_partials_out(red, j + 1, partials, nullptr);  // reduced by the update kernel
}

// Start of a GMRES cycle: r = M^-1 (b - L sigma) with F(b - L sigma) =
// F_y(P) - i ky F_y(Q).  With need_b, b_hat = F_y(R1) - i ky F_y(R2) gives
// beta0 = ||M^-1 b|| and ||b||.  flags: 1 = new solve (reset the counters),
// 2 = report the unpreconditioned residual only (no cycle set-up).
template <int N>
__global__ void __launch_bounds__(512, N <= 1024 ? 4 : 2) k_col_resid(Geom g, const cplx* __restrict__ P, const cplx* __restrict__ Q,
                                                    const cplx* __restrict__ R1, const cplx* __restrict__ R2,
                                                    int need_b, int flags, GmresState* st, cplx* __restrict__ W,
                                                    double* partials, int nblocks, cplx* __restrict__ Eo,
                                                    cplx* __restrict__ Go) {
  P = mshift(g, P); Q = mshift(g, Q); R1 = mshift(g, R1); R2 = mshift(g, R2); st = mshift(g, st);
  W = mshift(g, W); partials = mshift(g, partials); Eo = mshift(g, Eo); Go = mshift(g, Go);
  // flags & 4: an ensemble restart, run only for the members that restart
  // (each block reads the status before any block of the member takes a
  // ticket, and only the last block rewrites it)
  if ((flags & 4) && !restart_due(st)) return;
  COL_SETUP(N)
  __shared__ double red[3 * 16];
  __shared__ double outv[3];
  const bool true_only = (flags & 2) != 0;
  cplx v[E];
  col_combine<N>(g, v, buf, t, col, valid, P, Q, twy);
  const double kx = col * g.inv_Lx;
  const double wt = valid ? col_weight(col) : 0.0;
  double nr = 0.0;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = t + r * TPF;
    if (!true_only) v[r] = cscale(v[r], inv_symbol(g, kx, wavenumber(p, N, g.inv_Ly)));
    nr += cnorm2(v[r]);
  }
  if (!true_only) store_spec<N>(v, W, col, t, valid);
  wave_partial(wt * nr, red, 0);
  if (Eo) {
    // the start of the three-kernel Arnoldi cycle (kernel A of step 0):
    // E = F_y^-1 r / ny and G = F_y^-1 (i ky r) / ny of the residual r
    cplx u[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      u[r] = mul_ik(v[r], wavenumber(t + r * TPF, N, g.inv_Ly) * g.inv_ny);
      v[r] = cscale(v[r], g.inv_ny);
    }
    fft<N, true, decltype(map)>(v, buf, t, twy, map);
    store_col<N>(v, Eo, g.nh, col, t, valid);
    fft<N, true, decltype(map)>(u, buf, t, twy, map);
    store_col<N>(u, Go, g.nh, col, t, valid);
  }
  int nvals = 1;
  if (need_b) {
    col_combine<N>(g, v, buf, t, col, valid, R1, R2, twy);
    double nb = 0.0, nbm = 0.0;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int p = t + r * TPF;
      const double m = inv_symbol(g, kx, wavenumber(p, N, g.inv_Ly));
      const double a2 = cnorm2(v[r]);
      nb += a2;
      nbm += a2 * m * m;
    }
    wave_partial(wt * nbm, red, 1);
    wave_partial(wt * nb, red, 2);
    nvals = 3;
  }
  block_partials_out(red, nvals, partials, nullptr);
  if (last_block_arrive(st->ctr, nblocks)) {
    reduce_partials(partials, nblocks, nvals, nullptr, outv);
    if (flat_tid() == 0) {
      if (true_only) {
        st->st.true_resid2 = outv[0] * g.inv_n;
      } else {
        if (flags & 1) {
          st->st.total_iters = 0;
          st->st.zero = 0;
        }
        st->cycle_base = st->st.total_iters;
        st->st.cyc = flags >> 8;  // the host's cycle round (ensembles: which members' update runs)
        if (need_b) {
          st->st.beta0 = sqrt(outv[1] * g.inv_n);
          st->st.bnorm = sqrt(outv[2] * g.inv_n);
          st->st.zero = st->st.beta0 == 0.0 ? 1 : 0;
        }
        const double beta = sqrt(outv[0] * g.inv_n);
        st->beta = beta;
        st->gv[0] = beta;
        st->st.jdone = 0;
        st->st.resid = beta;
        st->st.done = (st->st.zero || beta <= st->tol * st->st.beta0) ? 1 : 0;
      }
    }
  }
}

// Inverse y-transform of a 2D spectrum: out = F_y^-1 S / ny.
template <int N>
__global__ void __launch_bounds__(512) k_col_inv(Geom g, const cplx* __restrict__ S, cplx* __restrict__ out) {
  S = mshift(g, S); out = mshift(g, out);
  COL_SETUP(N)
  cplx v[E];
  load_spec<N>(v, S, col, t, valid);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = cscale(v[r], g.inv_ny);
  fft<N, true, decltype(map)>(v, buf, t, twy, map);
  store_col<N>(v, out, g.nh, col, t, valid);
}

// Learned guess: from W = M^-1 r0_hat (the 2D spectrum the GMRES start forms)
// the x-half spectra of r0 (out_r = F_y^-1 (M W) / ny) and of M^-1 r0
// (out_m = F_y^-1 W / ny), for the x-inverse transforms that follow.
template <int N>
__global__ void __launch_bounds__(512) k_col_learn(Geom g, const cplx* __restrict__ W, cplx* __restrict__ out_r,
                                                    cplx* __restrict__ out_m) {
  COL_SETUP(N)
  cplx v[E], u[E];
  load_spec<N>(v, W, col, t, valid);
  const double kx = col * g.inv_Lx;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    u[r] = cscale(v[r], g.inv_ny / inv_symbol(g, kx, wavenumber(t + r * TPF, N, g.inv_Ly)));
    v[r] = cscale(v[r], g.inv_ny);
  }
  fft<N, true, decltype(map)>(v, buf, t, twy, map);
  store_col<N>(v, out_m, g.nh, col, t, valid);
  __syncthreads();
  fft<N, true, decltype(map)>(u, buf, t, twy, map);
  store_col<N>(u, out_r, g.nh, col, t, valid);
}

// Apply the 2D operator F(L s) (from P, Q) and optionally M^-1; out = 2D spectrum.
template <int N>
__global__ void __launch_bounds__(512) k_col_apply(Geom g, const cplx* __restrict__ P, const cplx* __restrict__ Q,
                                                    int precond, cplx* __restrict__ out) {
  P = mshift(g, P); Q = mshift(g, Q); out = mshift(g, out);
  COL_SETUP(N)
  cplx v[E];
  col_combine<N>(g, v, buf, t, col, valid, P, Q, twy);
  if (precond) {
    const double kx = col * g.inv_Lx;
#pragma unroll
    for (int r = 0; r < E; ++r)
      v[r] = cscale(v[r], inv_symbol(g, kx, wavenumber(t + r * TPF, N, g.inv_Ly)));
  }
  store_spec<N>(v, out, col, t, valid);
}

// x-half spectra -> multiplied by a 2D symbol -> x-half spectra.
//   op 0: M^-1 (preconditioner)
//   op 1: Krasny filter, zero modes with |X| / (nx ny) < thr
//   op 2: op 1, and also zero modes with 3 |m_x| > nx or 3 |m_y| > ny (the
//         two-thirds rule of Orszag, an option beyond the paper's scheme)
template <int N>
__global__ void __launch_bounds__(512) k_col_filter(Geom g, Trio io, int op, double thr) {
  const cplx* __restrict__ Sx = mshift(g, static_cast<const cplx*>(io.in[blockIdx.y]));
  cplx* __restrict__ out = mshift(g, static_cast<cplx*>(io.out[blockIdx.y]));
  COL_SETUP(N)
  cplx v[E];
  load_col<N>(v, Sx, g.nh, col, t, valid);
  fft<N, false, decltype(map)>(v, buf, t, twy, map);
  if (op == 0) {
    const double kx = col * g.inv_Lx;
#pragma unroll
    for (int r = 0; r < E; ++r)
      v[r] = cscale(v[r], inv_symbol(g, kx, wavenumber(t + r * TPF, N, g.inv_Ly)));
  } else {
    const double T = thr * (double)g.nx * (double)g.ny;
    const double T2 = T * T;
    const bool dealias = op == 2;
    // x index of this column (column 0 holds m_x = 0 and m_x = nx/2; the
    // latter is always outside the two-thirds band).
    const bool keep_x = !dealias || 3 * col <= g.nx;
    // column 0 packs two real-signal spectra (kx = 0 and kx = nx/2): split
    // them with the +-ky partner, threshold each, recombine.
#pragma unroll
    for (int r = 0; r < E; ++r) buf[map.at(t + r * TPF)] = v[r];
    __syncthreads();
    cplx partner[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int p = t + r * TPF;
      partner[r] = buf[map.at((N - p) & (N - 1))];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int p = t + r * TPF;
      const int my = p <= N / 2 ? p : N - p;
      const bool keep_y = !dealias || 3 * my <= N;
      if (col == 0) {
        const cplx z = v[r], zc = partner[r];
        cplx a = make_cplx(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));   // kx = 0 mode
        cplx b = make_cplx(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));  // kx = nx/2 mode
        if (!keep_y || a.x * a.x + a.y * a.y < T2) a = make_cplx(0.0, 0.0);
        if (dealias || b.x * b.x + b.y * b.y < T2) b = make_cplx(0.0, 0.0);
        v[r] = make_cplx(a.x - b.y, a.y + b.x);
      } else {
        if (!(keep_x && keep_y) || cnorm2(v[r]) < T2) v[r] = make_cplx(0.0, 0.0);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = cscale(v[r], g.inv_ny);
  fft<N, true, decltype(map)>(v, buf, t, twy, map);
  store_col<N>(v, out, g.nh, col, t, valid);
}

// Largest normalised 2D DFT coefficient with |mx| > nx/4 or |my| > ny/4.
template <int N>
__global__ void __launch_bounds__(512) k_col_tail(Geom g, const cplx* __restrict__ Sx, GmresState* st,
                                                   double* partials, int nblocks) {
  Sx = mshift(g, Sx); st = mshift(g, st); partials = mshift(g, partials);
  COL_SETUP(N)
  __shared__ double red[16];
  __shared__ double outv[1];
  cplx v[E];
  load_col<N>(v, Sx, g.nh, col, t, valid);
  fft<N, false, decltype(map)>(v, buf, t, twy, map);
#pragma unroll
  for (int r = 0; r < E; ++r) buf[map.at(t + r * TPF)] = v[r];
  __syncthreads();
  cplx partner[E];
#pragma unroll
  for (int r = 0; r < E; ++r) partner[r] = buf[map.at((N - (t + r * TPF)) & (N - 1))];
  __syncthreads();
  double mx = 0.0;
  if (valid) {
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int p = t + r * TPF;
      const int my = p <= N / 2 ? p : N - p;
      const bool yin = 4 * my > N;
      if (col == 0) {
        const cplx z = v[r], zc = partner[r];
        const cplx a = make_cplx(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));
        const cplx b = make_cplx(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));
        if (yin) mx = fmax(mx, sqrt(a.x * a.x + a.y * a.y));
        mx = fmax(mx, sqrt(b.x * b.x + b.y * b.y));  // kx = nx/2 is always outside nx/4
      } else if (yin || 4 * col > g.nx) {
        mx = fmax(mx, sqrt(cnorm2(v[r])));
      }
    }
  }
  const int* kinds = kKindsMax;
  {
    const int tid = flat_tid();
    const double m = wave_max(mx);
    if ((tid & 63) == 0) red[tid >> 6] = m;
  }
  block_partials_out(red, 1, partials, kinds);
  if (last_block_arrive(st->ctr, nblocks)) {
    reduce_partials(partials, nblocks, 1, kinds, outv);
    if (flat_tid() == 0) {
      st->st.red[7] = outv[0] * g.inv_n;
    }
  }
}

// out = d/dy f for a physical field (two real columns per complex column).
template <int N>
__global__ void __launch_bounds__(512) k_col_dy(Geom g, const real* __restrict__ f, real* __restrict__ out) {
  f = mshift(g, f); out = mshift(g, out);
  COL_SETUP(N)
  cplx v[E];
  load_col<N>(v, reinterpret_cast<const cplx*>(f), g.nh, col, t, valid);
  fft<N, false, decltype(map)>(v, buf, t, twy, map);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = mul_ik(v[r], wavenumber(t + r * TPF, N, g.inv_Ly) * g.inv_ny);
  fft<N, true, decltype(map)>(v, buf, t, twy, map);
  store_col<N>(v, reinterpret_cast<cplx*>(out), g.nh, col, t, valid);
}

// Fluxes, y part: dh = dhp - d_y qy, k_vy = -d_y B, through the RK combine.
template <int N>
__global__ void __launch_bounds__(512) k_col_flux(Geom g, const real* __restrict__ dhp, const real* __restrict__ qy,
                                                   const real* __restrict__ Bf, RkStage rk, RkField fh, RkField fvy) {
  dhp = mshift(g, dhp); qy = mshift(g, qy); Bf = mshift(g, Bf); rk.pred = mshift(g, rk.pred);
  fh = mshift_field(g, fh); fvy = mshift_field(g, fvy);
  COL_SETUP(N)
  cplx v[E], u[E];
  load_col<N>(v, reinterpret_cast<const cplx*>(qy), g.nh, col, t, valid);
  load_col<N>(u, reinterpret_cast<const cplx*>(Bf), g.nh, col, t, valid);
  if (rk.pred && rk.pred->done != 1) return;  // tested after the (in-bounds) loads are issued
  fft<N, false, decltype(map)>(v, buf, t, twy, map);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = mul_ik(v[r], -wavenumber(t + r * TPF, N, g.inv_Ly) * g.inv_ny);
  fft<N, true, decltype(map)>(v, buf, t, twy, map);  // -d_y qy
  fft<N, false, decltype(map)>(u, buf, t, twy, map);
#pragma unroll
  for (int r = 0; r < E; ++r) u[r] = mul_ik(u[r], -wavenumber(t + r * TPF, N, g.inv_Ly) * g.inv_ny);
  fft<N, true, decltype(map)>(u, buf, t, twy, map);  // -d_y B
  if (!valid) return;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = t + r * TPF;
    const size_t i0 = ((size_t)p * g.nh + col) * 2;
    rk_one(rk, fh, i0, dhp[i0] + v[r].x);
    rk_one(rk, fh, i0 + 1, dhp[i0 + 1] + v[r].y);
    rk_one(rk, fvy, i0, u[r].x);
    rk_one(rk, fvy, i0 + 1, u[r].y);
  }
}

// The same with its two transform chains run concurrently by two thread
// groups of the block (threadIdx.z): chain 0 forms -d_y qy and the RK combine
// of h, chain 1 -d_y B and the RK combine of v_y (no exchange between them).
template <int N>
__global__ void __launch_bounds__(1024) k_col_flux2(Geom g, const real* __restrict__ dhp, const real* __restrict__ qy,
                                                    const real* __restrict__ Bf, RkStage rk, RkField fh,
                                                    RkField fvy) {
  dhp = mshift(g, dhp); qy = mshift(g, qy); Bf = mshift(g, Bf); rk.pred = mshift(g, rk.pred);
  fh = mshift_field(g, fh); fvy = mshift_field(g, fvy);
  COL2_SETUP(N)
  cplx v[E];
  load_col<N>(v, reinterpret_cast<const cplx*>(chain == 0 ? qy : Bf), g.nh, col, t, valid);
  if (rk.pred && rk.pred->done != 1) return;  // tested after the (in-bounds) loads are issued
  fft<N, false, ColMap>(v, buf, t, twy, map);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = mul_ik(v[r], -wavenumber(t + r * TPF, N, g.inv_Ly) * g.inv_ny);
  fft<N, true, ColMap>(v, buf, t, twy, map);
  if (!valid) return;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const size_t i0 = ((size_t)(t + r * TPF) * g.nh + col) * 2;
    if (chain == 0) {
      rk_one(rk, fh, i0, dhp[i0] + v[r].x);
      rk_one(rk, fh, i0 + 1, dhp[i0 + 1] + v[r].y);
    } else {
      rk_one(rk, fvy, i0, v[r].x);
      rk_one(rk, fvy, i0 + 1, v[r].y);
    }
  }
}

// ----------------------------------------------------------------------------
// Elementwise kernels
// ----------------------------------------------------------------------------

constexpr int kUpdThreads = 1024;  // large blocks: fewer partials for the next kernel to reduce
constexpr int kUpdEpt = 4;

// Gram-Schmidt, both passes of CGS2 in one sweep of memory:
//   w1 = w - sum_{i<=j} s_i V_i (stored in W),
//   s2_i = <V_i, w1>, ||w1||^2; the last block finishes Arnoldi step j.
__global__ void __launch_bounds__(kUpdThreads) k_upd(Geom g, cplx* __restrict__ W, const cplx* __restrict__ V,
                                                     size_t vstride, int j, GmresState* st, double* partials,
                                                     const double* __restrict__ pin, int nbin) {
  W = mshift(g, W); V = mshift(g, V); st = mshift(g, st); partials = mshift(g, partials); pin = mshift(g, pin);
  if (st->st.done) return;
  __shared__ double coef[kMaxRestart + 1];
  __shared__ double red[(kMaxRestart + 2) * (kUpdThreads / 64)];
  const int tid = threadIdx.x;
  // s_i = <V_i, w> from the nbin block partials of the projection kernel
  reduce_partials<false>(pin, nbin, j + 1, nullptr, coef);
  for (int i = tid; i <= j; i += kUpdThreads) coef[i] *= g.inv_n;
  __syncthreads();
  if (blockIdx.x == 0)
    for (int i = tid; i <= j; i += kUpdThreads) st->s[i] = coef[i];
  const size_t total = (size_t)g.nh * g.ny;
  cplx w[kUpdEpt];
  double wt[kUpdEpt];
  size_t idx[kUpdEpt];
#pragma unroll
  for (int e = 0; e < kUpdEpt; ++e) {
    idx[e] = (size_t)blockIdx.x * (kUpdThreads * kUpdEpt) + e * kUpdThreads + tid;
    const bool ok = idx[e] < total;
    w[e] = ok ? W[idx[e]] : make_cplx(0.0, 0.0);
    wt[e] = ok ? col_weight((int)(idx[e] / g.ny)) : 0.0;  // column-major 2D spectra
  }
  // b keeps the last batch (V_last..V_j) for the second pass, which re-reads
  // only the earlier vectors (the re-reads miss L2 once the basis is long)
  const int last = (j / 4) * 4;
  cplx b[4][kUpdEpt];
  for (int i0 = 0; i0 <= j; i0 += 4) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < kUpdEpt; ++e)
        b[q][e] = (i0 + q <= j && idx[e] < total) ? V[(i0 + q) * vstride + idx[e]] : make_cplx(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double s = (i0 + q <= j) ? coef[i0 + q] : 0.0;
#pragma unroll
      for (int e = 0; e < kUpdEpt; ++e) {
        w[e].x -= s * b[q][e].x;
        w[e].y -= s * b[q][e].y;
      }
    }
  }
  double nr = 0.0;
#pragma unroll
  for (int e = 0; e < kUpdEpt; ++e) {
    if (idx[e] < total) W[idx[e]] = w[e];
    nr += wt[e] * cnorm2(w[e]);
  }
  // value 0: ||w1||^2; value 1 + i: <V_i, w1> (V_i re-read for i < last;
  // the last batch's from the registers that still hold it)
  double dl0 = 0.0, dl1 = 0.0, dl2 = 0.0, dl3 = 0.0;
#pragma unroll
  for (int e = 0; e < kUpdEpt; ++e) {
    if (idx[e] < total) {
      dl0 += wt[e] * cdot(b[0][e], w[e]);
      dl1 += wt[e] * cdot(b[1][e], w[e]);
      dl2 += wt[e] * cdot(b[2][e], w[e]);
      dl3 += wt[e] * cdot(b[3][e], w[e]);
    }
  }
  for (int k0 = 0; k0 <= j + 1; k0 += 8) {
    double a[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = k0 + q, i = k - 1, sel = i - last;
      double d = 0.0;
      if (k == 0) {
        d = nr;
      } else if (k <= j + 1) {
        if (sel < 0) {
#pragma unroll
          for (int e = 0; e < kUpdEpt; ++e) {
            if (idx[e] < total) {
              const cplx bv = V[i * vstride + idx[e]];
              d += wt[e] * cdot(bv, w[e]);
            }
          }
        } else {
          d = sel == 0 ? dl0 : sel == 1 ? dl1 : sel == 2 ? dl2 : dl3;
        }
      }
      a[q] = d;
    }
    wave_partials8(a, red, k0, j + 2);
  }
  block_partials_out(red, j + 2, partials, nullptr);  // finished by the next basis kernel
}

// Learned guess, pointwise passes (n points).
// st->learn_scale = RMS of r0 (block partials, last block).
__global__ void __launch_bounds__(256) k_learn_norm(const real* __restrict__ r0, size_t n, GmresState* st,
                                                    double* partials, int nblocks) {
  __shared__ double red[4];
  __shared__ double outv[1];
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)nblocks * 256) {
    const double a = r0[i];
    s += a * a;
  }
  wave_partial(s, red, 0);
  block_partials_out(red, 1, partials, nullptr);
  if (last_block_arrive(st->ctr, nblocks)) {
    reduce_partials(partials, nblocks, 1, nullptr, outv);
    if (threadIdx.x == 0) st->learn_scale = sqrt(outv[0] / (double)n);
  }
}

// Network input [n][3] (FP32): r0 / s, M^-1 r0 / s, h - h_inf (0 for s = 0).
__global__ void __launch_bounds__(256) k_learn_pack(const real* __restrict__ r0, const real* __restrict__ mr0,
                                                    const real* __restrict__ h, size_t n, double h_inf,
                                                    const GmresState* __restrict__ st, float* __restrict__ in3) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double s = st->learn_scale;
  const double is = s > 0.0 ? 1.0 / s : 0.0;
  in3[3 * i] = (float)(r0[i] * is);
  in3[3 * i + 1] = (float)(mr0[i] * is);
  in3[3 * i + 2] = (float)(h[i] - h_inf);
}

// sig_guess = sig_prev + s * out.
__global__ void __launch_bounds__(256) k_learn_apply(const real* __restrict__ sig_prev, const float* __restrict__ out,
                                                     const GmresState* __restrict__ st, real* __restrict__ sig_guess,
                                                     size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  sig_guess[i] = (real)(sig_prev[i] + st->learn_scale * (double)out[i]);
}

// Training target (FP32): (sig_new - sig_prev) / s (0 for s = 0).
__global__ void __launch_bounds__(256) k_learn_target(const real* __restrict__ sig_new, const real* __restrict__ sig_prev,
                                                      const GmresState* __restrict__ st, float* __restrict__ target,
                                                      size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double s = st->learn_scale;
  target[i] = s > 0.0 ? (float)(((double)sig_new[i] - (double)sig_prev[i]) / s) : 0.f;
}

// min h and a non-finite flag over (h, vx, vy).
__global__ void __launch_bounds__(256) k_field_stats(Geom g, const real* __restrict__ h, const real* __restrict__ vx,
                                                     const real* __restrict__ vy, size_t n, GmresState* st,
                                                     double* partials, int nblocks) {
  h = mshift(g, h); vx = mshift(g, vx); vy = mshift(g, vy); st = mshift(g, st); partials = mshift(g, partials);
  __shared__ double red[2 * 4];
  __shared__ double outv[2];
  double mn = 1e300, bad = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)nblocks * 256) {
    const double a = h[i], b = vx[i], c = vy[i];
    mn = fmin(mn, a);
    if (!isfinite(a) || !isfinite(b) || !isfinite(c)) bad = 1.0;
  }
  const int* kinds = kKindsStats;
  const double a = wave_min(mn), b = wave_max(bad);
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = a;
    red[4 + (threadIdx.x >> 6)] = b;
  }
  block_partials_out(red, 2, partials, kinds);
  if (last_block_arrive(st->ctr, nblocks)) {
    reduce_partials(partials, nblocks, 2, kinds, outv);
    if (threadIdx.x == 0) {
      st->st.stat_minh = outv[0];
      st->st.stat_nonfinite = outv[1] > 0.0 ? 1 : 0;
    }
  }
}

// ----------------------------------------------------------------------------
// Launch helper: the next launch can carry a pair of HIP events that the
// runtime records at the start and end of that dispatch (kernel timing).
// ----------------------------------------------------------------------------

// (t_ev_start / t_ev_stop: namespace sgn, shared by both precisions)
template <typename K, typename... Args>
static void launch(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, Args... args) {
  grid.z = t_members;  // ensemble members (blockIdx.z), set by the dispatch from Geom::members
  if (t_ev_start) {
    hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, s, t_ev_start, t_ev_stop, 0u, args...);
    t_ev_start = t_ev_stop = nullptr;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
  }
}

// ----------------------------------------------------------------------------
// Host launchers (dispatch on the transform length)
// ----------------------------------------------------------------------------

#define SGN_SIZES(X) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

template <int N>
struct RowLaunch {
  // row pairs per block: enough for g.row_threads threads (at least one
  // wave), at most 512 threads and no more than there are row pairs
  static dim3 block(const Geom& g) {
    int rpb = g.row_threads / Row<N>::TPF;
    if (rpb < 1) rpb = 1;
    while (rpb > 1 && (rpb > g.ny / 2 || rpb * Row<N>::TPF > 512)) rpb >>= 1;
    return dim3(Row<N>::TPF, rpb);
  }
  static size_t lds(const Geom& g) { return (size_t)block(g).y * Row<N>::LDS * sizeof(cplx); }
  static dim3 grid(const Geom& g) { return dim3((g.ny / 2) / block(g).y); }
};

// Column tiles: tc complex columns per block (a runtime choice).  At least
// one full wave per block, at most 512 threads and 64 KB of LDS (128 KB for
// the longest columns), and as wide as keeps >= g.tile_blocks blocks in
// flight.
template <int N>
struct ColLaunch {
  static int tc(const Geom& g) {
    constexpr int TPF = Col<N>::TPF;
    const size_t ldsmax = N >= 2048 ? 131072 : 65536;
    int t = 1;
    while (t * TPF < 64) t *= 2;
    while (t * 2 * TPF <= 512 && (size_t)t * 2 * N * sizeof(cplx) <= ldsmax && g.nh / (t * 2) >= g.tile_blocks)
      t *= 2;
    return t;
  }
  static dim3 block(const Geom& g) { return dim3(tc(g), Col<N>::TPF); }
  static size_t lds(const Geom& g) { return (size_t)tc(g) * N * sizeof(cplx); }
  static dim3 grid(const Geom& g) { return dim3((g.nh + tc(g) - 1) / tc(g)); }
  // the passes outside the Arnoldi step with no reduction (solution update,
  // filter): wider tiles while the launch keeps kWideBlocks blocks over all
  // members
  static constexpr int kWideBlocks = 1024;
  static int tcw(const Geom& g) {
    constexpr int TPF = Col<N>::TPF;
    const size_t ldsmax = N >= 2048 ? 131072 : 65536;
    const int mem = g.members > 1 ? g.members : 1;
    int t = tc(g);
    while (t * 2 * TPF <= 512 && (size_t)t * 2 * N * sizeof(cplx) <= ldsmax && (g.nh / (t * 2)) * mem >= kWideBlocks)
      t *= 2;
    return t;
  }
  static dim3 block_w(const Geom& g) { return dim3(tcw(g), Col<N>::TPF); }
  static size_t lds_w(const Geom& g) { return (size_t)tcw(g) * N * sizeof(cplx); }
  static dim3 grid_w(const Geom& g) { return dim3((g.nh + tcw(g) - 1) / tcw(g)); }
};

// Dynamic LDS of a kernel that may finish an Arnoldi step (finish): at least
// the m^2 doubles of the back substitution.
static size_t with_finish_lds(const Geom& g, size_t bytes, bool finish) {
  const size_t need = finish ? (size_t)g.m * g.m * sizeof(double) : 0;
  return bytes > need ? bytes : need;
}

static hipError_t allow_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

#define ROW_LAUNCH(KERNEL, ...)                                                             \
  do {                                                                                      \
    const size_t lb = RowLaunch<N>::lds(g);                                              \
    hipError_t e_ = allow_lds(reinterpret_cast<const void*>(KERNEL), lb);                   \
    if (e_ != hipSuccess) return e_;                                                        \
    launch(KERNEL, RowLaunch<N>::grid(g), RowLaunch<N>::block(g), lb, s, __VA_ARGS__); \
    return hipGetLastError();                                                               \
  } while (0)

// The same with gridDim.y = NY independent fields (Trio).
#define ROW_LAUNCH_Y(KERNEL, NY, ...)                                                       \
  do {                                                                                      \
    const size_t lb = RowLaunch<N>::lds(g);                                                 \
    hipError_t e_ = allow_lds(reinterpret_cast<const void*>(KERNEL), lb);                   \
    if (e_ != hipSuccess) return e_;                                                        \
    dim3 grid_ = RowLaunch<N>::grid(g);                                                     \
    grid_.y = (NY);                                                                         \
    launch(KERNEL, grid_, RowLaunch<N>::block(g), lb, s, __VA_ARGS__);                      \
    return hipGetLastError();                                                               \
  } while (0)

#define COL_LAUNCH_W(KERNEL, NY, ...)                                                       \
  do {                                                                                      \
    const size_t lb = ColLaunch<N>::lds_w(g);                                               \
    hipError_t e_ = allow_lds(reinterpret_cast<const void*>(KERNEL), lb);                   \
    if (e_ != hipSuccess) return e_;                                                        \
    dim3 grid_ = ColLaunch<N>::grid_w(g);                                                   \
    grid_.y = (NY);                                                                         \
    launch(KERNEL, grid_, ColLaunch<N>::block_w(g), lb, s, __VA_ARGS__);                    \
    return hipGetLastError();                                                               \
  } while (0)

#define COL_LAUNCH(KERNEL, ...)                                                             \
  do {                                                                                      \
    const size_t lb = ColLaunch<N>::lds(g);                                              \
    hipError_t e_ = allow_lds(reinterpret_cast<const void*>(KERNEL), lb);                   \
    if (e_ != hipSuccess) return e_;                                                        \
    launch(KERNEL, ColLaunch<N>::grid(g), ColLaunch<N>::block(g), lb, s, __VA_ARGS__); \
    return hipGetLastError();                                                               \
  } while (0)

#define DISPATCH_NX(FN, ...)                                                \
  switch (g.nx) {                                                           \
    case 8: return FN<8>(__VA_ARGS__);                                      \
    case 16: return FN<16>(__VA_ARGS__);                                    \
    case 32: return FN<32>(__VA_ARGS__);                                    \
    case 64: return FN<64>(__VA_ARGS__);                                    \
    case 128: return FN<128>(__VA_ARGS__);                                  \
    case 256: return FN<256>(__VA_ARGS__);                                  \
    case 512: return FN<512>(__VA_ARGS__);                                  \
    case 1024: return FN<1024>(__VA_ARGS__);                                \
    case 2048: return FN<2048>(__VA_ARGS__);                                \
    case 4096: return FN<4096>(__VA_ARGS__);                                \
    default: return hipErrorInvalidValue;                                   \
  }
#define DISPATCH_NY(FN, ...)                                                \
  switch (g.ny) {                                                           \
    case 8: return FN<8>(__VA_ARGS__);                                      \
    case 16: return FN<16>(__VA_ARGS__);                                    \
    case 32: return FN<32>(__VA_ARGS__);                                    \
    case 64: return FN<64>(__VA_ARGS__);                                    \
    case 128: return FN<128>(__VA_ARGS__);                                  \
    case 256: return FN<256>(__VA_ARGS__);                                  \
    case 512: return FN<512>(__VA_ARGS__);                                  \
    case 1024: return FN<1024>(__VA_ARGS__);                                \
    case 2048: return FN<2048>(__VA_ARGS__);                                \
    case 4096: return FN<4096>(__VA_ARGS__);                                \
    default: return hipErrorInvalidValue;                                   \
  }

template <int N>
static hipError_t row_r2c_n(const Geom& g, Trio io, int nf, hipStream_t s) {
  ROW_LAUNCH_Y(k_row_r2c<N>, nf, g, io);
}

template <int N>
static hipError_t row_c2r_n(const Geom& g, Trio io, int nf, hipStream_t s) {
  ROW_LAUNCH_Y(k_row_c2r<N>, nf, g, io);
}

template <int N>
static hipError_t row_dx_n(const Geom& g, const real* f, real* o, hipStream_t s) {
  ROW_LAUNCH(k_row_dx<N>, g, f, o);
}

template <int N>
static hipError_t row_op_n(const Geom& g, int mode, const cplx* E, const cplx* G, const real* h, const real* vx,
                           const real* vy, cplx* P, cplx* Q, cplx* R1, cplx* R2, int need_b, int pred,
                           const GmresState* st, hipStream_t s) {
  if (mode == 0 && g.status_first) ROW_LAUNCH((k_row_op<N, 0, true>), g, E, G, h, vx, vy, P, Q, R1, R2, need_b, pred, st);
  if (mode == 0) ROW_LAUNCH((k_row_op<N, 0>), g, E, G, h, vx, vy, P, Q, R1, R2, need_b, pred, st);
  if (mode == 1) ROW_LAUNCH((k_row_op<N, 1>), g, E, G, h, vx, vy, P, Q, R1, R2, need_b, pred, st);
  ROW_LAUNCH((k_row_op<N, 2>), g, E, G, h, vx, vy, P, Q, R1, R2, need_b, pred, st);
}

template <int N>
static hipError_t row_flux_n(const Geom& g, const cplx* E, const cplx* G, const real* h, const real* vx,
                             const real* vy, real* dhp, real* qy, real* B, RkStage rk, RkField fvx,
                             hipStream_t s) {
  ROW_LAUNCH(k_row_flux<N>, g, E, G, h, vx, vy, dhp, qy, B, rk, fvx);
}

template <int N>
static hipError_t row_invariants_n(const Geom& g, const cplx* E, const cplx* G, const real* h, const real* vx,
                                   const real* vy, const real* dyvx, double* partials, GmresState* st,
                                   hipStream_t s) {
  int rpb = 64 / Row<N>::TPF;
  if (rpb < 1) rpb = 1;
  const dim3 block(Row<N>::TPF, rpb);
  const int nb = (g.ny / 2 + rpb - 1) / rpb;
  const size_t lb = (size_t)rpb * Row<N>::LDS * sizeof(cplx);
  hipError_t e = allow_lds(reinterpret_cast<const void*>(k_row_invariants<N>), lb);
  if (e != hipSuccess) return e;
  launch(k_row_invariants<N>, dim3(nb), block, lb, s, g, E, G, h, vx, vy, dyvx, partials, st, nb);
  return hipGetLastError();
}

template <int N>
static hipError_t col_fwd_eg_n(const Geom& g, const cplx* Ein, cplx* SIG, cplx* Go, hipStream_t s) {
  COL_LAUNCH(k_col_fwd_eg<N>, g, Ein, SIG, Go);
}

int upd_blocks(const Geom& g);

template <int N>
static hipError_t col_basis_eg_n(const Geom& g, const cplx* W, cplx* V, size_t vs, int j, GmresState* st, cplx* Eo,
                                 cplx* Go, const double* pin, hipStream_t s) {
  const size_t lb = with_finish_lds(g, ColLaunch<N>::lds(g), j > 0);
  hipError_t e = allow_lds(reinterpret_cast<const void*>(k_col_basis_eg<N>), lb);
  if (e != hipSuccess) return e;
  launch(k_col_basis_eg<N>, ColLaunch<N>::grid(g), ColLaunch<N>::block(g), lb, s, g, W, V, vs, j, st, Eo, Go,
         pin, upd_blocks(g));
  return hipGetLastError();
}

template <int N>
static hipError_t col_update_eg_n(const Geom& g, cplx* SIG, const cplx* V, size_t vs, GmresState* st, cplx* Eo,
                                  cplx* Go, cplx* D, int spec, hipStream_t s) {
  COL_LAUNCH_W(k_col_update_eg<N>, 1, g, SIG, V, vs, st, Eo, Go, D, spec);
}

template <int N>
static hipError_t col_guess_eg_n(const Geom& g, cplx* SIG, const cplx* D, cplx* Eo, cplx* Go, hipStream_t s) {
  COL_LAUNCH(k_col_guess_eg<N>, g, SIG, D, Eo, Go);
}

template <int N>
static hipError_t col_precond_dot_n(const Geom& g, const cplx* P, const cplx* Q, const cplx* V, size_t vs, int j,
                                    GmresState* st, cplx* W, double* partials, hipStream_t s) {
  COL_LAUNCH(k_col_precond_dot<N>, g, P, Q, V, vs, j, st, W, partials);
}

template <int N>
static hipError_t col_resid_n(const Geom& g, const cplx* P, const cplx* Q, const cplx* R1, const cplx* R2, int need_b,
                              int flags, GmresState* st, cplx* W, double* partials, cplx* Eo, cplx* Go,
                              hipStream_t s) {
  // the single grid's tiles for members too: the norms' block partials (and
  // so their rounding) depend on the tile width
  const int nb = (int)ColLaunch<N>::grid(g).x;
  COL_LAUNCH(k_col_resid<N>, g, P, Q, R1, R2, need_b, flags, st, W, partials, nb, Eo, Go);
}

template <int N>
static hipError_t col_learn_n(const Geom& g, const cplx* W, cplx* out_r, cplx* out_m, hipStream_t s) {
  COL_LAUNCH(k_col_learn<N>, g, W, out_r, out_m);
}

template <int N>
static hipError_t col_inv_n(const Geom& g, const cplx* S, cplx* o, hipStream_t s) {
  COL_LAUNCH(k_col_inv<N>, g, S, o);
}

template <int N>
static hipError_t col_apply_n(const Geom& g, const cplx* P, const cplx* Q, int precond, cplx* o, hipStream_t s) {
  COL_LAUNCH(k_col_apply<N>, g, P, Q, precond, o);
}

template <int N>
static hipError_t col_filter_n(const Geom& g, Trio io, int nf, int op, double thr, hipStream_t s) {
  COL_LAUNCH_W(k_col_filter<N>, nf, g, io, op, thr);
}

template <int N>
static hipError_t col_tail_n(const Geom& g, const cplx* Sx, GmresState* st, double* partials, hipStream_t s) {
  const int nb = (int)ColLaunch<N>::grid(g).x;
  COL_LAUNCH(k_col_tail<N>, g, Sx, st, partials, nb);
}

template <int N>
static hipError_t col_dy_n(const Geom& g, const real* f, real* o, hipStream_t s) {
  COL_LAUNCH(k_col_dy<N>, g, f, o);
}

// Chain-parallel Arnoldi passes: usable when the chained block fits.
template <int N>
struct Chain {
  static constexpr bool row_ok = 3 * Row<N>::TPF <= 1024;
  // row pairs per block of the three-chain row kernel: g.row_threads threads
  // per chain when the rows are short, <= 1024 threads in all
  static int rpb(const Geom& g) {
    int r = g.row_threads / Row<N>::TPF;
    if (r < 1) r = 1;
    while (r > 1 && (r > g.ny / 2 || 3 * r * Row<N>::TPF > 1024)) r >>= 1;
    return r;
  }
  // column tile for two chains: at least one wave per chain, <= 1024 threads,
  // dynamic LDS <= kChainLds (the kernels add up to ~50 KB of static LDS, the
  // Hessenberg staging of the GMRES finish among it, within 160 KB per block),
  // >= g.tile_blocks blocks when possible
  static constexpr size_t kChainLds = 98304;
  static int tc(const Geom& g) {
    constexpr int TPF = Col<N>::TPF;
    int t = 1;
    while (t * TPF < 64) t *= 2;
    while (2 * (t * 2) * TPF <= 1024 && (size_t)2 * (t * 2) * N * sizeof(cplx) <= kChainLds &&
           g.nh / (t * 2) >= g.tile_blocks)
      t *= 2;
    return t;
  }
  static bool col_ok(const Geom& g) {
    return 2 * tc(g) * Col<N>::TPF <= 1024 && (size_t)2 * tc(g) * N * sizeof(cplx) <= kChainLds;
  }
  // column tile of the y part of the fluxes: wider than the Arnoldi kernels'
  // while the launch keeps kFluxBlocks blocks over all members (nine 1024x512
  // members: 4 columns per block instead of 2, 153 -> 138 us per launch); a
  // single grid keeps tc(g)
  static constexpr int kFluxBlocks = 1024;
  static int tc_flux(const Geom& g) {
    constexpr int TPF = Col<N>::TPF;
    const int mem = g.members > 1 ? g.members : 1;
    int t = tc(g);
    while (2 * (t * 2) * TPF <= 1024 && (size_t)2 * (t * 2) * N * sizeof(cplx) <= kChainLds &&
           (g.nh / (t * 2)) * mem >= kFluxBlocks)
      t *= 2;
    return t;
  }
};

template <int N>
static hipError_t col_flux_n(const Geom& g, const real* dhp, const real* qy, const real* B, RkStage rk,
                             RkField fh, RkField fvy, hipStream_t s) {
  // the two chains in parallel; the radix-8 columns would spill at 1024 threads
  if constexpr (N < SGN_E8_MIN) {
    if (Chain<N>::col_ok(g)) {
      const int tc = Chain<N>::tc_flux(g);
      const size_t lb = (size_t)2 * tc * N * sizeof(cplx);
      hipError_t e = allow_lds(reinterpret_cast<const void*>(k_col_flux2<N>), lb);
      if (e != hipSuccess) return e;
      launch(k_col_flux2<N>, dim3((g.nh + tc - 1) / tc), dim3(tc, Col<N>::TPF, 2), lb, s, g, dhp, qy, B, rk, fh,
             fvy);
      return hipGetLastError();
    }
  }
  COL_LAUNCH(k_col_flux<N>, g, dhp, qy, B, rk, fh, fvy);
}

// Blocks of the single-chain column kernels for this grid.
template <int N>
static int col1_blocks_n(const Geom& g) {
  return (int)ColLaunch<N>::grid(g).x;
}
static int col1_blocks(const Geom& g) {
  switch (g.ny) {
#define X(n) \
  case n:    \
    return col1_blocks_n<n>(g);
    SGN_SIZES(X)
#undef X
    default:
      return 0;
  }
}

// Blocks of the chain-parallel column kernels for this grid.
template <int N>
static int col2_blocks_n(const Geom& g) {
  const int tc = Chain<N>::tc(g);
  return (g.nh + tc - 1) / tc;
}
static int col2_blocks(const Geom& g) {
  switch (g.ny) {
#define X(n) \
  case n:    \
    return col2_blocks_n<n>(g);
    SGN_SIZES(X)
#undef X
    default:
      return 0;
  }
}

template <int N>
static hipError_t row_matvec3_n(const Geom& g, const cplx* E, const cplx* G, const real* h, cplx* P, cplx* Q,
                                const GmresState* st, hipStream_t s) {
  if constexpr (!Chain<N>::row_ok) {
    return hipErrorNotSupported;
  } else {
    const int r = Chain<N>::rpb(g);
    const dim3 block(Row<N>::TPF, 3 * r);
    const size_t lb = (size_t)3 * r * Row<N>::LDS * sizeof(cplx);
    if (g.members > 1 && 2 * Row<N>::TPF <= 512 && (g.ny / 2) % 2 == 0 && g.row_split) {
      // several grids per launch: blocks of two chains, two of which share a CU
      const int np = g.ny / 2;
      const size_t lb2 = (size_t)2 * Row<N>::LDS * sizeof(cplx);
      auto* k2 = g.status_first ? &k_row_matvec2<N, true> : &k_row_matvec2<N, false>;
      int tpf = Row<N>::TPF;
      if constexpr (N == 512 || N == 1024) {
        // radix-8 row transforms (a tuning choice, Geom::row_radix)
        if (g.row_radix == 8) {
          k2 = g.status_first ? &k_row_matvec2<N, true, 8> : &k_row_matvec2<N, false, 8>;
          tpf = N / 8;
        }
      }
      hipError_t e2 = allow_lds(reinterpret_cast<const void*>(k2), lb2);
      if (e2 != hipSuccess) return e2;
      launch(k2, dim3(np + np / 2), dim3(tpf, 2), lb2, s, g, E, G, h, P, Q, st);
      return hipGetLastError();
    }
    // the status tested first in captured graphs, after the loads otherwise
    auto* const kf = g.status_first ? &k_row_matvec3<N, true> : &k_row_matvec3<N, false>;
    hipError_t e = allow_lds(reinterpret_cast<const void*>(kf), lb);
    if (e != hipSuccess) return e;
    launch(kf, dim3((g.ny / 2) / r), block, lb, s, g, E, G, h, P, Q, st);
    return hipGetLastError();
  }
}

template <int N>
static int row_rpb_n(const Geom& g) { return (int)RowLaunch<N>::block(g).y; }
template <int N>
static int chain_rpb_n(const Geom& g) {
  if constexpr (Chain<N>::row_ok) return Chain<N>::rpb(g);
  return 0;
}
template <int N>
static int col_tc_n(const Geom& g) { return ColLaunch<N>::tc(g); }
template <int N>
static int chain_tc_n(const Geom& g) { return Chain<N>::tc(g); }

void launch_shape(const Geom& g, int* out) {
  out[0] = out[1] = out[2] = out[3] = 0;
  switch (g.nx) {
#define X(n)                      \
  case n:                         \
    out[0] = row_rpb_n<n>(g);     \
    out[1] = chain_rpb_n<n>(g);   \
    break;
    SGN_SIZES(X)
#undef X
    default:
      break;
  }
  switch (g.ny) {
#define X(n)                      \
  case n:                         \
    out[2] = col_tc_n<n>(g);      \
    out[3] = chain_tc_n<n>(g);    \
    break;
    SGN_SIZES(X)
#undef X
    default:
      break;
  }
}

template <int N>
static bool col2_ok_n(const Geom& g) { return Chain<N>::col_ok(g); }
template <int N>
static bool row3_ok_n(const Geom&) { return Chain<N>::row_ok; }
bool chained_ok(const Geom& g) {
  bool r = false, c = false;
  switch (g.nx) {
#define X(n) case n: r = row3_ok_n<n>(g); break;
    SGN_SIZES(X)
#undef X
    default: r = false;
  }
  switch (g.ny) {
#define X(n) case n: c = col2_ok_n<n>(g); break;
    SGN_SIZES(X)
#undef X
    default: c = false;
  }
  return r && c;
}

template <int N>
static hipError_t col_basis2_n(const Geom& g, const cplx* W, cplx* V, size_t vs, int j, GmresState* st, cplx* Eo,
                               cplx* Go, const double* pin, hipStream_t s) {
  const int tc = Chain<N>::tc(g);
  const dim3 block(tc, Col<N>::TPF, 2);
  const size_t lb = with_finish_lds(g, (size_t)2 * tc * N * sizeof(cplx), j > 0);
  hipError_t e = allow_lds(reinterpret_cast<const void*>(k_col_basis2<N>), lb);
  if (e != hipSuccess) return e;
  launch(k_col_basis2<N>, dim3((g.nh + tc - 1) / tc), block, lb, s, g, W, V, vs, j, st, Eo, Go, pin, upd_blocks(g));
  return hipGetLastError();
}

template <int N>
static hipError_t col_precond_dot2_n(const Geom& g, const cplx* P, const cplx* Q, const cplx* V, size_t vs, int j,
                                     GmresState* st, cplx* W, double* partials, hipStream_t s) {
  const int tc = Chain<N>::tc(g);
  const dim3 block(tc, Col<N>::TPF, 2);
  const int nb = (g.nh + tc - 1) / tc;
  const size_t lb = (size_t)2 * tc * N * sizeof(cplx);
  // the status tested first in captured graphs, after the loads otherwise
  auto* const kf = g.status_first ? &k_col_precond_dot2<N, true> : &k_col_precond_dot2<N, false>;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(kf), lb);
  if (e != hipSuccess) return e;
  launch(kf, dim3(nb), block, lb, s, g, P, Q, V, vs, j, st, W, partials);
  return hipGetLastError();
}

template <int N>
static hipError_t col_proj_n(const Geom& g, const cplx* win, cplx* W, const cplx* V, size_t vs, int j, GmresState* st,
                             cplx* Eo, cplx* Go, const double* pin, hipStream_t s) {
  const int tc = Chain<N>::tc(g);
  const dim3 block(tc, Col<N>::TPF, 2);
  const int nb = (g.nh + tc - 1) / tc;
  const size_t lb = with_finish_lds(g, (size_t)2 * tc * N * sizeof(cplx), true);
  // the status tested first in captured graphs, after the loads otherwise
  auto* const kf = g.status_first ? &k_col_proj<N, true> : &k_col_proj<N, false>;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(kf), lb);
  if (e != hipSuccess) return e;
  launch(kf, dim3(nb), block, lb, s, g, win, W, V, vs, j, st, Eo, Go, pin);
  return hipGetLastError();
}

template <int N>
static hipError_t col_precond_new_n(const Geom& g, const cplx* P, const cplx* Q, const cplx* W, cplx* V, cplx* Z,
                                    size_t vs, int j, GmresState* st, double* partials, hipStream_t s) {
  const int tc = Chain<N>::tc(g);
  const dim3 block(tc, Col<N>::TPF, 2);
  const int nb = (g.nh + tc - 1) / tc;
  const size_t lb = (size_t)2 * tc * N * sizeof(cplx);
  // the status tested first in captured graphs, after the loads otherwise
  auto* const kf = g.status_first ? &k_col_precond_new<N, true> : &k_col_precond_new<N, false>;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(kf), lb);
  if (e != hipSuccess) return e;
  launch(kf, dim3(nb), block, lb, s, g, P, Q, W, V, Z, vs, j, st, partials);
  return hipGetLastError();
}

int upd_blocks(const Geom& g) {
  const size_t total = (size_t)g.nh * g.ny;
  return (int)((total + kUpdThreads * kUpdEpt - 1) / (kUpdThreads * kUpdEpt));
}



// ---- public launchers of this precision (untyped pointers, see sgn_launch.hpp)
#define R_(p) static_cast<const real*>(p)
#define W_(p) static_cast<real*>(p)
#define RC_(p) static_cast<const cplx*>(p)
#define WC_(p) static_cast<cplx*>(p)

hipError_t launch_row_r2c(const Geom& g, const void* f, void* S, hipStream_t s) {
  const Trio io{{f, f, f}, {S, S, S}};
  DISPATCH_NX(row_r2c_n, g, io, 1, s)
}
hipError_t launch_row_c2r(const Geom& g, const void* S, void* f, hipStream_t s) {
  const Trio io{{S, S, S}, {f, f, f}};
  DISPATCH_NX(row_c2r_n, g, io, 1, s)
}
hipError_t launch_row_r2c3(const Geom& g, Trio io, hipStream_t s) { DISPATCH_NX(row_r2c_n, g, io, 3, s) }
hipError_t launch_row_c2r3(const Geom& g, Trio io, hipStream_t s) { DISPATCH_NX(row_c2r_n, g, io, 3, s) }
hipError_t launch_row_dx(const Geom& g, const void* f, void* o, hipStream_t s) {
  DISPATCH_NX(row_dx_n, g, R_(f), W_(o), s)
}
hipError_t launch_row_op(const Geom& g, int mode, const void* E, const void* G, const void* h, const void* vx,
                         const void* vy, void* P, void* Q, void* R1, void* R2, int need_b, int pred,
                         const GmresState* st, hipStream_t s) {
  DISPATCH_NX(row_op_n, g, mode, RC_(E), RC_(G), R_(h), R_(vx), R_(vy), WC_(P), WC_(Q), WC_(R1), WC_(R2), need_b,
              pred, st, s)
}
hipError_t launch_row_flux(const Geom& g, const void* E, const void* G, const void* h, const void* vx, const void* vy,
                           void* dhp, void* qy, void* B, RkStage rk, RkField fvx, hipStream_t s) {
  DISPATCH_NX(row_flux_n, g, RC_(E), RC_(G), R_(h), R_(vx), R_(vy), W_(dhp), W_(qy), W_(B), rk, fvx, s)
}
hipError_t launch_row_invariants(const Geom& g, const void* E, const void* G, const void* h, const void* vx,
                                 const void* vy, const void* dyvx, double* partials, GmresState* st, hipStream_t s) {
  DISPATCH_NX(row_invariants_n, g, RC_(E), RC_(G), R_(h), R_(vx), R_(vy), R_(dyvx), partials, st, s)
}
hipError_t launch_row_matvec3(const Geom& g, const void* E, const void* G, const void* h, void* P, void* Q,
                              const GmresState* st, hipStream_t s) {
  DISPATCH_NX(row_matvec3_n, g, RC_(E), RC_(G), R_(h), WC_(P), WC_(Q), st, s)
}
hipError_t launch_col_fwd_eg(const Geom& g, const void* Ein, void* SIG, void* Go, hipStream_t s) {
  DISPATCH_NY(col_fwd_eg_n, g, RC_(Ein), WC_(SIG), WC_(Go), s)
}
hipError_t launch_col_basis_eg(const Geom& g, const void* W, void* V, size_t vs, int j, GmresState* st, void* Eo,
                               void* Go, const double* pin, hipStream_t s) {
  DISPATCH_NY(col_basis_eg_n, g, RC_(W), WC_(V), vs, j, st, WC_(Eo), WC_(Go), pin, s)
}
hipError_t launch_col_basis2(const Geom& g, const void* W, void* V, size_t vs, int j, GmresState* st, void* Eo,
                             void* Go, const double* pin, hipStream_t s) {
  DISPATCH_NY(col_basis2_n, g, RC_(W), WC_(V), vs, j, st, WC_(Eo), WC_(Go), pin, s)
}
hipError_t launch_col_update_eg(const Geom& g, void* SIG, const void* V, size_t vs, GmresState* st, void* Eo,
                                void* Go, void* D, int spec, hipStream_t s) {
  DISPATCH_NY(col_update_eg_n, g, WC_(SIG), RC_(V), vs, st, WC_(Eo), WC_(Go), WC_(D), spec, s)
}
hipError_t launch_col_guess_eg(const Geom& g, void* SIG, const void* D, void* Eo, void* Go, hipStream_t s) {
  DISPATCH_NY(col_guess_eg_n, g, WC_(SIG), RC_(D), WC_(Eo), WC_(Go), s)
}
hipError_t launch_col_precond_dot(const Geom& g, const void* P, const void* Q, const void* V, size_t vs, int j,
                                  GmresState* st, void* W, double* partials, hipStream_t s) {
  DISPATCH_NY(col_precond_dot_n, g, RC_(P), RC_(Q), RC_(V), vs, j, st, WC_(W), partials, s)
}
hipError_t launch_col_precond_dot2(const Geom& g, const void* P, const void* Q, const void* V, size_t vs, int j,
                                   GmresState* st, void* W, double* partials, hipStream_t s) {
  DISPATCH_NY(col_precond_dot2_n, g, RC_(P), RC_(Q), RC_(V), vs, j, st, WC_(W), partials, s)
}
hipError_t launch_col_proj(const Geom& g, const void* win, void* W, const void* V, size_t vs, int j, GmresState* st,
                           void* Eo, void* Go, const double* pin, hipStream_t s) {
  DISPATCH_NY(col_proj_n, g, RC_(win), WC_(W), RC_(V), vs, j, st, WC_(Eo), WC_(Go), pin, s)
}
hipError_t launch_col_precond_new(const Geom& g, const void* P, const void* Q, const void* W, void* V, void* Z,
                                  size_t vs, int j, GmresState* st, double* partials, hipStream_t s) {
  DISPATCH_NY(col_precond_new_n, g, RC_(P), RC_(Q), RC_(W), WC_(V), WC_(Z), vs, j, st, partials, s)
}
hipError_t launch_col_resid(const Geom& g, const void* P, const void* Q, const void* R1, const void* R2, int need_b,
                            int flags, GmresState* st, void* W, double* partials, void* Eo, void* Go, hipStream_t s) {
  DISPATCH_NY(col_resid_n, g, RC_(P), RC_(Q), RC_(R1), RC_(R2), need_b, flags, st, WC_(W), partials, WC_(Eo),
              WC_(Go), s)
}
hipError_t launch_col_learn(const Geom& g, const void* W, void* out_r, void* out_m, hipStream_t s) {
  DISPATCH_NY(col_learn_n, g, RC_(W), WC_(out_r), WC_(out_m), s)
}
hipError_t launch_learn_norm(const Geom&, const void* r0, size_t n, GmresState* st, double* partials,
                             hipStream_t s) {
  int nb = (int)((n + 255) / 256);
  if (nb > 1024) nb = 1024;
  launch(k_learn_norm, dim3(nb), dim3(256), 0, s, R_(r0), n, st, partials, nb);
  return hipGetLastError();
}
hipError_t launch_learn_pack(const Geom& g, const void* r0, const void* mr0, const void* h, size_t n,
                             const GmresState* st, float* in3, hipStream_t s) {
  launch(k_learn_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, R_(r0), R_(mr0), R_(h), n, g.h_inf, st,
         in3);
  return hipGetLastError();
}
hipError_t launch_learn_apply(const Geom&, const void* sig_prev, const float* out, const GmresState* st,
                              void* sig_guess, size_t n, hipStream_t s) {
  launch(k_learn_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, R_(sig_prev), out, st, W_(sig_guess), n);
  return hipGetLastError();
}
hipError_t launch_learn_target(const Geom&, const void* sig_new, const void* sig_prev, const GmresState* st,
                               float* target, size_t n, hipStream_t s) {
  launch(k_learn_target, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, R_(sig_new), R_(sig_prev), st, target,
         n);
  return hipGetLastError();
}
hipError_t launch_col_inv(const Geom& g, const void* S, void* o, hipStream_t s) {
  DISPATCH_NY(col_inv_n, g, RC_(S), WC_(o), s)
}
hipError_t launch_col_apply(const Geom& g, const void* P, const void* Q, int precond, void* o, hipStream_t s) {
  DISPATCH_NY(col_apply_n, g, RC_(P), RC_(Q), precond, WC_(o), s)
}
hipError_t launch_col_filter(const Geom& g, const void* Sx, int op, double thr, void* o, hipStream_t s) {
  const Trio io{{Sx, Sx, Sx}, {o, o, o}};
  DISPATCH_NY(col_filter_n, g, io, 1, op, thr, s)
}
hipError_t launch_col_filter3(const Geom& g, Trio io, int op, double thr, hipStream_t s) {
  DISPATCH_NY(col_filter_n, g, io, 3, op, thr, s)
}
hipError_t launch_col_tail(const Geom& g, const void* Sx, GmresState* st, double* partials, hipStream_t s) {
  DISPATCH_NY(col_tail_n, g, RC_(Sx), st, partials, s)
}
hipError_t launch_col_dy(const Geom& g, const void* f, void* o, hipStream_t s) {
  DISPATCH_NY(col_dy_n, g, R_(f), W_(o), s)
}
hipError_t launch_col_flux(const Geom& g, const void* dhp, const void* qy, const void* B, RkStage rk, RkField fh,
                           RkField fvy, hipStream_t s) {
  DISPATCH_NY(col_flux_n, g, R_(dhp), R_(qy), R_(B), rk, fh, fvy, s)
}
hipError_t launch_upd(const Geom& g, void* W, const void* V, size_t vs, int j, GmresState* st, double* partials,
                      const double* pin, int chained, hipStream_t s) {
  const int nb = upd_blocks(g);
  const int nbin = chained ? col2_blocks(g) : col1_blocks(g);  // blocks of the projection kernel
  launch(k_upd, dim3(nb), dim3(kUpdThreads), 0, s, g, WC_(W), RC_(V), vs, j, st, partials, pin, nbin);
  return hipGetLastError();
}
hipError_t launch_field_stats(const Geom& g, const void* h, const void* vx, const void* vy, size_t n, GmresState* st,
                              double* partials, hipStream_t s) {
  int nb = (int)((n + 255) / 256);
  if (nb > 1024) nb = 1024;
  launch(k_field_stats, dim3(nb), dim3(256), 0, s, g, R_(h), R_(vx), R_(vy), n, st, partials, nb);
  return hipGetLastError();
}

int max_partial_blocks(const Geom& g) {
  int m = upd_blocks(g);
  const int rows = g.ny / 2;  // at most one block per row pair
  if (rows > m) m = rows;
  const int cols = g.nh;      // at most one block per column
  if (cols > m) m = cols;
  if (1024 > m) m = 1024;
  return m;
}

}  // namespace SGN_NS
}  // namespace sgn

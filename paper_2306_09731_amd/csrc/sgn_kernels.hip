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
// passes transform TC adjacent complex columns per block (coalesced loads of
// TC*16 bytes per row), two real columns per complex column for physical data.
#include "sgn_fft.hpp"
#include "sgn_internal.hpp"
#include "sgn_launch.hpp"

namespace sgn {

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

__device__ __forceinline__ int flat_tid() { return threadIdx.x + threadIdx.y * blockDim.x; }
__device__ __forceinline__ int block_threads() { return blockDim.x * blockDim.y; }

// Every block calls this once after writing its partials.  Returns true in
// exactly one block (the last to arrive), after an acquire fence.
__device__ bool last_block_arrive(uint32_t* counter, int nblocks) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (flat_tid() == 0) {
    const uint32_t prev = atomicAdd(counter, 1u);
    s_last = (prev == (uint32_t)(nblocks - 1)) ? 1 : 0;
  }
  __syncthreads();
  if (s_last) __threadfence();
  return s_last != 0;
}

// kind: 0 sum, 1 min, 2 max.  out[k] (LDS) = reduction over blocks of
// partials[b * kPartialStride + k], in a fixed order.
__device__ void reduce_partials(const double* partials, int nblocks, int nvals, const int* kind,
                                double* out) {
  const int tid = flat_tid();
  const int lane = tid & 63, wave = tid >> 6, nw = block_threads() >> 6;
  for (int k = wave; k < nvals; k += nw) {
    const int kd = kind ? kind[k] : 0;
    double s = kd == 0 ? 0.0 : (kd == 1 ? 1e300 : -1e300);
    for (int b = lane; b < nblocks; b += 64) {
      const double x = partials[(size_t)b * kPartialStride + k];
      s = kd == 0 ? s + x : (kd == 1 ? fmin(s, x) : fmax(s, x));
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
    partials[(size_t)blockIdx.x * kPartialStride + k] = s;
  }
}

// ----------------------------------------------------------------------------
// GMRES scalar work (single thread of the last block)
// ----------------------------------------------------------------------------

// Finish Arnoldi step j: H(:, j) = s + s2, H(j+1, j) = ||w2||, Givens, test.
__device__ void gmres_finish_step(GmresState* st, int j, double nrm2, const double* s2) {
  double* H = st->H;
  double sum2 = 0.0;
  for (int i = 0; i <= j; ++i) {
    H[hidx(i, j)] = st->s[i] + s2[i];
    st->s2[i] = s2[i];
    sum2 += s2[i] * s2[i];
  }
  const double b2 = nrm2 - sum2;
  const double beta = b2 > 0.0 ? sqrt(b2) : 0.0;
  H[hidx(j + 1, j)] = beta;
  st->beta = beta;
  for (int i = 0; i < j; ++i) {
    const double a = H[hidx(i, j)], b = H[hidx(i + 1, j)];
    H[hidx(i, j)] = st->cs[i] * a + st->sn[i] * b;
    H[hidx(i + 1, j)] = -st->sn[i] * a + st->cs[i] * b;
  }
  const double a = H[hidx(j, j)], b = H[hidx(j + 1, j)];
  const double rho = hypot(a, b);
  double c = 1.0, s = 0.0;
  if (rho > 0.0) {
    c = a / rho;
    s = b / rho;
  }
  st->cs[j] = c;
  st->sn[j] = s;
  H[hidx(j, j)] = rho;
  H[hidx(j + 1, j)] = 0.0;
  st->gv[j + 1] = -s * st->gv[j];
  st->gv[j] = c * st->gv[j];
  const double resid = fabs(st->gv[j + 1]);
  for (int i = j; i >= 0; --i) {
    double acc = st->gv[i];
    for (int l = i + 1; l <= j; ++l) acc -= H[hidx(i, l)] * st->y[l];
    const double d = H[hidx(i, i)];
    st->y[i] = d != 0.0 ? acc / d : 0.0;
  }
  st->st.jdone = j + 1;
  st->st.total_iters += 1;
  st->st.resid = resid;
  if (resid <= st->tol * st->st.beta0 || beta == 0.0)
    st->st.done = 1;
  else if (j + 1 >= st->m)
    st->st.done = 2;
}

// ----------------------------------------------------------------------------
// Row passes
// ----------------------------------------------------------------------------

template <int N>
struct Row {
  static constexpr int E = FftShape<N>::E;
  static constexpr int TPF = FftShape<N>::TPF;
  using Map = LdsMap<1, true>;
  static constexpr int LDS = LdsMap<1, true>::size(N);  // cplx per row pair
};

template <int N>
__device__ __forceinline__ void load_phys_pair(cplx* v, const double* __restrict__ f, int ya, int t) {
  const double* a = f + (size_t)ya * N;
  const double* b = a + N;
#pragma unroll
  for (int r = 0; r < Row<N>::E; ++r) {
    const int p = t + r * Row<N>::TPF;
    v[r] = make_double2(a[p], b[p]);
  }
}

template <int N>
__device__ __forceinline__ void store_phys_pair(const cplx* v, double* __restrict__ f, int ya, int t) {
  double* a = f + (size_t)ya * N;
  double* b = a + N;
#pragma unroll
  for (int r = 0; r < Row<N>::E; ++r) {
    const int p = t + r * Row<N>::TPF;
    a[p] = v[r].x;
    b[p] = v[r].y;
  }
}

// Full spectrum of (row ya) + i (row ya+1) from their x-half spectra, times s.
template <int N>
__device__ __forceinline__ void load_spec_pair(cplx* v, const cplx* __restrict__ S, int ya, int t, double s) {
  constexpr int H = N / 2;
  const cplx* A = S + (size_t)ya * H;
  const cplx* B = A + H;
#pragma unroll
  for (int r = 0; r < Row<N>::E; ++r) {
    const int p = t + r * Row<N>::TPF;
    cplx z;
    if (p == 0) {
      const cplx a = A[0], b = B[0];
      z = make_double2(a.x, b.x);
    } else if (p == H) {
      const cplx a = A[0], b = B[0];
      z = make_double2(a.y, b.y);
    } else if (p < H) {
      const cplx a = A[p], b = B[p];
      z = make_double2(a.x - b.y, a.y + b.x);
    } else {
      const cplx a = A[N - p], b = B[N - p];
      z = make_double2(a.x + b.y, b.x - a.y);
    }
    v[r] = cscale(z, s);
  }
}

// Split the full spectrum of a packed row pair into the two half spectra.
template <int N>
__device__ __forceinline__ void store_spec_pair(const cplx* v, cplx* __restrict__ S, int ya, int t, cplx* buf) {
  using M = typename Row<N>::Map;
  constexpr int H = N / 2;
#pragma unroll
  for (int r = 0; r < Row<N>::E; ++r) buf[M::at(t + r * Row<N>::TPF)] = v[r];
  __syncthreads();
  cplx* A = S + (size_t)ya * H;
  cplx* B = A + H;
#pragma unroll
  for (int r = 0; r < Row<N>::E / 2; ++r) {
    const int k = t + r * Row<N>::TPF;
    if (k == 0) {
      const cplx z0 = buf[M::at(0)], zn = buf[M::at(H)];
      A[0] = make_double2(z0.x, zn.x);
      B[0] = make_double2(z0.y, zn.y);
    } else {
      const cplx z = buf[M::at(k)], zc = buf[M::at(N - k)];
      A[k] = make_double2(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));
      B[k] = make_double2(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));
    }
  }
  __syncthreads();
}

#define ROW_SETUP(N)                                   \
  constexpr int E = Row<N>::E;                         \
  constexpr int TPF = Row<N>::TPF;                     \
  using Map = typename Row<N>::Map;                    \
  extern __shared__ cplx lds[];                        \
  const int t = threadIdx.x;                           \
  const int ya = 2 * (blockIdx.x * blockDim.y + threadIdx.y); \
  cplx* buf = lds + threadIdx.y * Row<N>::LDS;         \
  (void)TPF;

// physical f -> x-half spectra S
template <int N>
__global__ void __launch_bounds__(512) k_row_r2c(Geom g, const double* __restrict__ f, cplx* __restrict__ S) {
  ROW_SETUP(N)
  cplx v[E];
  load_phys_pair<N>(v, f, ya, t);
  fft<N, false, Map>(v, buf, t, g.twx);
  store_spec_pair<N>(v, S, ya, t, buf);
}

// x-half spectra S -> physical f
template <int N>
__global__ void __launch_bounds__(512) k_row_c2r(Geom g, const cplx* __restrict__ S, double* __restrict__ f) {
  ROW_SETUP(N)
  cplx v[E];
  load_spec_pair<N>(v, S, ya, t, g.inv_nx);
  fft<N, true, Map>(v, buf, t, g.twx);
  store_phys_pair<N>(v, f, ya, t);
}

// out = d/dx f
template <int N>
__global__ void __launch_bounds__(512) k_row_dx(Geom g, const double* __restrict__ f, double* __restrict__ out) {
  ROW_SETUP(N)
  cplx v[E];
  load_phys_pair<N>(v, f, ya, t);
  fft<N, false, Map>(v, buf, t, g.twx);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = mul_ik(v[r], wavenumber(t + r * TPF, N, g.inv_Lx) * g.inv_nx);
  fft<N, true, Map>(v, buf, t, g.twx);
  store_phys_pair<N>(v, out, ya, t);
}

// Elliptic operator, x part, in x-spectral form.  From E = F_x sigma and
// G = F_x d_y sigma (x-half spectra) and the depth h:
//   A1 = F_x(3 sigma / h^3) - i kx F_x(d_x sigma / h),   A2 = F_x(d_y sigma / h)
// so that F(L_h sigma) = F_y(A1) - i ky F_y(A2).
// MODE 0: P = A1, Q = A2 (the Arnoldi matvec; skipped once GMRES is done).
// MODE 1: residual with b = -div v:  B1 = -i kx F_x vx, B2 = F_x vy,
//         P = B1 - A1, Q = B2 - A2 (and R1 = B1, R2 = B2 if need_b).
// MODE 2: residual with an explicit b (passed in vx): B1 = F_x b, B2 = 0.
template <int N, int MODE>
__global__ void __launch_bounds__(512) k_row_op(Geom g, const cplx* __restrict__ Es, const cplx* __restrict__ Gs,
                                                const double* __restrict__ h, const double* __restrict__ vx,
                                                const double* __restrict__ vy, cplx* __restrict__ P,
                                                cplx* __restrict__ Q, cplx* __restrict__ R1, cplx* __restrict__ R2,
                                                int need_b, int predicate, const GmresState* __restrict__ st) {
  if (MODE == 0 && predicate && st->st.done) return;
  ROW_SETUP(N)
  const double* ha = h + (size_t)ya * N;
  const double* hb = ha + N;
  cplx v[E], u[E];
  load_spec_pair<N>(v, Es, ya, t, g.inv_nx);
#pragma unroll
  for (int r = 0; r < E; ++r) u[r] = mul_ik(v[r], wavenumber(t + r * TPF, N, g.inv_Lx));
  fft<N, true, Map>(v, buf, t, g.twx);  // sigma
  fft<N, true, Map>(u, buf, t, g.twx);  // d_x sigma
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = t + r * TPF;
    const double ia = 1.0 / ha[p], ib = 1.0 / hb[p];
    v[r] = make_double2(3.0 * v[r].x * ia * ia * ia, 3.0 * v[r].y * ib * ib * ib);
    u[r] = make_double2(u[r].x * ia, u[r].y * ib);
  }
  fft<N, false, Map>(v, buf, t, g.twx);
  fft<N, false, Map>(u, buf, t, g.twx);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = csub(v[r], mul_ik(u[r], wavenumber(t + r * TPF, N, g.inv_Lx)));  // A1
  load_spec_pair<N>(u, Gs, ya, t, g.inv_nx);
  fft<N, true, Map>(u, buf, t, g.twx);  // d_y sigma
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = t + r * TPF;
    u[r] = make_double2(u[r].x / ha[p], u[r].y / hb[p]);
  }
  fft<N, false, Map>(u, buf, t, g.twx);  // A2
  if constexpr (MODE == 0) {
    store_spec_pair<N>(v, P, ya, t, buf);
    store_spec_pair<N>(u, Q, ya, t, buf);
  } else {
    cplx w[E];
    load_phys_pair<N>(w, vx, ya, t);
    fft<N, false, Map>(w, buf, t, g.twx);
    if constexpr (MODE == 1) {
#pragma unroll
      for (int r = 0; r < E; ++r) w[r] = mul_ik(w[r], -wavenumber(t + r * TPF, N, g.inv_Lx));
    }
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = csub(w[r], v[r]);
    store_spec_pair<N>(v, P, ya, t, buf);
    if (need_b) store_spec_pair<N>(w, R1, ya, t, buf);
    if constexpr (MODE == 1) {
      load_phys_pair<N>(w, vy, ya, t);
      fft<N, false, Map>(w, buf, t, g.twx);
#pragma unroll
      for (int r = 0; r < E; ++r) u[r] = csub(w[r], u[r]);
      store_spec_pair<N>(u, Q, ya, t, buf);
      if (need_b) store_spec_pair<N>(w, R2, ya, t, buf);
    } else {
#pragma unroll
      for (int r = 0; r < E; ++r) u[r] = make_double2(-u[r].x, -u[r].y);
      store_spec_pair<N>(u, Q, ya, t, buf);
    }
  }
}

__device__ __forceinline__ void rk_one(const RkStage& rk, const RkField& f, size_t i, double k) {
  if (rk.mode == 0) {
    f.out[i] = k;
  } else if (rk.mode == 1) {
    const double a = rk.first ? 0.0 : f.acc[i];
    f.acc[i] = a + rk.wacc * k;
    f.out[i] = f.yn[i] + rk.cnext * k;
  } else {
    f.out[i] = f.yn[i] + rk.dt * (f.acc[i] + rk.wacc * k);
  }
}

// Fluxes, x part.  With sigma from (E, G), the stage state (h, vx, vy):
//   qx = h vx - d_x sigma,  qy = h vy - d_y sigma,
//   B  = (vx^2 + vy^2)/2 - |grad sigma|^2 / (2 h^2) + g h - 9/2 sigma^2 / h^4
// writes dhp = -d_x qx, qy, B and k_vx = -d_x B (through the RK combine).
template <int N>
__global__ void __launch_bounds__(512) k_row_flux(Geom g, const cplx* __restrict__ Es, const cplx* __restrict__ Gs,
                                                  const double* h, const double* vx, const double* vy,
                                                  double* __restrict__ dhp, double* __restrict__ qy,
                                                  double* __restrict__ Bo, RkStage rk, RkField fvx) {
  ROW_SETUP(N)
  const size_t oa = (size_t)ya * N, ob = oa + N;
  cplx v[E], B[E];
  load_spec_pair<N>(v, Es, ya, t, g.inv_nx);
  fft<N, true, Map>(v, buf, t, g.twx);  // sigma
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = t + r * TPF;
    const double a = h[oa + p], b = h[ob + p];
    const double ia = 1.0 / a, ib = 1.0 / b;
    const double sa = v[r].x * ia * ia, sb = v[r].y * ib * ib;
    B[r] = make_double2(g.g * a - 4.5 * sa * sa, g.g * b - 4.5 * sb * sb);
  }
  load_spec_pair<N>(v, Es, ya, t, g.inv_nx);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = mul_ik(v[r], wavenumber(t + r * TPF, N, g.inv_Lx));
  fft<N, true, Map>(v, buf, t, g.twx);  // d_x sigma
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = t + r * TPF;
    const double a = h[oa + p], b = h[ob + p];
    const double ua = vx[oa + p], ub = vx[ob + p];
    const double ra = v[r].x / a, rb = v[r].y / b;
    B[r].x += 0.5 * ua * ua - 0.5 * ra * ra;
    B[r].y += 0.5 * ub * ub - 0.5 * rb * rb;
    v[r] = make_double2(a * ua - v[r].x, b * ub - v[r].y);  // qx
  }
  fft<N, false, Map>(v, buf, t, g.twx);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = mul_ik(v[r], -wavenumber(t + r * TPF, N, g.inv_Lx) * g.inv_nx);
  fft<N, true, Map>(v, buf, t, g.twx);
  store_phys_pair<N>(v, dhp, ya, t);  // -d_x qx
  load_spec_pair<N>(v, Gs, ya, t, g.inv_nx);
  fft<N, true, Map>(v, buf, t, g.twx);  // d_y sigma
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = t + r * TPF;
    const double a = h[oa + p], b = h[ob + p];
    const double wa = vy[oa + p], wb = vy[ob + p];
    const double ra = v[r].x / a, rb = v[r].y / b;
    B[r].x += 0.5 * wa * wa - 0.5 * ra * ra;
    B[r].y += 0.5 * wb * wb - 0.5 * rb * rb;
    qy[oa + p] = a * wa - v[r].x;
    qy[ob + p] = b * wb - v[r].y;
  }
  store_phys_pair<N>(B, Bo, ya, t);
  fft<N, false, Map>(B, buf, t, g.twx);
#pragma unroll
  for (int r = 0; r < E; ++r) B[r] = mul_ik(B[r], -wavenumber(t + r * TPF, N, g.inv_Lx) * g.inv_nx);
  fft<N, true, Map>(B, buf, t, g.twx);  // k_vx = -d_x B
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
                                                        const cplx* __restrict__ Gs, const double* __restrict__ h,
                                                        const double* __restrict__ vx, const double* __restrict__ vy,
                                                        const double* __restrict__ dyvx, double* partials,
                                                        GmresState* st, int nblocks) {
  constexpr int E = Row<N>::E;
  constexpr int TPF = Row<N>::TPF;
  using Map = typename Row<N>::Map;
  extern __shared__ cplx lds[];
  const int t = threadIdx.x;
  // blocks hold at least one full wave; slots past the last row pair read a
  // valid row pair and contribute nothing
  const int ya_raw = 2 * (blockIdx.x * blockDim.y + threadIdx.y);
  const bool rvalid = ya_raw < g.ny;
  const int ya = rvalid ? ya_raw : g.ny - 2;
  cplx* buf = lds + threadIdx.y * Row<N>::LDS;
  __shared__ double red[7 * 8];
  __shared__ double outv[8];
  const size_t oa = (size_t)ya * N, ob = oa + N;
  cplx s[E], d[E];
  double acc[5] = {0, 0, 0, 0, 0};
  double mn = 1e300, mx = -1e300;
  load_spec_pair<N>(s, Es, ya, t, g.inv_nx);
#pragma unroll
  for (int r = 0; r < E; ++r) d[r] = mul_ik(s[r], wavenumber(t + r * TPF, N, g.inv_Lx));
  fft<N, true, Map>(s, buf, t, g.twx);  // sigma
  fft<N, true, Map>(d, buf, t, g.twx);  // d_x sigma
  cplx e[E];
  load_spec_pair<N>(e, Gs, ya, t, g.inv_nx);
  fft<N, true, Map>(e, buf, t, g.twx);  // d_y sigma
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
  fft<N, false, Map>(d, buf, t, g.twx);
#pragma unroll
  for (int r = 0; r < E; ++r) d[r] = mul_ik(d[r], wavenumber(t + r * TPF, N, g.inv_Lx) * g.inv_nx);
  fft<N, true, Map>(d, buf, t, g.twx);
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
  if (last_block_arrive(&st->counter, nblocks)) {
    reduce_partials(partials, nblocks, 7, kinds, outv);
    if (flat_tid() == 0) {
      st->st.red[0] = outv[0] * g.dA;
      st->st.red[1] = outv[1] * g.dA;
      st->st.red[2] = outv[2] * g.dA;
      st->st.red[3] = outv[3] * g.dA;
      st->st.red[4] = sqrt(outv[4] * g.dA);
      st->st.red[5] = outv[5];
      st->st.red[6] = outv[6];
      st->counter = 0;
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
  static constexpr int TC0 = (N >= 2048) ? (131072 / 16) / N : (65536 / 16) / N;  // LDS budget
  static constexpr int TC1 = TC0 < 16 ? TC0 : 16;
  static constexpr int TC2 = (512 / TPF) < TC1 ? (512 / TPF) : TC1;
  static constexpr int TCmin = (64 / TPF) > 1 ? (64 / TPF) : 1;  // at least one wave per block
  static constexpr int TC = TC2 > TCmin ? TC2 : TCmin;
  using Map = LdsMap<TC, false>;
  static constexpr int LDS = TC * N;
};

#define COL_SETUP(N)                                         \
  constexpr int E = Col<N>::E;                               \
  constexpr int TPF = Col<N>::TPF;                           \
  constexpr int TC = Col<N>::TC;                             \
  using Map = typename Col<N>::Map;                          \
  extern __shared__ cplx lds[];                              \
  const int c = threadIdx.x;                                 \
  const int t = threadIdx.y;                                 \
  const int col = blockIdx.x * TC + c;                       \
  const bool valid = col < g.nh;                             \
  cplx* buf = lds + c;                                       \
  (void)valid;

template <int N>
__device__ __forceinline__ void load_col(cplx* v, const cplx* __restrict__ S, int nh, int col, int t, bool valid) {
#pragma unroll
  for (int r = 0; r < Col<N>::E; ++r) {
    const int p = t + r * Col<N>::TPF;
    v[r] = valid ? S[(size_t)p * nh + col] : make_double2(0.0, 0.0);
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
  COL_SETUP(N)
  cplx v[E];
  load_col<N>(v, Ein, g.nh, col, t, valid);
  fft<N, false, Map>(v, buf, t, g.twy);
  store_col<N>(v, SIG, g.nh, col, t, valid);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = mul_ik(v[r], wavenumber(t + r * TPF, N, g.inv_Ly) * g.inv_ny);
  fft<N, true, Map>(v, buf, t, g.twy);
  store_col<N>(v, Gout, g.nh, col, t, valid);
}

// Inverse y-transforms of a 2D spectrum x: E = F_y^-1 x, G = F_y^-1 (i ky x).
template <int N>
__device__ __forceinline__ void col_emit_eg(Geom& g, cplx* v, cplx* buf, int t, int col, bool valid,
                                            cplx* __restrict__ Eo, cplx* __restrict__ Go) {
  constexpr int E = Col<N>::E, TPF = Col<N>::TPF;
  using Map = typename Col<N>::Map;
  cplx u[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    u[r] = mul_ik(v[r], wavenumber(t + r * TPF, N, g.inv_Ly) * g.inv_ny);
    v[r] = cscale(v[r], g.inv_ny);
  }
  fft<N, true, Map>(v, buf, t, g.twy);
  store_col<N>(v, Eo, g.nh, col, t, valid);
  fft<N, true, Map>(u, buf, t, g.twy);
  store_col<N>(u, Go, g.nh, col, t, valid);
}

// Arnoldi: V_j = (W - sum_{i<j} s2_i V_i) / beta, then E, G of V_j.
template <int N>
__global__ void __launch_bounds__(512) k_col_basis_eg(Geom g, const cplx* __restrict__ W, cplx* __restrict__ V,
                                                       size_t vstride, int j, const GmresState* __restrict__ st,
                                                       cplx* __restrict__ Eo, cplx* __restrict__ Go) {
  if (st->st.done) return;
  COL_SETUP(N)
  __shared__ double coef[kMaxRestart + 1];
  const int tid = flat_tid();
  for (int i = tid; i < j; i += block_threads()) coef[i] = st->s2[i];
  __syncthreads();
  const double ib = 1.0 / st->beta;
  cplx v[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = t + r * TPF;
    const size_t idx = (size_t)p * g.nh + col;
    cplx x = make_double2(0.0, 0.0);
    if (valid) {
      x = W[idx];
      for (int i = 0; i < j; ++i) {
        const cplx b = V[i * vstride + idx];
        x.x -= coef[i] * b.x;
        x.y -= coef[i] * b.y;
      }
      x = cscale(x, ib);
      V[j * vstride + idx] = x;
    }
    v[r] = x;
  }
  col_emit_eg<N>(g, v, buf, t, col, valid, Eo, Go);
}

// sigma_hat += sum_{i<k} y_i V_i (or 0 when b == 0), then E, G of sigma_hat.
template <int N>
__global__ void __launch_bounds__(512) k_col_update_eg(Geom g, cplx* __restrict__ SIG, const cplx* __restrict__ V,
                                                        size_t vstride, const GmresState* __restrict__ st,
                                                        cplx* __restrict__ Eo, cplx* __restrict__ Go) {
  COL_SETUP(N)
  __shared__ double coef[kMaxRestart];
  const int tid = flat_tid();
  const int k = st->st.jdone;
  const int zero = st->st.zero;
  for (int i = tid; i < k; i += block_threads()) coef[i] = st->y[i];
  __syncthreads();
  cplx v[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = t + r * TPF;
    const size_t idx = (size_t)p * g.nh + col;
    cplx x = make_double2(0.0, 0.0);
    if (valid) {
      if (!zero) {
        x = SIG[idx];
        for (int i = 0; i < k; ++i) {
          const cplx b = V[i * vstride + idx];
          x.x += coef[i] * b.x;
          x.y += coef[i] * b.y;
        }
      }
      SIG[idx] = x;
    }
    v[r] = x;
  }
  col_emit_eg<N>(g, v, buf, t, col, valid, Eo, Go);
}

__device__ __forceinline__ double inv_symbol(const Geom& g, double kx, double ky) {
  return 1.0 / (g.m0 + g.m1 * (kx * kx + ky * ky));
}

// F_y(P) - i ky F_y(Q) for the tile; P, Q are x-half spectra (Q may be null).
template <int N>
__device__ __forceinline__ void col_combine(Geom& g, cplx* v, cplx* buf, int t, int col, bool valid,
                                            const cplx* __restrict__ P, const cplx* __restrict__ Q) {
  constexpr int E = Col<N>::E, TPF = Col<N>::TPF;
  using Map = typename Col<N>::Map;
  load_col<N>(v, P, g.nh, col, t, valid);
  fft<N, false, Map>(v, buf, t, g.twy);
  if (Q == nullptr) return;  // second term absent (an explicit b has no y part)
  cplx u[E];
  load_col<N>(u, Q, g.nh, col, t, valid);
  fft<N, false, Map>(u, buf, t, g.twy);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = csub(v[r], mul_ik(u[r], wavenumber(t + r * TPF, N, g.inv_Ly)));
}

// Weight of a half-spectrum column in a physical inner product:
// column 0 carries kx = 0 and the Nyquist column once, others stand for +-kx.
__device__ __forceinline__ double col_weight(int col) { return col == 0 ? 1.0 : 2.0; }

// Arnoldi: w = M^-1 F(L V_j) (= (F_y P - i ky F_y Q) / M), s_i = <V_i, w>, i <= j.
template <int N>
__global__ void __launch_bounds__(512) k_col_precond_dot(Geom g, const cplx* __restrict__ P,
                                                          const cplx* __restrict__ Q, const cplx* __restrict__ V,
                                                          size_t vstride, int j, GmresState* st, cplx* __restrict__ W,
                                                          double* partials, int nblocks) {
  if (st->st.done) return;
  COL_SETUP(N)
  __shared__ double red[(kMaxRestart + 1) * 16];
  __shared__ double outv[kMaxRestart + 1];
  cplx v[E];
  col_combine<N>(g, v, buf, t, col, valid, P, Q);
  const double kx = col * g.inv_Lx;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = t + r * TPF;
    v[r] = cscale(v[r], inv_symbol(g, kx, wavenumber(p, N, g.inv_Ly)));
  }
  store_col<N>(v, W, g.nh, col, t, valid);
  const double wt = valid ? col_weight(col) : 0.0;
  for (int i = 0; i <= j; ++i) {
    double d = 0.0;
    if (valid) {
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int p = t + r * TPF;
        const cplx b = V[i * vstride + (size_t)p * g.nh + col];
        d += b.x * v[r].x + b.y * v[r].y;
      }
    }
    wave_partial(wt * d, red, i);
  }
  block_partials_out(red, j + 1, partials, nullptr);
  if (last_block_arrive(&st->counter, nblocks)) {
    reduce_partials(partials, nblocks, j + 1, nullptr, outv);
    for (int i = flat_tid(); i <= j; i += block_threads()) st->s[i] = outv[i] * g.inv_n;
    __syncthreads();
    if (flat_tid() == 0) st->counter = 0;
  }
}

// Start of a GMRES cycle: r = M^-1 (b - L sigma) with F(b - L sigma) =
// F_y(P) - i ky F_y(Q).  With need_b, b_hat = F_y(R1) - i ky F_y(R2) gives
// beta0 = ||M^-1 b|| and ||b||.  flags: 1 = new solve (reset the counters),
// 2 = report the unpreconditioned residual only (no cycle set-up).
template <int N>
__global__ void __launch_bounds__(512) k_col_resid(Geom g, const cplx* __restrict__ P, const cplx* __restrict__ Q,
                                                    const cplx* __restrict__ R1, const cplx* __restrict__ R2,
                                                    int need_b, int flags, GmresState* st, cplx* __restrict__ W,
                                                    double* partials, int nblocks) {
  COL_SETUP(N)
  __shared__ double red[3 * 16];
  __shared__ double outv[3];
  const bool true_only = (flags & 2) != 0;
  cplx v[E];
  col_combine<N>(g, v, buf, t, col, valid, P, Q);
  const double kx = col * g.inv_Lx;
  const double wt = valid ? col_weight(col) : 0.0;
  double nr = 0.0;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = t + r * TPF;
    if (!true_only) v[r] = cscale(v[r], inv_symbol(g, kx, wavenumber(p, N, g.inv_Ly)));
    nr += v[r].x * v[r].x + v[r].y * v[r].y;
  }
  if (!true_only) store_col<N>(v, W, g.nh, col, t, valid);
  wave_partial(wt * nr, red, 0);
  int nvals = 1;
  if (need_b) {
    col_combine<N>(g, v, buf, t, col, valid, R1, R2);
    double nb = 0.0, nbm = 0.0;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int p = t + r * TPF;
      const double m = inv_symbol(g, kx, wavenumber(p, N, g.inv_Ly));
      const double a2 = v[r].x * v[r].x + v[r].y * v[r].y;
      nb += a2;
      nbm += a2 * m * m;
    }
    wave_partial(wt * nbm, red, 1);
    wave_partial(wt * nb, red, 2);
    nvals = 3;
  }
  block_partials_out(red, nvals, partials, nullptr);
  if (last_block_arrive(&st->counter, nblocks)) {
    reduce_partials(partials, nblocks, nvals, nullptr, outv);
    if (flat_tid() == 0) {
      if (true_only) {
        st->st.true_resid2 = outv[0] * g.inv_n;
      } else {
        if (flags & 1) {
          st->st.total_iters = 0;
          st->st.zero = 0;
        }
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
      st->counter = 0;
    }
  }
}

// Inverse y-transform of a 2D spectrum: out = F_y^-1 S / ny.
template <int N>
__global__ void __launch_bounds__(512) k_col_inv(Geom g, const cplx* __restrict__ S, cplx* __restrict__ out) {
  COL_SETUP(N)
  cplx v[E];
  load_col<N>(v, S, g.nh, col, t, valid);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = cscale(v[r], g.inv_ny);
  fft<N, true, Map>(v, buf, t, g.twy);
  store_col<N>(v, out, g.nh, col, t, valid);
}

// Apply the 2D operator F(L s) (from P, Q) and optionally M^-1; out = 2D spectrum.
template <int N>
__global__ void __launch_bounds__(512) k_col_apply(Geom g, const cplx* __restrict__ P, const cplx* __restrict__ Q,
                                                    int precond, cplx* __restrict__ out) {
  COL_SETUP(N)
  cplx v[E];
  col_combine<N>(g, v, buf, t, col, valid, P, Q);
  if (precond) {
    const double kx = col * g.inv_Lx;
#pragma unroll
    for (int r = 0; r < E; ++r)
      v[r] = cscale(v[r], inv_symbol(g, kx, wavenumber(t + r * TPF, N, g.inv_Ly)));
  }
  store_col<N>(v, out, g.nh, col, t, valid);
}

// x-half spectra -> multiplied by a 2D symbol -> x-half spectra.
//   op 0: M^-1 (preconditioner)
//   op 1: Krasny filter, zero modes with |X| / (nx ny) < thr
template <int N>
__global__ void __launch_bounds__(512) k_col_filter(Geom g, const cplx* __restrict__ Sx, int op, double thr,
                                                     cplx* __restrict__ out) {
  COL_SETUP(N)
  cplx v[E];
  load_col<N>(v, Sx, g.nh, col, t, valid);
  fft<N, false, Map>(v, buf, t, g.twy);
  if (op == 0) {
    const double kx = col * g.inv_Lx;
#pragma unroll
    for (int r = 0; r < E; ++r)
      v[r] = cscale(v[r], inv_symbol(g, kx, wavenumber(t + r * TPF, N, g.inv_Ly)));
  } else {
    const double T = thr * (double)g.nx * (double)g.ny;
    const double T2 = T * T;
    // column 0 packs two real-signal spectra (kx = 0 and kx = nx/2): split
    // them with the +-ky partner, threshold each, recombine.
#pragma unroll
    for (int r = 0; r < E; ++r) buf[Map::at(t + r * TPF)] = v[r];
    __syncthreads();
    cplx partner[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int p = t + r * TPF;
      partner[r] = buf[Map::at((N - p) & (N - 1))];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) {
      if (col == 0) {
        const cplx z = v[r], zc = partner[r];
        cplx a = make_double2(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));   // kx = 0 mode
        cplx b = make_double2(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));  // kx = nx/2 mode
        if (a.x * a.x + a.y * a.y < T2) a = make_double2(0.0, 0.0);
        if (b.x * b.x + b.y * b.y < T2) b = make_double2(0.0, 0.0);
        v[r] = make_double2(a.x - b.y, a.y + b.x);
      } else {
        if (v[r].x * v[r].x + v[r].y * v[r].y < T2) v[r] = make_double2(0.0, 0.0);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = cscale(v[r], g.inv_ny);
  fft<N, true, Map>(v, buf, t, g.twy);
  store_col<N>(v, out, g.nh, col, t, valid);
}

// Largest normalised 2D DFT coefficient with |mx| > nx/4 or |my| > ny/4.
template <int N>
__global__ void __launch_bounds__(512) k_col_tail(Geom g, const cplx* __restrict__ Sx, GmresState* st,
                                                   double* partials, int nblocks) {
  COL_SETUP(N)
  __shared__ double red[16];
  __shared__ double outv[1];
  cplx v[E];
  load_col<N>(v, Sx, g.nh, col, t, valid);
  fft<N, false, Map>(v, buf, t, g.twy);
#pragma unroll
  for (int r = 0; r < E; ++r) buf[Map::at(t + r * TPF)] = v[r];
  __syncthreads();
  cplx partner[E];
#pragma unroll
  for (int r = 0; r < E; ++r) partner[r] = buf[Map::at((N - (t + r * TPF)) & (N - 1))];
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
        const cplx a = make_double2(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));
        const cplx b = make_double2(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));
        if (yin) mx = fmax(mx, sqrt(a.x * a.x + a.y * a.y));
        mx = fmax(mx, sqrt(b.x * b.x + b.y * b.y));  // kx = nx/2 is always outside nx/4
      } else if (yin || 4 * col > g.nx) {
        mx = fmax(mx, sqrt(v[r].x * v[r].x + v[r].y * v[r].y));
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
  if (last_block_arrive(&st->counter, nblocks)) {
    reduce_partials(partials, nblocks, 1, kinds, outv);
    if (flat_tid() == 0) {
      st->st.red[7] = outv[0] * g.inv_n;
      st->counter = 0;
    }
  }
}

// out = d/dy f for a physical field (two real columns per complex column).
template <int N>
__global__ void __launch_bounds__(512) k_col_dy(Geom g, const double* __restrict__ f, double* __restrict__ out) {
  COL_SETUP(N)
  cplx v[E];
  load_col<N>(v, reinterpret_cast<const cplx*>(f), g.nh, col, t, valid);
  fft<N, false, Map>(v, buf, t, g.twy);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = mul_ik(v[r], wavenumber(t + r * TPF, N, g.inv_Ly) * g.inv_ny);
  fft<N, true, Map>(v, buf, t, g.twy);
  store_col<N>(v, reinterpret_cast<cplx*>(out), g.nh, col, t, valid);
}

// Fluxes, y part: dh = dhp - d_y qy, k_vy = -d_y B, through the RK combine.
template <int N>
__global__ void __launch_bounds__(512) k_col_flux(Geom g, const double* __restrict__ dhp, const double* __restrict__ qy,
                                                   const double* __restrict__ Bf, RkStage rk, RkField fh, RkField fvy) {
  COL_SETUP(N)
  cplx v[E], u[E];
  load_col<N>(v, reinterpret_cast<const cplx*>(qy), g.nh, col, t, valid);
  fft<N, false, Map>(v, buf, t, g.twy);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = mul_ik(v[r], -wavenumber(t + r * TPF, N, g.inv_Ly) * g.inv_ny);
  fft<N, true, Map>(v, buf, t, g.twy);  // -d_y qy
  load_col<N>(u, reinterpret_cast<const cplx*>(Bf), g.nh, col, t, valid);
  fft<N, false, Map>(u, buf, t, g.twy);
#pragma unroll
  for (int r = 0; r < E; ++r) u[r] = mul_ik(u[r], -wavenumber(t + r * TPF, N, g.inv_Ly) * g.inv_ny);
  fft<N, true, Map>(u, buf, t, g.twy);  // -d_y B
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

// ----------------------------------------------------------------------------
// Elementwise kernels
// ----------------------------------------------------------------------------

constexpr int kUpdThreads = 256;
constexpr int kUpdEpt = 4;

// Gram-Schmidt, both passes of CGS2 in one sweep of memory:
//   w1 = w - sum_{i<=j} s_i V_i (stored in W),
//   s2_i = <V_i, w1>, ||w1||^2; the last block finishes Arnoldi step j.
__global__ void __launch_bounds__(kUpdThreads) k_upd(Geom g, cplx* __restrict__ W, const cplx* __restrict__ V,
                                                     size_t vstride, int j, GmresState* st, double* partials,
                                                     int nblocks) {
  if (st->st.done) return;
  __shared__ double coef[kMaxRestart + 1];
  __shared__ double red[(kMaxRestart + 2) * (kUpdThreads / 64)];
  __shared__ double outv[kMaxRestart + 2];
  const int tid = threadIdx.x;
  for (int i = tid; i <= j; i += kUpdThreads) coef[i] = st->s[i];
  __syncthreads();
  const size_t total = (size_t)g.nh * g.ny;
  cplx w[kUpdEpt];
  double wt[kUpdEpt];
  size_t idx[kUpdEpt];
#pragma unroll
  for (int e = 0; e < kUpdEpt; ++e) {
    idx[e] = (size_t)blockIdx.x * (kUpdThreads * kUpdEpt) + e * kUpdThreads + tid;
    const bool ok = idx[e] < total;
    w[e] = ok ? W[idx[e]] : make_double2(0.0, 0.0);
    wt[e] = ok ? col_weight((int)(idx[e] % g.nh)) : 0.0;
  }
  for (int i = 0; i <= j; ++i) {
    const double s = coef[i];
#pragma unroll
    for (int e = 0; e < kUpdEpt; ++e) {
      if (idx[e] < total) {
        const cplx b = V[i * vstride + idx[e]];
        w[e].x -= s * b.x;
        w[e].y -= s * b.y;
      }
    }
  }
  double nr = 0.0;
#pragma unroll
  for (int e = 0; e < kUpdEpt; ++e) {
    if (idx[e] < total) W[idx[e]] = w[e];
    nr += wt[e] * (w[e].x * w[e].x + w[e].y * w[e].y);
  }
  wave_partial(nr, red, 0);
  for (int i = 0; i <= j; ++i) {
    double d = 0.0;
#pragma unroll
    for (int e = 0; e < kUpdEpt; ++e) {
      if (idx[e] < total) {
        const cplx b = V[i * vstride + idx[e]];
        d += wt[e] * (b.x * w[e].x + b.y * w[e].y);
      }
    }
    wave_partial(d, red, i + 1);
  }
  block_partials_out(red, j + 2, partials, nullptr);
  if (last_block_arrive(&st->counter, nblocks)) {
    reduce_partials(partials, nblocks, j + 2, nullptr, outv);
    if (tid == 0) {
      for (int i = 0; i <= j + 1; ++i) outv[i] *= g.inv_n;
      gmres_finish_step(st, j, outv[0], outv + 1);
      st->counter = 0;
    }
  }
}

// min h and a non-finite flag over (h, vx, vy).
__global__ void __launch_bounds__(256) k_field_stats(const double* __restrict__ h, const double* __restrict__ vx,
                                                     const double* __restrict__ vy, size_t n, GmresState* st,
                                                     double* partials, int nblocks) {
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
  if (last_block_arrive(&st->counter, nblocks)) {
    reduce_partials(partials, nblocks, 2, kinds, outv);
    if (threadIdx.x == 0) {
      st->st.stat_minh = outv[0];
      st->st.stat_nonfinite = outv[1] > 0.0 ? 1 : 0;
      st->counter = 0;
    }
  }
}

// ----------------------------------------------------------------------------
// Host launchers (dispatch on the transform length)
// ----------------------------------------------------------------------------

#define SGN_SIZES(X) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

template <int N>
struct RowLaunch {
  static dim3 block(int ny) {
    int rpb = 64 / Row<N>::TPF;
    if (rpb < 1) rpb = 1;
    while (rpb > 1 && rpb > ny / 2) rpb >>= 1;
    return dim3(Row<N>::TPF, rpb);
  }
  static size_t lds(int ny) { return (size_t)block(ny).y * Row<N>::LDS * sizeof(cplx); }
  static dim3 grid(int ny) { return dim3((ny / 2) / block(ny).y); }
};

template <int N>
struct ColLaunch {
  static dim3 block() { return dim3(Col<N>::TC, Col<N>::TPF); }
  static size_t lds() { return (size_t)Col<N>::LDS * sizeof(cplx); }
  static dim3 grid(int nh) { return dim3((nh + Col<N>::TC - 1) / Col<N>::TC); }
};

static hipError_t allow_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

#define ROW_LAUNCH(KERNEL, ...)                                                             \
  do {                                                                                      \
    const size_t lb = RowLaunch<N>::lds(g.ny);                                              \
    hipError_t e_ = allow_lds(reinterpret_cast<const void*>(KERNEL), lb);                   \
    if (e_ != hipSuccess) return e_;                                                        \
    hipLaunchKernelGGL(KERNEL, RowLaunch<N>::grid(g.ny), RowLaunch<N>::block(g.ny), lb, s, __VA_ARGS__); \
    return hipGetLastError();                                                               \
  } while (0)

#define COL_LAUNCH(KERNEL, ...)                                                             \
  do {                                                                                      \
    const size_t lb = ColLaunch<N>::lds();                                                  \
    hipError_t e_ = allow_lds(reinterpret_cast<const void*>(KERNEL), lb);                   \
    if (e_ != hipSuccess) return e_;                                                        \
    hipLaunchKernelGGL(KERNEL, ColLaunch<N>::grid(g.nh), ColLaunch<N>::block(), lb, s, __VA_ARGS__); \
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
static hipError_t row_r2c_n(const Geom& g, const double* f, cplx* S, hipStream_t s) {
  ROW_LAUNCH(k_row_r2c<N>, g, f, S);
}
hipError_t launch_row_r2c(const Geom& g, const double* f, cplx* S, hipStream_t s) { DISPATCH_NX(row_r2c_n, g, f, S, s) }

template <int N>
static hipError_t row_c2r_n(const Geom& g, const cplx* S, double* f, hipStream_t s) {
  ROW_LAUNCH(k_row_c2r<N>, g, S, f);
}
hipError_t launch_row_c2r(const Geom& g, const cplx* S, double* f, hipStream_t s) { DISPATCH_NX(row_c2r_n, g, S, f, s) }

template <int N>
static hipError_t row_dx_n(const Geom& g, const double* f, double* o, hipStream_t s) {
  ROW_LAUNCH(k_row_dx<N>, g, f, o);
}
hipError_t launch_row_dx(const Geom& g, const double* f, double* o, hipStream_t s) { DISPATCH_NX(row_dx_n, g, f, o, s) }

template <int N>
static hipError_t row_op_n(const Geom& g, int mode, const cplx* E, const cplx* G, const double* h, const double* vx,
                           const double* vy, cplx* P, cplx* Q, cplx* R1, cplx* R2, int need_b, int pred,
                           const GmresState* st, hipStream_t s) {
  if (mode == 0) ROW_LAUNCH((k_row_op<N, 0>), g, E, G, h, vx, vy, P, Q, R1, R2, need_b, pred, st);
  if (mode == 1) ROW_LAUNCH((k_row_op<N, 1>), g, E, G, h, vx, vy, P, Q, R1, R2, need_b, pred, st);
  ROW_LAUNCH((k_row_op<N, 2>), g, E, G, h, vx, vy, P, Q, R1, R2, need_b, pred, st);
}
hipError_t launch_row_op(const Geom& g, int mode, const cplx* E, const cplx* G, const double* h, const double* vx,
                         const double* vy, cplx* P, cplx* Q, cplx* R1, cplx* R2, int need_b, int pred,
                         const GmresState* st, hipStream_t s) {
  DISPATCH_NX(row_op_n, g, mode, E, G, h, vx, vy, P, Q, R1, R2, need_b, pred, st, s)
}

template <int N>
static hipError_t row_flux_n(const Geom& g, const cplx* E, const cplx* G, const double* h, const double* vx,
                             const double* vy, double* dhp, double* qy, double* B, RkStage rk, RkField fvx,
                             hipStream_t s) {
  ROW_LAUNCH(k_row_flux<N>, g, E, G, h, vx, vy, dhp, qy, B, rk, fvx);
}
hipError_t launch_row_flux(const Geom& g, const cplx* E, const cplx* G, const double* h, const double* vx,
                           const double* vy, double* dhp, double* qy, double* B, RkStage rk, RkField fvx,
                           hipStream_t s) {
  DISPATCH_NX(row_flux_n, g, E, G, h, vx, vy, dhp, qy, B, rk, fvx, s)
}

template <int N>
static hipError_t row_invariants_n(const Geom& g, const cplx* E, const cplx* G, const double* h, const double* vx,
                                   const double* vy, const double* dyvx, double* partials, GmresState* st,
                                   hipStream_t s) {
  int rpb = 64 / Row<N>::TPF;
  if (rpb < 1) rpb = 1;
  const dim3 block(Row<N>::TPF, rpb);
  const int nb = (g.ny / 2 + rpb - 1) / rpb;
  const size_t lb = (size_t)rpb * Row<N>::LDS * sizeof(cplx);
  hipError_t e = allow_lds(reinterpret_cast<const void*>(k_row_invariants<N>), lb);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_row_invariants<N>, dim3(nb), block, lb, s, g, E, G, h, vx, vy, dyvx, partials, st, nb);
  return hipGetLastError();
}
hipError_t launch_row_invariants(const Geom& g, const cplx* E, const cplx* G, const double* h, const double* vx,
                                 const double* vy, const double* dyvx, double* partials, GmresState* st,
                                 hipStream_t s) {
  DISPATCH_NX(row_invariants_n, g, E, G, h, vx, vy, dyvx, partials, st, s)
}

template <int N>
static hipError_t col_fwd_eg_n(const Geom& g, const cplx* Ein, cplx* SIG, cplx* Go, hipStream_t s) {
  COL_LAUNCH(k_col_fwd_eg<N>, g, Ein, SIG, Go);
}
hipError_t launch_col_fwd_eg(const Geom& g, const cplx* Ein, cplx* SIG, cplx* Go, hipStream_t s) {
  DISPATCH_NY(col_fwd_eg_n, g, Ein, SIG, Go, s)
}

template <int N>
static hipError_t col_basis_eg_n(const Geom& g, const cplx* W, cplx* V, size_t vs, int j, const GmresState* st,
                                 cplx* Eo, cplx* Go, hipStream_t s) {
  COL_LAUNCH(k_col_basis_eg<N>, g, W, V, vs, j, st, Eo, Go);
}
hipError_t launch_col_basis_eg(const Geom& g, const cplx* W, cplx* V, size_t vs, int j, const GmresState* st,
                               cplx* Eo, cplx* Go, hipStream_t s) {
  DISPATCH_NY(col_basis_eg_n, g, W, V, vs, j, st, Eo, Go, s)
}

template <int N>
static hipError_t col_update_eg_n(const Geom& g, cplx* SIG, const cplx* V, size_t vs, const GmresState* st, cplx* Eo,
                                  cplx* Go, hipStream_t s) {
  COL_LAUNCH(k_col_update_eg<N>, g, SIG, V, vs, st, Eo, Go);
}
hipError_t launch_col_update_eg(const Geom& g, cplx* SIG, const cplx* V, size_t vs, const GmresState* st, cplx* Eo,
                                cplx* Go, hipStream_t s) {
  DISPATCH_NY(col_update_eg_n, g, SIG, V, vs, st, Eo, Go, s)
}

template <int N>
static hipError_t col_precond_dot_n(const Geom& g, const cplx* P, const cplx* Q, const cplx* V, size_t vs, int j,
                                    GmresState* st, cplx* W, double* partials, hipStream_t s) {
  const int nb = (int)ColLaunch<N>::grid(g.nh).x;
  COL_LAUNCH(k_col_precond_dot<N>, g, P, Q, V, vs, j, st, W, partials, nb);
}
hipError_t launch_col_precond_dot(const Geom& g, const cplx* P, const cplx* Q, const cplx* V, size_t vs, int j,
                                  GmresState* st, cplx* W, double* partials, hipStream_t s) {
  DISPATCH_NY(col_precond_dot_n, g, P, Q, V, vs, j, st, W, partials, s)
}

template <int N>
static hipError_t col_resid_n(const Geom& g, const cplx* P, const cplx* Q, const cplx* R1, const cplx* R2, int need_b,
                              int flags, GmresState* st, cplx* W, double* partials, hipStream_t s) {
  const int nb = (int)ColLaunch<N>::grid(g.nh).x;
  COL_LAUNCH(k_col_resid<N>, g, P, Q, R1, R2, need_b, flags, st, W, partials, nb);
}
hipError_t launch_col_resid(const Geom& g, const cplx* P, const cplx* Q, const cplx* R1, const cplx* R2, int need_b,
                            int flags, GmresState* st, cplx* W, double* partials, hipStream_t s) {
  DISPATCH_NY(col_resid_n, g, P, Q, R1, R2, need_b, flags, st, W, partials, s)
}

template <int N>
static hipError_t col_inv_n(const Geom& g, const cplx* S, cplx* o, hipStream_t s) {
  COL_LAUNCH(k_col_inv<N>, g, S, o);
}
hipError_t launch_col_inv(const Geom& g, const cplx* S, cplx* o, hipStream_t s) { DISPATCH_NY(col_inv_n, g, S, o, s) }

template <int N>
static hipError_t col_apply_n(const Geom& g, const cplx* P, const cplx* Q, int precond, cplx* o, hipStream_t s) {
  COL_LAUNCH(k_col_apply<N>, g, P, Q, precond, o);
}
hipError_t launch_col_apply(const Geom& g, const cplx* P, const cplx* Q, int precond, cplx* o, hipStream_t s) {
  DISPATCH_NY(col_apply_n, g, P, Q, precond, o, s)
}

template <int N>
static hipError_t col_filter_n(const Geom& g, const cplx* Sx, int op, double thr, cplx* o, hipStream_t s) {
  COL_LAUNCH(k_col_filter<N>, g, Sx, op, thr, o);
}
hipError_t launch_col_filter(const Geom& g, const cplx* Sx, int op, double thr, cplx* o, hipStream_t s) {
  DISPATCH_NY(col_filter_n, g, Sx, op, thr, o, s)
}

template <int N>
static hipError_t col_tail_n(const Geom& g, const cplx* Sx, GmresState* st, double* partials, hipStream_t s) {
  const int nb = (int)ColLaunch<N>::grid(g.nh).x;
  COL_LAUNCH(k_col_tail<N>, g, Sx, st, partials, nb);
}
hipError_t launch_col_tail(const Geom& g, const cplx* Sx, GmresState* st, double* partials, hipStream_t s) {
  DISPATCH_NY(col_tail_n, g, Sx, st, partials, s)
}

template <int N>
static hipError_t col_dy_n(const Geom& g, const double* f, double* o, hipStream_t s) {
  COL_LAUNCH(k_col_dy<N>, g, f, o);
}
hipError_t launch_col_dy(const Geom& g, const double* f, double* o, hipStream_t s) { DISPATCH_NY(col_dy_n, g, f, o, s) }

template <int N>
static hipError_t col_flux_n(const Geom& g, const double* dhp, const double* qy, const double* B, RkStage rk,
                             RkField fh, RkField fvy, hipStream_t s) {
  COL_LAUNCH(k_col_flux<N>, g, dhp, qy, B, rk, fh, fvy);
}
hipError_t launch_col_flux(const Geom& g, const double* dhp, const double* qy, const double* B, RkStage rk, RkField fh,
                           RkField fvy, hipStream_t s) {
  DISPATCH_NY(col_flux_n, g, dhp, qy, B, rk, fh, fvy, s)
}

int upd_blocks(const Geom& g) {
  const size_t total = (size_t)g.nh * g.ny;
  return (int)((total + kUpdThreads * kUpdEpt - 1) / (kUpdThreads * kUpdEpt));
}

hipError_t launch_upd(const Geom& g, cplx* W, const cplx* V, size_t vs, int j, GmresState* st, double* partials,
                      hipStream_t s) {
  const int nb = upd_blocks(g);
  hipLaunchKernelGGL(k_upd, dim3(nb), dim3(kUpdThreads), 0, s, g, W, V, vs, j, st, partials, nb);
  return hipGetLastError();
}

hipError_t launch_field_stats(const double* h, const double* vx, const double* vy, size_t n, GmresState* st,
                              double* partials, hipStream_t s) {
  int nb = (int)((n + 255) / 256);
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_field_stats, dim3(nb), dim3(256), 0, s, h, vx, vy, n, st, partials, nb);
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

}  // namespace sgn

// Device-side complex arithmetic and the register/LDS FFT engine used by
// every spectral pass of the SGN solver (gfx950).  Included once per working
// precision: the including file defines SGN_NS (namespace), SGN_REAL and
// SGN_CPLX (double/double2 or float/float2).
//
// The engine is a Stockham autosort FFT.  An FFT of length N is computed by
// TPF = N/E threads, each holding E complex values in registers.  The first
// and the last stage both have radix E, so a thread holds the elements at
// positions p = t + r*TPF (r = 0..E-1) both on entry and on exit: pointwise
// work between a forward and an inverse transform (a spectral multiplier, a
// division by the depth h) needs no data exchange.  Middle stages (radix
// <= E) exchange through LDS.  Twiddles come from a host-computed FP64 table
// tw[k] = exp(-2 pi i k / N).
#pragma once
#include <hip/hip_runtime.h>

namespace sgn {
namespace SGN_NS {

typedef SGN_REAL real;
typedef SGN_CPLX cplx;

__device__ __forceinline__ cplx make_cplx(real x, real y) {
  cplx z;
  z.x = x;
  z.y = y;
  return z;
}
__device__ __forceinline__ cplx czero() { return make_cplx(real(0), real(0)); }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return make_cplx(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return make_cplx(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return make_cplx(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ cplx cmulc(cplx a, cplx b) {
  return make_cplx(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ cplx cscale(cplx a, double s) {
  const real t = (real)s;
  return make_cplx(a.x * t, a.y * t);
}
__device__ __forceinline__ cplx mul_i(cplx a) { return make_cplx(-a.y, a.x); }   // i a
__device__ __forceinline__ cplx mul_mi(cplx a) { return make_cplx(a.y, -a.x); }  // -i a
__device__ __forceinline__ cplx conjc(cplx a) { return make_cplx(a.x, -a.y); }
// i*k*a for a real k
__device__ __forceinline__ cplx mul_ik(cplx a, double k) {
  const real t = (real)k;
  return make_cplx(-t * a.y, t * a.x);
}
// Re(a conj(b)) accumulated in FP64 (exact products of FP32 operands)
__device__ __forceinline__ double cdot(cplx a, cplx b) {
  return (double)a.x * (double)b.x + (double)a.y * (double)b.y;
}
__device__ __forceinline__ double cnorm2(cplx a) { return (double)a.x * (double)a.x + (double)a.y * (double)a.y; }

// cos(pi m / 8) and sin(pi m / 8), m = 0..8: the twiddles of DFTs up to size 16.
struct Tw16 {
  static constexpr double C1 = 0.92387953251128675613;  // cos(pi/8)
  static constexpr double S1 = 0.38268343236508977173;  // sin(pi/8)
  static constexpr double R2 = 0.70710678118654752440;  // cos(pi/4)
};

// Multiply by W_R^k = exp(-+2 pi i k / R) (sign by INV) for compile-time R, k.
template <int R, int K, bool INV>
__device__ __forceinline__ cplx twc(cplx a) {
  constexpr int m = (16 / R) * K;  // angle = pi m / 8, m in [0, 8)
  static_assert(16 % R == 0 && m < 8, "radix up to 16");
  if constexpr (m == 0) {
    return a;
  } else if constexpr (m == 4) {
    return INV ? mul_i(a) : mul_mi(a);
  } else {
    constexpr real c = (real)((m == 1) ? Tw16::C1 : (m == 2) ? Tw16::R2 : (m == 3) ? Tw16::S1
                             : (m == 5) ? -Tw16::S1 : (m == 6) ? -Tw16::R2 : -Tw16::C1);
    constexpr real s = (real)((m == 1) ? Tw16::S1 : (m == 2) ? Tw16::R2 : (m == 3) ? Tw16::C1
                             : (m == 5) ? Tw16::C1 : (m == 6) ? Tw16::R2 : Tw16::S1);
    // forward: (c - i s); inverse: (c + i s)
    return INV ? make_cplx(a.x * c - a.y * s, a.x * s + a.y * c)
               : make_cplx(a.x * c + a.y * s, a.y * c - a.x * s);
  }
}

template <int R, bool INV, int K = 0>
__device__ __forceinline__ void combine_halves(cplx* e, cplx* o, cplx* v) {
  if constexpr (K < R / 2) {
    cplx t = twc<R, K, INV>(o[K]);
    v[K] = cadd(e[K], t);
    v[K + R / 2] = csub(e[K], t);
    combine_halves<R, INV, K + 1>(e, o, v);
  }
}

// In-register DFT of size R (1, 2, 4, 8, 16), natural order in and out.
template <int R, bool INV>
__device__ __forceinline__ void dft(cplx* v) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    cplx a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
  } else if constexpr (R == 4) {
    cplx s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    cplx s13 = cadd(v[1], v[3]);
    cplx d13 = INV ? mul_i(csub(v[1], v[3])) : mul_mi(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
  } else {
    cplx e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    dft<R / 2, INV>(e);
    dft<R / 2, INV>(o);
    combine_halves<R, INV>(e, o, v);
  }
}

// Elements per thread for a transform of length N: 4, or 8 from 2048 points
// (half the threads per transform and two fewer LDS exchanges; measured
// faster there in both precisions, slower at 1024 and 512 points in FP64).
#ifndef SGN_E8_MIN
#define SGN_E8_MIN 2048
#endif
template <int N>
struct FftShape {
  static constexpr int E = (N <= 8) ? N : (N >= SGN_E8_MIN) ? 8 : 4;
  static constexpr int TPF = N / E;
  static_assert(N == E || N % (E * E) == 0, "plan needs N == E or E^2 | N");
};

// LDS addressing.  Row transforms pad one slot every 8 complex values to
// spread strided writes over the banks; column transforms interleave the
// tc columns of a block (lane-fast) with a runtime stride.
struct RowMap {
  __device__ __forceinline__ int at(int p) const { return p + (p >> 3); }
  static constexpr int size(int n) { return n + n / 8; }
};
struct ColMap {
  int tc;
  __device__ __forceinline__ int at(int p) const { return p * tc; }
};

// Twiddles used by one thread, gathered once per kernel into registers (they
// are the same for every transform of that length the thread performs; the
// inverse uses their conjugates).  Layout: the middle stages in order, each
// with (E/R) butterflies x (R-1) twiddles, then the last stage's E-1.
template <int N, int E, int Ns>
constexpr int mid_twiddles() {
  constexpr int rem = N / (Ns * E);
  if constexpr (rem > 1) {
    constexpr int R = rem >= E ? E : rem;
    return (E / R) * (R - 1) + mid_twiddles<N, E, Ns * R>();
  } else {
    return 0;
  }
}

template <int N, int EE = FftShape<N>::E>
struct TwiddleSet {
  static constexpr int E = EE;
  static constexpr int MID = (N == E) ? 0 : mid_twiddles<N, E, E>();
  static constexpr int COUNT = (N == E) ? 1 : MID + (E - 1);
  cplx w[COUNT];
};

template <int N, int E, int Ns, int OFF>
__device__ __forceinline__ void gather_mid_twiddles(cplx* w, int t, const cplx* __restrict__ tw) {
  constexpr int rem = N / (Ns * E);
  if constexpr (rem > 1) {
    constexpr int R = rem >= E ? E : rem;
    constexpr int TPF = N / E;
#pragma unroll
    for (int q = 0; q < E / R; ++q) {
      const int jm = (t + q * TPF) % Ns;
#pragma unroll
      for (int r = 1; r < R; ++r) w[OFF + q * (R - 1) + (r - 1)] = tw[jm * r * (N / (Ns * R))];
    }
    gather_mid_twiddles<N, E, Ns * R, OFF + (E / R) * (R - 1)>(w, t, tw);
  }
}

// tw: the length-N table exp(-2 pi i k / N); t: the thread's index in its transform.
// EE: values per thread (the default of FftShape, or another radix with
// E^2 | N that a kernel is instantiated for).
template <int N, int EE>
__device__ __forceinline__ void gather_twiddles(TwiddleSet<N, EE>& ts, int t, const cplx* __restrict__ tw) {
  constexpr int E = EE;
  if constexpr (N == E) {
    ts.w[0] = make_cplx(real(1), real(0));
  } else {
    gather_mid_twiddles<N, E, E, 0>(ts.w, t, tw);
#pragma unroll
    for (int r = 1; r < E; ++r) ts.w[TwiddleSet<N, EE>::MID + r - 1] = tw[t * r];
  }
}

template <bool INV>
__device__ __forceinline__ cplx twmul(cplx a, cplx w) {
  return INV ? cmulc(a, w) : cmul(a, w);
}

// One middle Stockham stage of radix R (<= E); Ns = product of earlier
// radices; OFF = offset of this stage's twiddles in the thread's set.
template <int N, int E, int R, int Ns, int OFF, bool INV, class Map>
__device__ __forceinline__ void fft_middle_stage(cplx* buf, int t, const cplx* w_tw, const Map& map) {
  constexpr int TPF = N / E;
  constexpr int NB = E / R;  // butterflies per thread
  cplx w[E];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int j = t + q * TPF;
#pragma unroll
    for (int r = 0; r < R; ++r) w[q * R + r] = buf[map.at(j + r * (N / R))];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int j = t + q * TPF;
    const int jm = j % Ns;
#pragma unroll
    for (int r = 1; r < R; ++r) w[q * R + r] = twmul<INV>(w[q * R + r], w_tw[OFF + q * (R - 1) + (r - 1)]);
    dft<R, INV>(&w[q * R]);
    const int base = (j / Ns) * Ns * R + jm;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[map.at(base + r * Ns)] = w[q * R + r];
  }
  __syncthreads();
}

template <int N, int E, int Ns, int OFF, bool INV, class Map>
__device__ __forceinline__ void fft_middle_stages(cplx* buf, int t, const cplx* w_tw, const Map& map) {
  constexpr int rem = N / (Ns * E);
  if constexpr (rem > 1) {
    constexpr int R = rem >= E ? E : rem;
    fft_middle_stage<N, E, R, Ns, OFF, INV, Map>(buf, t, w_tw, map);
    fft_middle_stages<N, E, Ns * R, OFF + (E / R) * (R - 1), INV, Map>(buf, t, w_tw, map);
  }
}

// Full transform of length N on registers v[E] (positions t + r*TPF in and
// out).  buf: this transform's LDS region (map addressing); ts: the thread's
// twiddles.  Unnormalised in both directions.  Ends with a barrier so buf
// may be reused at once.
template <int N, bool INV, class Map, int EE>
__device__ __forceinline__ void fft(cplx* v, cplx* buf, int t, const TwiddleSet<N, EE>& ts, const Map& map) {
  constexpr int E = EE;
  constexpr int TPF = N / E;
  static_assert(N == E || N % (E * E) == 0, "plan needs N == E or E^2 | N");
  dft<E, INV>(v);
  if constexpr (N == E) return;
  // first stage output (Ns = 1): position t*E + r
#pragma unroll
  for (int r = 0; r < E; ++r) buf[map.at(t * E + r)] = v[r];
  __syncthreads();
  fft_middle_stages<N, E, E, 0, INV, Map>(buf, t, ts.w, map);
  // last stage: radix E, Ns = TPF, butterfly j = t, positions t + r*TPF
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = buf[map.at(t + r * TPF)];
  __syncthreads();
#pragma unroll
  for (int r = 1; r < E; ++r) v[r] = twmul<INV>(v[r], ts.w[TwiddleSet<N, EE>::MID + r - 1]);
  dft<E, INV>(v);
}

// Signed wavenumber of DFT index p of a length-n transform on a period
// 2 pi L (inv_L = 1/L), with the Nyquist index mapped to 0.
__device__ __forceinline__ double wavenumber(int p, int n, double inv_L) {
  const int h = n >> 1;
  if (p == h) return 0.0;
  return (double)(p < h ? p : p - n) * inv_L;
}

}  // namespace SGN_NS
}  // namespace sgn

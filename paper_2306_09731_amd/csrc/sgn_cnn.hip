// The learned initial guess: a 6-layer network of 3x3 periodic convolutions
// with BF16 weights and activations and FP32 accumulation on the matrix cores
// (v_mfma_f32_32x32x16_bf16), its backward pass, the MSE loss and Adam.
//
// Layouts: activations [H][W][32] BF16 (channels last, 64 B per point);
// weights of a layer w[tap][cout][cin] (tap = 3 ky + kx reads the input at
// (y + ky - 1, x + kx - 1) modulo the grid); every layer is 32 -> 32 (the
// three input channels and the single output channel are zero-padded, and
// padded weights never reach the output or receive gradient).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sgn.h"
#include "sgn_cnn_internal.hpp"

namespace sgnn {

constexpr int C = 32;                  // channels of every layer
constexpr int L = SGN_CNN_LAYERS;      // layers
constexpr int TAPS = 9;
constexpr int WL = TAPS * C * C;       // weights per layer
constexpr int PL = WL + C;             // parameters per layer (weights, then biases)
constexpr int NP = L * PL;             // all parameters
constexpr int SEG = 128;               // points of a row per weight-gradient pass
constexpr int kWgBlocks = 512;         // blocks of the weight-gradient kernel (partials)
constexpr int kRedThreads = 256;

static_assert(NP == SGN_CNN_PARAMS, "parameter count");

typedef uint16_t bf16;
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bf2f(bf16 u) { return __uint_as_float((uint32_t)u << 16); }
// round to nearest even (NaN kept quiet)
__device__ __forceinline__ bf16 f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (bf16)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16)(u >> 16);
}

// ---------------------------------------------------------------------------
// Convolution, forward and input gradient.  A wave computes kTilesPerWave
// tiles of 32 consecutive points of a row (A rows) x 32 output channels (B
// columns), holding the layer's weights (the B operands of all 18 MFMA steps)
// in registers across its tiles; K = 9 taps x 32 input channels in 18 MFMA
// steps of 16.  Lane l supplies A[l % 32][8 (l / 32) + v] and B[8 (l / 32) +
// v][l % 32], v < 8, and receives D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32], v < 16.
// ---------------------------------------------------------------------------
struct ConvArgs {
  const bf16* x;      // [H][W][C]
  const bf16* w;      // [9][C][C] (tap, out, in)
  const float* bias;  // [C] or null
  const bf16* mask;   // [H][W][C] or null: output channel c at p zeroed unless mask[p][c] > 0
  bf16* y;            // [H][W][C] or null
  float* y0;          // [H][W]: FP32 output channel 0, or null
  int H, W, relu;
};

constexpr int kTilesPerWave = 4;

__global__ void __launch_bounds__(256) k_conv(ConvArgs a) {
  const int lane = threadIdx.x & 63;
  const int ntiles = (a.H * a.W) / 32;
  const int first = (blockIdx.x * 4 + (threadIdx.x >> 6)) * kTilesPerWave;
  if (first >= ntiles) return;
  const int i = lane & 31, kh = lane >> 5;
  bf8 wv[TAPS][2];
#pragma unroll
  for (int tap = 0; tap < TAPS; ++tap)
#pragma unroll
    for (int h = 0; h < 2; ++h)
      wv[tap][h] = *reinterpret_cast<const bf8*>(a.w + (size_t)tap * C * C + (size_t)i * C + 16 * h + 8 * kh);
  const int co = i;
  const float bb = a.bias ? a.bias[co] : 0.f;
  for (int tile = first; tile < first + kTilesPerWave && tile < ntiles; ++tile) {
    const int p0 = tile * 32;
    const int y = p0 / a.W, x0 = p0 % a.W;  // W is a multiple of 32: one row per tile
    f16v acc = {};
#pragma unroll
    for (int tap = 0; tap < TAPS; ++tap) {
      const int yy = (y + tap / 3 - 1) & (a.H - 1);
      const int xx = (x0 + i + tap % 3 - 1) & (a.W - 1);
      const bf16* xp = a.x + ((size_t)yy * a.W + xx) * C + 8 * kh;
#pragma unroll
      for (int h = 0; h < 2; ++h)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf8*>(xp + 16 * h), wv[tap][h], acc,
                                                      0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const size_t p = (size_t)p0 + 8 * (v >> 2) + 4 * kh + (v & 3);
      float o = acc[v] + bb;
      if (a.relu) o = fmaxf(o, 0.f);
      if (a.mask && !(bf2f(a.mask[p * C + co]) > 0.f)) o = 0.f;
      if (a.y) a.y[p * C + co] = f2bf(o);
      if (a.y0 && co == 0) a.y0[p] = o;
    }
  }
}

// ---------------------------------------------------------------------------
// Convolution on an LDS tile: a block of four waves computes kRowsLds output
// rows x 128 points x 32 output channels.  The (kRowsLds + 2) x 130-point
// input tile with its periodic halo is staged once in LDS (64 B per point,
// the four 16-byte channel chunks of a point swizzled by ((q >> 1) & 3) so
// that the eight lanes of an LDS access phase hit distinct banks); wave w
// takes points 32 w .. 32 w + 31 of every row.  Each A fragment read from LDS
// (input row r, tap column kx, channel half) feeds the MFMAs of every output
// row it reaches (ky = r - o), so a wave reads 36 fragments for 72 MFMAs.
// The BF16 outputs are gathered in LDS (the input tile's space, once every
// wave has read it) and written as whole 16-byte channel chunks, the mask
// applied there.  IN3: the input is the solver's FP32 [n][3] triplets, packed
// to BF16 (zero channels 3..31) while the tile is staged.
// ---------------------------------------------------------------------------
constexpr int kRowsLds = 4;
constexpr int kTileW = 128;
constexpr int kTileQ = kTileW + 2;

__device__ __forceinline__ int swz(int q, int chunk) { return chunk ^ ((q >> 1) & 3); }

// The 8 BF16 values of x with those whose mask value is not > 0 zeroed.
__device__ __forceinline__ uint4 apply_mask(uint4 x, uint4 m) {
  uint32_t xv[4] = {x.x, x.y, x.z, x.w};
  const uint32_t mv[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t lo = bf2f((bf16)(mv[k] & 0xffffu)) > 0.f ? 0x0000ffffu : 0u;
    const uint32_t hi = bf2f((bf16)(mv[k] >> 16)) > 0.f ? 0xffff0000u : 0u;
    xv[k] &= lo | hi;
  }
  return make_uint4(xv[0], xv[1], xv[2], xv[3]);
}

template <bool IN3>
__global__ void __launch_bounds__(256) k_conv_lds(ConvArgs a, const float* __restrict__ in3) {
  __shared__ uint4 tile[(kRowsLds + 2) * kTileQ * 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 31, kh = lane >> 5;
  const int x0 = blockIdx.x * kTileW, y0 = blockIdx.y * kRowsLds;
  // stage the input rows y0 - 1 .. y0 + kRowsLds, points x0 - 1 .. x0 + kTileW
  if (IN3) {
    for (int c = tid; c < (kRowsLds + 2) * kTileQ; c += 256) {
      const int r = c / kTileQ, q = c % kTileQ;
      const size_t p = (size_t)((y0 - 1 + r) & (a.H - 1)) * a.W + ((x0 - 1 + q) & (a.W - 1));
      const uint32_t c0 = f2bf(in3[3 * p]), c1 = f2bf(in3[3 * p + 1]), c2 = f2bf(in3[3 * p + 2]);
      uint4* dst = tile + (r * kTileQ + q) * 4;
      dst[swz(q, 0)] = make_uint4(c0 | (c1 << 16), c2, 0u, 0u);
#pragma unroll
      for (int chunk = 1; chunk < 4; ++chunk) dst[swz(q, chunk)] = make_uint4(0u, 0u, 0u, 0u);
    }
  } else {
    for (int c = tid; c < (kRowsLds + 2) * kTileQ * 4; c += 256) {
      const int r = c / (kTileQ * 4), rem = c % (kTileQ * 4), q = rem >> 2, chunk = rem & 3;
      const size_t p = (size_t)((y0 - 1 + r) & (a.H - 1)) * a.W + ((x0 - 1 + q) & (a.W - 1));
      tile[(r * kTileQ + q) * 4 + swz(q, chunk)] = reinterpret_cast<const uint4*>(a.x + p * C)[chunk];
    }
  }
  bf8 wv[TAPS][2];
#pragma unroll
  for (int tap = 0; tap < TAPS; ++tap)
#pragma unroll
    for (int h = 0; h < 2; ++h)
      wv[tap][h] = *reinterpret_cast<const bf8*>(a.w + (size_t)tap * C * C + (size_t)i * C + 16 * h + 8 * kh);
  const int co = i;
  const float bb = a.bias ? a.bias[co] : 0.f;
  __syncthreads();
  f16v acc[kRowsLds] = {};
#pragma unroll
  for (int r = 0; r < kRowsLds + 2; ++r)
#pragma unroll
    for (int kx = 0; kx < 3; ++kx)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = 32 * wave + i + kx;
        const uint4 u = tile[(r * kTileQ + q) * 4 + swz(q, 2 * h + kh)];
        const bf8 av = __builtin_bit_cast(bf8, u);
#pragma unroll
        for (int o = 0; o < kRowsLds; ++o) {
          const int ky = r - o;
          if (ky >= 0 && ky <= 2)
            acc[o] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, wv[3 * ky + kx][h], acc[o], 0, 0, 0);
        }
      }
  __syncthreads();  // every wave has read its fragments: the tile space takes the outputs
  bf16* ob = reinterpret_cast<bf16*>(tile);
#pragma unroll
  for (int o = 0; o < kRowsLds; ++o) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int pt = 32 * wave + 8 * (v >> 2) + 4 * kh + (v & 3);
      float out = acc[o][v] + bb;
      if (a.relu) out = fmaxf(out, 0.f);
      if (a.y0 && co == 0) {
        const size_t p = (size_t)(y0 + o) * a.W + x0 + pt;
        a.y0[p] = (a.mask && !(bf2f(a.mask[p * C]) > 0.f)) ? 0.f : out;
      }
      ob[(o * kTileW + pt) * C + co] = f2bf(out);
    }
  }
  if (!a.y) return;
  __syncthreads();
  for (int u = tid; u < kRowsLds * kTileW * 4; u += 256) {
    const int o = u / (kTileW * 4), pt = (u >> 2) % kTileW, chunk = u & 3;
    const size_t p = (size_t)(y0 + o) * a.W + x0 + pt;
    uint4 val = tile[u];
    if (a.mask) val = apply_mask(val, reinterpret_cast<const uint4*>(a.mask + p * C)[chunk]);
    reinterpret_cast<uint4*>(a.y + p * C)[chunk] = val;
  }
}

// ---------------------------------------------------------------------------
// Weight and bias gradients: dw[tap][co][ci] = sum_p dz[p][co] x[p + off][ci],
// db[co] = sum_p dz[p][co].  A block walks row segments of SEG points, stages
// dz and the three input rows around the segment transposed in LDS ([c][p]),
// and each wave accumulates the 32 x 32 blocks of its taps (wave w: taps w,
// w + 4, w + 8) with A[co][k] = dz[k][co], B[k][ci] = x[k + off][ci].  Per-block
// partials [block][WL + C] are reduced by k_wgrad_reduce in a fixed order.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_wgrad(const bf16* __restrict__ dz, const bf16* __restrict__ x, int H,
                                               int W, float* __restrict__ part) {
  __shared__ bf16 sdz[C][SEG + 2];  // padded: rows of a wave's lanes on distinct banks
  __shared__ bf16 sx[3][C][SEG + 2];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int i = lane & 31, kh = lane >> 5;
  const int seg = W < SEG ? W : SEG;
  const int segs_row = W / seg;
  const int nseg = H * segs_row;
  f16v acc[3] = {};
  float db = 0.f;
  for (int s = blockIdx.x; s < nseg; s += gridDim.x) {
    const int y = s / segs_row, x0 = (s % segs_row) * seg;
    __syncthreads();
    for (int q = tid; q < seg; q += blockDim.x) {
      const uint4* src = reinterpret_cast<const uint4*>(dz + ((size_t)y * W + x0 + q) * C);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint4 r4 = src[u];
        const uint32_t w4[4] = {r4.x, r4.y, r4.z, r4.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          sdz[8 * u + 2 * k][q] = (bf16)(w4[k] & 0xffffu);
          sdz[8 * u + 2 * k + 1][q] = (bf16)(w4[k] >> 16);
        }
      }
    }
    for (int q = tid; q < 3 * (seg + 2); q += blockDim.x) {
      const int r = q / (seg + 2), qq = q % (seg + 2);
      const int yy = (y + r - 1) & (H - 1), xx = (x0 - 1 + qq) & (W - 1);
      const uint4* src = reinterpret_cast<const uint4*>(x + ((size_t)yy * W + xx) * C);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint4 r4 = src[u];
        const uint32_t w4[4] = {r4.x, r4.y, r4.z, r4.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          sx[r][8 * u + 2 * k][qq] = (bf16)(w4[k] & 0xffffu);
          sx[r][8 * u + 2 * k + 1][qq] = (bf16)(w4[k] >> 16);
        }
      }
    }
    __syncthreads();
    if (tid < C)
      for (int q = 0; q < seg; ++q) db += bf2f(sdz[tid][q]);
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int tap = wave + 4 * u;
      if (tap < TAPS) {
        const int ky = tap / 3, kx = tap % 3;
        for (int k0 = 0; k0 < seg; k0 += 16) {
          bf8 av, bv;
#pragma unroll
          for (int v = 0; v < 8; ++v) {
            av[v] = __builtin_bit_cast(__bf16, sdz[i][k0 + 8 * kh + v]);
            bv[v] = __builtin_bit_cast(__bf16, sx[ky][i][k0 + 8 * kh + v + kx]);
          }
          acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[u], 0, 0, 0);
        }
      }
    }
  }
  float* out = part + (size_t)blockIdx.x * PL;
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int tap = wave + 4 * u;
    if (tap < TAPS) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int co = 8 * (v >> 2) + 4 * kh + (v & 3), ci = i;
        out[tap * C * C + co * C + ci] = acc[u][v];
      }
    }
  }
  if (tid < C) out[WL + tid] = db;
}

// g[e] = sum over blocks b (in order) of part[b][e], e < PL; loads issued
// 16 blocks ahead, the additions kept in block order.
__global__ void __launch_bounds__(kRedThreads) k_wgrad_reduce(const float* __restrict__ part, int nblocks,
                                                              float* __restrict__ g) {
  const int e = blockIdx.x * kRedThreads + threadIdx.x;
  if (e >= PL) return;
  float s = 0.f;
  int b = 0;
  for (; b + 16 <= nblocks; b += 16) {
    float x[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) x[u] = part[(size_t)(b + u) * PL + e];
#pragma unroll
    for (int u = 0; u < 16; ++u) s += x[u];
  }
  for (; b < nblocks; ++b) s += part[(size_t)b * PL + e];
  g[e] = s;
}

// ---------------------------------------------------------------------------
// Loss, input packing, Adam
// ---------------------------------------------------------------------------
// d[p][0] = scale (pred[p] - t[p]), other channels 0; per-block sums of
// (pred - t)^2 in FP64.
__global__ void __launch_bounds__(256) k_mse_grad(const float* __restrict__ pred, const float* __restrict__ t,
                                                  bf16* __restrict__ d, double* __restrict__ part, int n,
                                                  float scale) {
  __shared__ double red[4];
  const int p = blockIdx.x * 256 + threadIdx.x;
  double e2 = 0.0;
  if (p < n) {
    const float e = pred[p] - t[p];
    e2 = (double)e * e;
    bf16* dp = d + (size_t)p * C;
    dp[0] = f2bf(scale * e);
#pragma unroll
    for (int c = 1; c < C; ++c) dp[c] = 0;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) e2 += __shfl_xor(e2, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e2;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// x[p][c] = in3[p][c] (c < 3), 0 for c >= 3 (four 16-byte stores per point).
__global__ void __launch_bounds__(256) k_pack3(const float* __restrict__ in3, bf16* __restrict__ x, int n) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  uint4* xp = reinterpret_cast<uint4*>(x + (size_t)p * C);
  const uint32_t c0 = f2bf(in3[(size_t)p * 3]), c1 = f2bf(in3[(size_t)p * 3 + 1]), c2 = f2bf(in3[(size_t)p * 3 + 2]);
  xp[0] = make_uint4(c0 | (c1 << 16), c2, 0u, 0u);
  xp[1] = make_uint4(0u, 0u, 0u, 0u);
  xp[2] = make_uint4(0u, 0u, 0u, 0u);
  xp[3] = make_uint4(0u, 0u, 0u, 0u);
}

// BF16 copies of the weights: wf[l][tap][co][ci] and, for the input gradient,
// wb[l][8 - tap][ci][co] (taps flipped, channels exchanged).
__device__ __forceinline__ void emit_bf16(int e, float w, bf16* wf, bf16* wb) {
  const int l = e / PL, r = e % PL;
  if (r >= WL) return;
  const int tap = r / (C * C), co = (r / C) % C, ci = r % C;
  const bf16 b = f2bf(w);
  wf[(size_t)l * WL + r] = b;
  wb[(size_t)l * WL + (TAPS - 1 - tap) * C * C + ci * C + co] = b;
}

__global__ void __launch_bounds__(256) k_emit(const float* __restrict__ w, bf16* wf, bf16* wb) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < NP) emit_bf16(e, w[e], wf, wb);
}

// One Adam step (Kingma & Ba, Algorithm 1) on every parameter; c1 = 1 / (1 -
// beta1^t), c2 = 1 / (1 - beta2^t).
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ w, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                              float b2, float eps, float c1, float c2, bf16* wf, bf16* wb) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= NP) return;
  const float ge = g[e];
  const float me = b1 * m[e] + (1.f - b1) * ge;
  const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
  m[e] = me;
  v[e] = ve;
  const float we = w[e] - lr * (me * c1) / (sqrtf(ve * c2) + eps);
  w[e] = we;
  emit_bf16(e, we, wf, wb);
}

}  // namespace sgnn

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
using namespace sgnn;

struct sgn_cnn {
  int H, W, n;
  hipStream_t stream;
  float *w, *g, *m, *v;   // FP32 master weights, gradients, Adam moments [NP]
  bf16 *wf, *wb;          // BF16 weights for the forward and input-gradient passes [L][WL]
  bf16* act[L + 1];       // act[0] = input, act[l + 1] = output of layer l
  bf16 *d0, *d1;          // gradients in the activations
  float* pred;            // FP32 output channel 0 [H][W]
  float* in3;             // input staging for the solver's learned guess [H][W][3]
  float* out;             // output staging for the solver's learned guess [H][W]
  float* part;            // weight-gradient partials [kWgBlocks][PL]
  double* lpart;          // loss partials
  double* hl;             // pinned host copy of the loss partials
  int t;                  // Adam steps taken
  std::string err;
};

namespace {

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct CnnLayout {
  size_t total;
  size_t off_w, off_g, off_m, off_v, off_wf, off_wb, off_act, off_d0, off_d1, off_pred, off_part, off_lpart, off_in3,
      off_out;
};

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

CnnLayout cnn_layout(int H, int W) {
  CnnLayout c{};
  const size_t n = (size_t)H * W;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += al(bytes);
    return at;
  };
  c.off_w = take(NP * 4);
  c.off_g = take(NP * 4);
  c.off_m = take(NP * 4);
  c.off_v = take(NP * 4);
  c.off_wf = take((size_t)L * WL * 2);
  c.off_wb = take((size_t)L * WL * 2);
  c.off_act = take((size_t)(L + 1) * al(n * C * 2));
  c.off_d0 = take(n * C * 2);
  c.off_d1 = take(n * C * 2);
  c.off_pred = take(n * 4);
  c.off_part = take((size_t)kWgBlocks * PL * 4);
  c.off_lpart = take(((n + 255) / 256) * 8);
  c.off_in3 = take(n * 3 * 4);
  c.off_out = take(n * 4);
  c.total = o;
  return c;
}

int cfail(sgn_cnn* c, hipError_t e, const char* what) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
  c->err = buf;
  return SGN_ERR_HIP;
}

#define CK(expr)                                       \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return cfail(c, e_, #expr);  \
  } while (0)

// The LDS-tile kernel needs whole 128-point row segments and 4-row bands.
bool lds_tiles(const sgn_cnn* c) { return c->W % kTileW == 0 && c->H % kRowsLds == 0; }

// One convolution layer; in3 (with x null): the layer reads the FP32 input
// triplets directly (LDS-tile grids only).
int conv(sgn_cnn* c, const bf16* x, const bf16* w, const float* bias, const bf16* mask, bf16* y, float* y0,
         int relu, const float* in3 = nullptr) {
  ConvArgs a{x, w, bias, mask, y, y0, c->H, c->W, relu};
  if (lds_tiles(c)) {
    const dim3 grid(c->W / kTileW, c->H / kRowsLds);
    if (in3)
      hipLaunchKernelGGL(k_conv_lds<true>, grid, dim3(256), 0, c->stream, a, in3);
    else
      hipLaunchKernelGGL(k_conv_lds<false>, grid, dim3(256), 0, c->stream, a, nullptr);
  } else {
    const int tiles = c->n / 32;
    const int per_block = 4 * kTilesPerWave;
    hipLaunchKernelGGL(k_conv, dim3((tiles + per_block - 1) / per_block), dim3(256), 0, c->stream, a);
  }
  CK(hipGetLastError());
  return SGN_OK;
}

// The six layers.  Inference on grids of the LDS-tile kernel reads the FP32
// input triplets in the first layer; otherwise (training, whose backward pass
// reads the packed input, or other grids) the input is packed first;
// the last layer writes only its FP32 output channel (the backward pass
// never reads the BF16 output of the last layer).
int forward_pass(sgn_cnn* c, const float* in3, bool keep_input = true) {
  const bool fused_input = !keep_input && lds_tiles(c);
  if (!fused_input) {
    hipLaunchKernelGGL(k_pack3, dim3((c->n + 255) / 256), dim3(256), 0, c->stream, in3, c->act[0], c->n);
    CK(hipGetLastError());
  }
  for (int l = 0; l < L; ++l) {
    const bool last = l == L - 1;
    int rc = conv(c, fused_input && l == 0 ? nullptr : c->act[l], c->wf + (size_t)l * WL,
                  c->w + (size_t)l * PL + WL, nullptr, last ? nullptr : c->act[l + 1], last ? c->pred : nullptr,
                  last ? 0 : 1, fused_input && l == 0 ? in3 : nullptr);
    if (rc) return rc;
  }
  return SGN_OK;
}

// Loss and gradients in c->g (FP32) for the current weights.
int backward_pass(sgn_cnn* c, const float* target, double* loss) {
  const int nb = (c->n + 255) / 256;
  hipLaunchKernelGGL(k_mse_grad, dim3(nb), dim3(256), 0, c->stream, c->pred, target, c->d0, c->lpart, c->n,
                     2.0f / (float)c->n);
  CK(hipGetLastError());
  bf16* d = c->d0;
  bf16* dn = c->d1;
  for (int l = L - 1; l >= 0; --l) {
    hipLaunchKernelGGL(k_wgrad, dim3(kWgBlocks), dim3(256), 0, c->stream, d, c->act[l], c->H, c->W, c->part);
    CK(hipGetLastError());
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((PL + kRedThreads - 1) / kRedThreads), dim3(kRedThreads), 0, c->stream,
                       c->part, kWgBlocks, c->g + (size_t)l * PL);
    CK(hipGetLastError());
    if (l > 0) {
      // through layer l's input ReLU: the input activation is the mask
      int rc = conv(c, d, c->wb + (size_t)l * WL, nullptr, c->act[l], dn, nullptr, 0);
      if (rc) return rc;
      bf16* tmp = d;
      d = dn;
      dn = tmp;
    }
  }
  if (loss) {
    CK(hipMemcpyAsync(c->hl, c->lpart, (size_t)nb * 8, hipMemcpyDeviceToHost, c->stream));
    CK(hipStreamSynchronize(c->stream));
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += c->hl[b];
    *loss = s / c->n;
  }
  return SGN_OK;
}

bool dev_ok(const void* p) { return p && (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

extern "C" {

size_t sgn_cnn_workspace_bytes(int32_t H, int32_t W) {
  if (!pow2(H) || !pow2(W) || W < 32 || H < 1 || (size_t)H * W > ((size_t)1 << 24)) return 0;
  return cnn_layout(H, W).total;
}

int sgn_cnn_init(int32_t H, int32_t W, void* ws, size_t ws_bytes, void* hip_stream, sgn_cnn** out) {
  if (!out) return SGN_ERR_INVALID_ARG;
  *out = nullptr;
  const size_t need = sgn_cnn_workspace_bytes(H, W);
  if (!need) return SGN_ERR_UNSUPPORTED;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0 || ws_bytes < need) return SGN_ERR_INVALID_ARG;
  const CnnLayout Lc = cnn_layout(H, W);
  sgn_cnn* c = new sgn_cnn();
  c->H = H;
  c->W = W;
  c->n = H * W;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  char* b = static_cast<char*>(ws);
  c->w = reinterpret_cast<float*>(b + Lc.off_w);
  c->g = reinterpret_cast<float*>(b + Lc.off_g);
  c->m = reinterpret_cast<float*>(b + Lc.off_m);
  c->v = reinterpret_cast<float*>(b + Lc.off_v);
  c->wf = reinterpret_cast<bf16*>(b + Lc.off_wf);
  c->wb = reinterpret_cast<bf16*>(b + Lc.off_wb);
  for (int l = 0; l <= L; ++l) c->act[l] = reinterpret_cast<bf16*>(b + Lc.off_act + (size_t)l * al((size_t)c->n * C * 2));
  c->d0 = reinterpret_cast<bf16*>(b + Lc.off_d0);
  c->d1 = reinterpret_cast<bf16*>(b + Lc.off_d1);
  c->pred = reinterpret_cast<float*>(b + Lc.off_pred);
  c->part = reinterpret_cast<float*>(b + Lc.off_part);
  c->lpart = reinterpret_cast<double*>(b + Lc.off_lpart);
  c->in3 = reinterpret_cast<float*>(b + Lc.off_in3);
  c->out = reinterpret_cast<float*>(b + Lc.off_out);
  c->t = 0;
  if (hipHostMalloc(reinterpret_cast<void**>(&c->hl), ((c->n + 255) / 256) * 8, 0) != hipSuccess) {
    delete c;
    return SGN_ERR_HIP;
  }
  // zero weights and moments until sgn_cnn_set_params
  hipError_t e = hipMemsetAsync(b + Lc.off_w, 0, Lc.off_wf - Lc.off_w, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(b + Lc.off_wf, 0, Lc.off_act - Lc.off_wf, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    (void)hipHostFree(c->hl);
    delete c;
    return SGN_ERR_HIP;
  }
  *out = c;
  return SGN_OK;
}

int sgn_cnn_destroy(sgn_cnn* c) {
  if (!c) return SGN_ERR_INVALID_ARG;
  if (c->hl) (void)hipHostFree(c->hl);
  delete c;
  return SGN_OK;
}

int sgn_cnn_set_params(sgn_cnn* c, const float* params) {
  if (!c || !params) return SGN_ERR_INVALID_ARG;
  CK(hipMemcpyAsync(c->w, params, NP * sizeof(float), hipMemcpyHostToDevice, c->stream));
  CK(hipMemsetAsync(c->m, 0, NP * sizeof(float), c->stream));
  CK(hipMemsetAsync(c->v, 0, NP * sizeof(float), c->stream));
  hipLaunchKernelGGL(k_emit, dim3((NP + 255) / 256), dim3(256), 0, c->stream, c->w, c->wf, c->wb);
  CK(hipGetLastError());
  CK(hipStreamSynchronize(c->stream));  // params is the caller's host memory
  c->t = 0;
  return SGN_OK;
}

int sgn_cnn_get_params(sgn_cnn* c, float* params) {
  if (!c || !params) return SGN_ERR_INVALID_ARG;
  CK(hipMemcpyAsync(params, c->w, NP * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  CK(hipStreamSynchronize(c->stream));
  return SGN_OK;
}

int sgn_cnn_forward(sgn_cnn* c, const float* in3, float* out) {
  if (!c || !dev_ok(in3) || !dev_ok(out)) return SGN_ERR_INVALID_ARG;
  int rc = forward_pass(c, in3, false);
  if (rc) return rc;
  CK(hipMemcpyAsync(out, c->pred, (size_t)c->n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  return SGN_OK;
}

int sgn_cnn_gradients(sgn_cnn* c, const float* in3, const float* target, float* grads, double* loss) {
  if (!c || !dev_ok(in3) || !dev_ok(target)) return SGN_ERR_INVALID_ARG;
  int rc = forward_pass(c, in3);
  if (!rc) rc = backward_pass(c, target, loss);
  if (rc) return rc;
  if (grads) {
    CK(hipMemcpyAsync(grads, c->g, NP * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    CK(hipStreamSynchronize(c->stream));
  }
  return SGN_OK;
}

int sgn_cnn_train_step(sgn_cnn* c, const float* in3, const float* target, float lr, double* loss) {
  if (!c || !dev_ok(in3) || !dev_ok(target) || !(lr >= 0.f) || !std::isfinite(lr)) return SGN_ERR_INVALID_ARG;
  int rc = forward_pass(c, in3);
  if (!rc) rc = backward_pass(c, target, loss);
  if (rc) return rc;
  c->t += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, c->t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, c->t)));
  hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, c->stream, c->w, c->g, c->m, c->v, lr, b1, b2,
                     eps, c1, c2, c->wf, c->wb);
  CK(hipGetLastError());
  return SGN_OK;
}

const char* sgn_cnn_last_error(const sgn_cnn* c) { return c ? c->err.c_str() : ""; }

}  // extern "C"

// ---- for the solver's learned guess (sgn_cnn_internal.hpp) ----------------
int sgn_cnn_grid(const sgn_cnn* c, int* H, int* W) {
  *H = c->H;
  *W = c->W;
  return SGN_OK;
}
float* sgn_cnn_in3_buffer(sgn_cnn* c) { return c->in3; }
float* sgn_cnn_out_buffer(sgn_cnn* c) { return c->out; }
int sgn_cnn_forward_on(sgn_cnn* c, const float* in3, float* out, hipStream_t s) {
  const hipStream_t own = c->stream;
  c->stream = s;
  int rc = forward_pass(c, in3, false);
  if (!rc && hipMemcpyAsync(out, c->pred, (size_t)c->n * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess)
    rc = SGN_ERR_HIP;
  c->stream = own;
  return rc;
}

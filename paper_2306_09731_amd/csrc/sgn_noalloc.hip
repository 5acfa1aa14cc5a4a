// sgn_apply_operator_noalloc: the elliptic operator (and optionally the
// preconditioner) of sgn_apply_operator with no context and no workspace.
// Its scratch -- the FP64 and FP32 twiddle tables and four x-half or 2D
// spectra -- lives in a file-scope device array that the library holds on
// every GPU it runs on until the process ends, so the call allocates nothing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>

#include "sgn.h"
#include "sgn_host.hpp"
#include "sgn_internal.hpp"
#include "sgn_launch.hpp"

namespace {

constexpr size_t kTablesBytes = 256 * 1024;  // (nx + ny) <= 8192 twiddles: 128 KiB FP64 + 64 KiB FP32
constexpr size_t kSlotBytes = (size_t)SGN_NOALLOC_MAX_POINTS * sizeof(double);
constexpr int kSlots = 4;
constexpr size_t kScratchBytes = kTablesBytes + kSlots * kSlotBytes;

// Device scratch of the call.  Host code never uses this name as an address:
// it is a host-side stand-in for the symbol; the device address comes from
// hipGetSymbolAddress, per device.
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_scratch[kMaxDevices] = {};  // device address of scratch, per device (null: not yet looked up)

// The twiddle tables exp(-2 pi i k / n), k < nx then k < ny, in FP64 and
// rounded to FP32, as the context's tables (sincospi takes the exact
// argument 2k/n, so each entry is within an ulp of the exact value).
__global__ void __launch_bounds__(256) k_fill_twiddles(double2* tw, float2* tw32, int nx, int ny) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nx + ny) return;
  const int n = k < nx ? nx : ny;
  const int kk = k < nx ? k : k - nx;
  double s, c;
  sincospi(2.0 * (double)kk / (double)n, &s, &c);
  tw[k] = make_double2(c, -s);
  tw32[k] = make_float2((float)c, (float)-s);
}

int fail_hip(hipError_t e, const char* what) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
  sgn::set_global_error(buf);
  return SGN_ERR_HIP;
}

// Device address of this device's scratch (looked up once per device, with
// that device current).
int scratch_address(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) {
    sgn::set_global_error("sgn_apply_operator_noalloc: device index beyond the supported 64");
    return SGN_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = static_cast<char*>(p);
  }
  *out = g_scratch[dev];
  return SGN_OK;
}

bool aligned16(const void* p) { return p && (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

extern "C" int sgn_apply_operator_noalloc(const sgn_config* cfg, const void* h, const void* s, void* out,
                                          int32_t precondition, void* hip_stream) {
  int rc = sgn::check_config(cfg);
  if (rc) {
    sgn::set_global_error("sgn_apply_operator_noalloc: invalid or unsupported configuration");
    return rc;
  }
  if (cfg->batch != 1 || !aligned16(h) || !aligned16(s) || !aligned16(out) || out == s || out == h) {
    sgn::set_global_error("sgn_apply_operator_noalloc: null, misaligned or aliased field");
    return SGN_ERR_INVALID_ARG;
  }
  if ((size_t)cfg->nx * (size_t)cfg->ny > (size_t)SGN_NOALLOC_MAX_POINTS) {
    char buf[256];
    snprintf(buf, sizeof buf,
             "sgn_apply_operator_noalloc: %d x %d grid exceeds the %d points its fixed scratch holds",
             cfg->nx, cfg->ny, SGN_NOALLOC_MAX_POINTS);
    sgn::set_global_error(buf);
    return SGN_ERR_UNSUPPORTED;
  }
  char* base = nullptr;
  if ((rc = scratch_address(&base))) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  sgn::Geom g;
  sgn::geom_init(*cfg, g);
  double2* tw = reinterpret_cast<double2*>(base);
  float2* tw32 = reinterpret_cast<float2*>(base + 128 * 1024);
  g.twx = tw;
  g.twy = tw + cfg->nx;
  g.twx32 = tw32;
  g.twy32 = tw32 + cfg->nx;
  char* slot[kSlots];
  for (int i = 0; i < kSlots; ++i) slot[i] = base + kTablesBytes + i * kSlotBytes;
  // every scratch region is written before it is read within the call, so
  // nothing depends on what an earlier call left there
  const int ntw = cfg->nx + cfg->ny;
  hipLaunchKernelGGL(k_fill_twiddles, dim3((ntw + 255) / 256), dim3(256), 0, st, tw, tw32, cfg->nx, cfg->ny);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_hip(e, "k_fill_twiddles");
  // the sequence of sgn_apply_operator with its six scratch fields folded
  // into four slots: E, G (spectra of s), then the 2D spectrum of s (unused,
  // into the P slot that the operator overwrites), P, Q, then F(L s) into
  // E's slot and its inverse y-transform into G's
  void *E = slot[0], *G = slot[1], *P = slot[2], *Q = slot[3];
  if ((e = sgn::launch_row_r2c(g, s, E, st)) != hipSuccess) return fail_hip(e, "row_r2c");
  if ((e = sgn::launch_col_fwd_eg(g, E, P, G, st)) != hipSuccess) return fail_hip(e, "col_fwd_eg");
  if ((e = sgn::launch_row_op(g, 0, E, G, h, nullptr, nullptr, P, Q, nullptr, nullptr, 0, 0, nullptr, st)) !=
      hipSuccess)
    return fail_hip(e, "row_op");
  if ((e = sgn::launch_col_apply(g, P, Q, precondition ? 1 : 0, E, st)) != hipSuccess) return fail_hip(e, "col_apply");
  if ((e = sgn::launch_col_inv(g, E, G, st)) != hipSuccess) return fail_hip(e, "col_inv");
  if ((e = sgn::launch_row_c2r(g, G, out, st)) != hipSuccess) return fail_hip(e, "row_c2r");
  return SGN_OK;
}

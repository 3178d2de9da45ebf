// Allocation-free form of the convolution weight gradient.
//
// hmg_conv3d_backward_weight splits the voxel sum of every weight over 64
// partial sums held in a caller-supplied workspace.  This form holds those
// partials in a fixed device array of this library instead, for callers that
// cannot allocate device memory (code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc).  It calls no allocating routine.
//
// The array lives in every GPU the library runs on until the process ends.
// In host code its name is only a stand-in for the device symbol: the device
// address is looked up once per device with hipGetSymbolAddress (that device
// current) and only that address is ever passed to kernels.  Every call on a
// GPU shares that GPU's array, so calls that overlap on one GPU (different
// streams or host threads) race; the kernels write every partial they later
// read, so nothing has to be cleared between calls.
#include <mutex>

#include "../../include/hmg_nn.h"
#include "hmg_internal.hpp"
#include "nn_internal.hpp"

namespace {

constexpr int64_t kScratchFloats = (int64_t)8 << 20;  // 32 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) float scratch[kScratchFloats];

std::mutex g_mu;
float* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
hipError_t scratch_address(float** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

int64_t hmg_conv3d_noalloc_scratch_floats(void) { return kScratchFloats; }

hmg_status hmg_conv3d_backward_weight_noalloc(void* hip_stream, const float* x, const float* dz,
                                              float* dw, float* dbias, int32_t B, int32_t Cin,
                                              int32_t Cout, int32_t D, int32_t H, int32_t W) {
  if (!x || !dz || !dw || B < 1 || Cin < 1 || Cout < 1 || Cout > 128 || Cin > 4096 || D < 1 ||
      H < 1 || W < 1 || (int64_t)B * D * H * W >= ((int64_t)1 << 31))
    return HMG_E_INVALID;
  if (hmg::nn_conv_work_floats(Cin, Cout) > kScratchFloats) return HMG_E_INVALID;
  float* work = nullptr;
  if (scratch_address(&work) != hipSuccess) return HMG_E_DEVICE;
  const int64_t V = (int64_t)D * H * W;
  hmg::nn_conv_backward_weight(hmg::TView{const_cast<float*>(x), Cin, Cin * V},
                               hmg::TView{const_cast<float*>(dz), Cout, Cout * V}, dw, dbias, work,
                               B, D, H, W, (hipStream_t)hip_stream);
  return hipGetLastError() == hipSuccess ? HMG_OK : HMG_E_DEVICE;
}

}  // extern "C"

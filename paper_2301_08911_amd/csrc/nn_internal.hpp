// Internal interface of the learned warm-start network (see include/hmg_nn.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace hmg {

// View of a [batch][channel][voxel] FP32 tensor: channel stride = voxels,
// sample stride = bstride (>= channels * voxels, larger inside a concatenation).
struct TView {
  float* p = nullptr;
  int c = 0;
  int64_t bstride = 0;
};

// ---- kernels (nn.hip)
// y = bias + conv(x, w) [ReLU]; dims (D, H, W) = (z, y, x) extents.
void nn_conv_forward(const TView& x, const float* w, const float* bias, const TView& y, int B,
                     int D, int H, int W, bool relu, hipStream_t st);
// dx += conv^T(dz, w)
void nn_conv_backward_data(const TView& dz, const float* w, const TView& dx, int B, int D, int H,
                           int W, hipStream_t st);
// dw += x (*) dz, db += sum dz; work: nn_conv_work_floats(...) floats
void nn_conv_backward_weight(const TView& x, const TView& dz, float* dw, float* db, float* work,
                             int B, int D, int H, int W, hipStream_t st);
int64_t nn_conv_work_floats(int Cin, int Cout);
void nn_relu_backward(const TView& y, const TView& dy, int B, int64_t V, hipStream_t st);
void nn_pool_forward(const TView& x, const TView& y, int B, int D, int H, int W, hipStream_t st);
void nn_pool_backward(const TView& dy, const TView& dx, int B, int D, int H, int W,
                      hipStream_t st);
void nn_up_forward(const TView& x, const TView& y, int B, int D, int H, int W, hipStream_t st);
void nn_up_backward(const TView& dy, const TView& dx, int B, int D, int H, int W,
                    hipStream_t st);
void nn_fill(float* p, int64_t n, float v, hipStream_t st);
void nn_mse(const float* y, const float* t, int64_t n, float* dy, double* part, int nblk,
            double* out_dev, hipStream_t st);
void nn_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
             float eps, float c1, float c2, hipStream_t st);

// ---- the encoder-decoder
class Net {
 public:
  Net(int levels, int base, int cin, int cout, hipStream_t st);
  ~Net();
  bool ok() const { return ok_; }
  int64_t param_count() const { return nparam_; }
  int in_channels() const { return cin_; }
  int out_channels() const { return cout_; }
  int min_dim() const { return 2 << (levels_ - 1); }
  int dim_multiple() const { return 1 << (levels_ - 1); }
  void init_params(uint64_t seed);  // host-side SplitMix64 + Box-Muller, then upload
  float* params() { return p_; }
  float* grads() { return g_; }
  // Returns an error message or empty.  The input is copied, so the caller
  // may release x and y before the matching backward.
  std::string forward(const float* x, int B, int D, float* y);
  std::string backward(const float* dy);
  void zero_grad();
  void adam(double lr, double b1, double b2, double eps, int step);
  hipStream_t stream() const { return st_; }

 private:
  struct Conv {
    int cin, cout;
    int64_t woff, boff;  // offsets into the flat parameter array
    bool relu;
  };
  std::string ensure(int B, int D);
  void free_work();

  int levels_, base_, cin_, cout_;
  hipStream_t st_;
  bool ok_ = false;
  std::vector<Conv> convs_;
  int64_t nparam_ = 0;
  float *p_ = nullptr, *g_ = nullptr, *m_ = nullptr, *v_ = nullptr;
  // work buffers (activations and their gradients), sized for cap_ voxels
  int64_t cap_ = 0;
  int B_ = 0, D_ = 0;
  const float* x_in_ = nullptr;
  float* y_out_ = nullptr;
  std::vector<float*> act_, grad_;
  float* work_ = nullptr;
  int64_t work_floats_ = 0;
};

}  // namespace hmg

struct hmg_nn_s;
// The network behind a C handle (defined with the handle).
hmg::Net* hmg_nn_internal(hmg_nn_s* h);

// extern "C" entry points of include/hmg_nn.h (network handle and single
// layers); hmg_warm_start lives with the solver it feeds.
#include <hip/hip_runtime.h>

#include <memory>
#include <string>

#include "../../include/hmg_nn.h"
#include "nn_internal.hpp"

struct hmg_nn_s {
  std::unique_ptr<hmg::Net> net;
  double* dscal = nullptr;  // device: loss
  double* part = nullptr;   // device: per-block partial sums of the loss
};

namespace {

constexpr int MSE_BLOCKS = 1024;

hmg_status sync_status(hipStream_t st) {
  if (hipStreamSynchronize(st) != hipSuccess) return HMG_E_DEVICE;
  return hipGetLastError() == hipSuccess ? HMG_OK : HMG_E_DEVICE;
}

bool conv_dims_ok(int32_t B, int32_t Cin, int32_t Cout, int32_t D, int32_t H, int32_t W) {
  if (B < 1 || Cin < 1 || Cout < 1 || Cout > 128 || Cin > 4096 || D < 1 || H < 1 || W < 1)
    return false;
  return (int64_t)B * D * H * W < ((int64_t)1 << 31);
}

}  // namespace

hmg::Net* hmg_nn_internal(hmg_nn_s* h) { return h->net.get(); }

extern "C" {

hmg_status hmg_nn_create(const hmg_nn_config* cfg, void* hip_stream, uint64_t seed, hmg_nn* out) {
  if (!cfg || !out) return HMG_E_INVALID;
  *out = nullptr;
  if (cfg->levels < 1 || cfg->levels > 5 || cfg->base_channels < 1 || cfg->base_channels > 32 ||
      cfg->in_channels < 1 || cfg->in_channels > 64 || cfg->out_channels < 1 ||
      cfg->out_channels > 128 || (cfg->base_channels << (cfg->levels - 1)) > 128)
    return HMG_E_INVALID;
  hmg_nn n = new hmg_nn_s;
  n->net.reset(new hmg::Net(cfg->levels, cfg->base_channels, cfg->in_channels,
                            cfg->out_channels, (hipStream_t)hip_stream));
  if (!n->net->ok() || hipMalloc((void**)&n->dscal, sizeof(double) * 8) != hipSuccess ||
      hipMalloc((void**)&n->part, sizeof(double) * MSE_BLOCKS) != hipSuccess) {
    hmg_nn_destroy(n);
    return HMG_E_OOM;
  }
  n->net->init_params(seed);
  *out = n;
  return sync_status((hipStream_t)hip_stream);
}

hmg_status hmg_nn_destroy(hmg_nn net) {
  if (!net) return HMG_OK;
  if (net->dscal) (void)hipFree(net->dscal);
  if (net->part) (void)hipFree(net->part);
  delete net;
  return HMG_OK;
}

hmg_status hmg_nn_param_count(hmg_nn net, int64_t* count_out) {
  if (!net || !count_out) return HMG_E_INVALID;
  *count_out = net->net->param_count();
  return HMG_OK;
}

hmg_status hmg_nn_get_params(hmg_nn net, float* host, int64_t count) {
  if (!net || !host || count != net->net->param_count()) return HMG_E_INVALID;
  hipStream_t st = net->net->stream();
  (void)hipMemcpyAsync(host, net->net->params(), sizeof(float) * count, hipMemcpyDeviceToHost, st);
  return sync_status(st);
}

hmg_status hmg_nn_set_params(hmg_nn net, const float* host, int64_t count) {
  if (!net || !host || count != net->net->param_count()) return HMG_E_INVALID;
  hipStream_t st = net->net->stream();
  (void)hipMemcpyAsync(net->net->params(), host, sizeof(float) * count, hipMemcpyHostToDevice, st);
  return sync_status(st);
}

hmg_status hmg_nn_get_grads(hmg_nn net, float* host, int64_t count) {
  if (!net || !host || count != net->net->param_count()) return HMG_E_INVALID;
  hipStream_t st = net->net->stream();
  (void)hipMemcpyAsync(host, net->net->grads(), sizeof(float) * count, hipMemcpyDeviceToHost, st);
  return sync_status(st);
}

hmg_status hmg_nn_forward(hmg_nn net, const float* x_dev, int32_t batch, int32_t dim,
                          float* y_dev) {
  if (!net || !x_dev || !y_dev) return HMG_E_INVALID;
  const std::string e = net->net->forward(x_dev, batch, dim, y_dev);
  if (e.empty()) return HMG_OK;
  return e.find("allocation") != std::string::npos ? HMG_E_OOM
         : e.find("dims") != std::string::npos     ? HMG_E_INVALID
                                                   : HMG_E_DEVICE;
}

hmg_status hmg_nn_backward(hmg_nn net, const float* dy_dev) {
  if (!net || !dy_dev) return HMG_E_INVALID;
  const std::string e = net->net->backward(dy_dev);
  if (e.empty()) return HMG_OK;
  return e.find("preceding") != std::string::npos ? HMG_E_STATE : HMG_E_DEVICE;
}

hmg_status hmg_nn_zero_grad(hmg_nn net) {
  if (!net) return HMG_E_INVALID;
  net->net->zero_grad();
  return HMG_OK;
}

hmg_status hmg_nn_adam_step(hmg_nn net, double lr, double beta1, double beta2, double eps,
                            int32_t step) {
  if (!net || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !(eps > 0.0) || step < 1)
    return HMG_E_INVALID;
  net->net->adam(lr, beta1, beta2, eps, step);
  return HMG_OK;
}

hmg_status hmg_nn_mse(hmg_nn net, const float* y_dev, const float* t_dev, int64_t count,
                      float* dy_dev, double* loss_out) {
  if (!net || !y_dev || !t_dev || !dy_dev || !loss_out || count < 1) return HMG_E_INVALID;
  hipStream_t st = net->net->stream();
  hmg::nn_mse(y_dev, t_dev, count, dy_dev, net->part, MSE_BLOCKS, net->dscal, st);
  (void)hipMemcpyAsync(loss_out, net->dscal, sizeof(double), hipMemcpyDeviceToHost, st);
  return sync_status(st);
}

hmg_status hmg_conv3d_forward(void* hip_stream, const float* x, const float* w, const float* bias,
                              float* y, int32_t B, int32_t Cin, int32_t Cout, int32_t D,
                              int32_t H, int32_t W, int32_t relu) {
  if (!x || !w || !y || !conv_dims_ok(B, Cin, Cout, D, H, W)) return HMG_E_INVALID;
  const int64_t V = (int64_t)D * H * W;
  hmg::nn_conv_forward(hmg::TView{const_cast<float*>(x), Cin, Cin * V}, w, bias,
                       hmg::TView{y, Cout, Cout * V}, B, D, H, W, relu != 0,
                       (hipStream_t)hip_stream);
  return hipGetLastError() == hipSuccess ? HMG_OK : HMG_E_DEVICE;
}

hmg_status hmg_conv3d_backward_data(void* hip_stream, const float* dz, const float* w, float* dx,
                                    int32_t B, int32_t Cin, int32_t Cout, int32_t D, int32_t H,
                                    int32_t W) {
  if (!dz || !w || !dx || !conv_dims_ok(B, Cin, Cout, D, H, W) || Cin > 128) return HMG_E_INVALID;
  const int64_t V = (int64_t)D * H * W;
  hmg::nn_conv_backward_data(hmg::TView{const_cast<float*>(dz), Cout, Cout * V}, w,
                             hmg::TView{dx, Cin, Cin * V}, B, D, H, W, (hipStream_t)hip_stream);
  return hipGetLastError() == hipSuccess ? HMG_OK : HMG_E_DEVICE;
}

hmg_status hmg_conv3d_backward_weight(void* hip_stream, const float* x, const float* dz,
                                      float* dw, float* dbias, float* work, int32_t B,
                                      int32_t Cin, int32_t Cout, int32_t D, int32_t H, int32_t W) {
  if (!x || !dz || !dw || !work || !conv_dims_ok(B, Cin, Cout, D, H, W)) return HMG_E_INVALID;
  const int64_t V = (int64_t)D * H * W;
  hmg::nn_conv_backward_weight(hmg::TView{const_cast<float*>(x), Cin, Cin * V},
                               hmg::TView{const_cast<float*>(dz), Cout, Cout * V}, dw, dbias, work,
                               B, D, H, W, (hipStream_t)hip_stream);
  return hipGetLastError() == hipSuccess ? HMG_OK : HMG_E_DEVICE;
}

int64_t hmg_conv3d_workspace(int32_t B, int32_t Cin, int32_t Cout, int32_t D, int32_t H,
                             int32_t W) {
  (void)B;
  (void)D;
  (void)H;
  (void)W;
  return hmg::nn_conv_work_floats(Cin, Cout);
}

}  // extern "C"

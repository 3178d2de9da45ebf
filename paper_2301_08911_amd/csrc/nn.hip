// Learned warm start: kernels and the encoder-decoder of include/hmg_nn.h.
//
// The 3x3x3 periodic convolutions are implicit GEMMs on the matrix cores with
// v_mfma_f32_16x16x16_bf16 (bf16 operands, FP32 accumulation).  Operand layout
// of that instruction for lane l = 16 g + i (i < 16, g < 4):
//   A (16 x 16, M x K): a[j] = A[i][4 g + j]
//   B (16 x 16, K x N): b[j] = B[4 g + j][i]
//   D (16 x 16, M x N): d[j] = D[4 g + j][i]
// Forward:        M = out channel, N = voxel, K = (in channel, tap).
// Backward data:  M = in channel,  N = voxel, K = (out channel, tap), shifts
//                 reversed (the adjoint of a circular shift).
// Backward weight: M = out channel, N = (in channel, tap), K = voxel; split
//                 over voxel ranges into per-split partials, then summed in a
//                 fixed order.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "hmg_internal.hpp"
#include "nn_internal.hpp"

namespace hmg {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int MTMAX = 8;  // up to 128 output rows (M) per wave

__device__ __forceinline__ short bf(float v) {
  return __builtin_bit_cast(short, (__bf16)v);
}

struct Dims {
  int D, H, W;
  int64_t V;  // D * H * W
};

// Voxel v shifted by tap t (sign +1 forward, -1 adjoint) with periodic wrap.
__device__ __forceinline__ int64_t shifted(const Dims& d, int x, int y, int z, int t, int sign) {
  const int dx = (t % 3 - 1) * sign, dy = ((t / 3) % 3 - 1) * sign, dz = (t / 9 - 1) * sign;
  int xx = x + dx, yy = y + dy, zz = z + dz;
  xx = xx < 0 ? xx + d.W : (xx >= d.W ? xx - d.W : xx);
  yy = yy < 0 ? yy + d.H : (yy >= d.H ? yy - d.H : yy);
  zz = zz < 0 ? zz + d.D : (zz >= d.D ? zz - d.D : zz);
  return ((int64_t)zz * d.H + yy) * d.W + xx;
}

// FWD (ADJ = false): y[b, m, v] = act(bias[m] + sum_k w[m, k] x[b, ci(k), v + t(k)])
// ADJ = true: y[b, m, v] += sum_{co, t} w[co, m, t] x[b, co, v - t]   (x holds dz)
// One wave = 16 voxels x all M rows; 4 waves per block.
template <bool ADJ>
__global__ void __launch_bounds__(256) conv_kernel(const float* __restrict__ x, int64_t xbs,
                                                   int xc, const float* __restrict__ w,
                                                   const float* __restrict__ bias,
                                                   float* __restrict__ y, int64_t ybs, int M,
                                                   Dims d, int64_t nvox_total, int relu) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int64_t vb = ((int64_t)blockIdx.x * 4 + wave) * 16;  // first voxel of this wave (b*V + v)
  if (vb >= nvox_total) return;                              // whole wave idle (uniform)
  // this lane's voxel (column i); a wave may span two samples when V < 16
  const int64_t gv = vb + i;
  const bool live = gv < nvox_total;
  const int b = live ? (int)(gv / d.V) : 0;
  const int64_t v = live ? gv - (int64_t)b * d.V : 0;
  const int x0 = (int)(v % d.W), y0 = (int)((v / d.W) % d.H), z0 = (int)(v / ((int64_t)d.W * d.H));
  const float* xb = x + (int64_t)b * xbs;
  const int K = xc * 27;  // K = (input channel of the GEMM, tap)
  const int MT = (M + 15) / 16;
  const int Cin_w = ADJ ? M : xc;  // second extent of w[co][ci][27]
  f4 acc[MTMAX];
#pragma unroll
  for (int mt = 0; mt < MTMAX; ++mt) acc[mt] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    s4 bo;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + 4 * g + j;
      float val = 0.f;
      if (k < K && live) {
        const int c = k / 27, t = k - 27 * (k / 27);
        val = xb[(int64_t)c * d.V + shifted(d, x0, y0, z0, t, ADJ ? -1 : 1)];
      }
      bo[j] = bf(val);
    }
#pragma unroll
    for (int mt = 0; mt < MTMAX; ++mt) {
      if (mt >= MT) break;
      s4 ao;
      const int m = mt * 16 + i;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = k0 + 4 * g + j;
        float val = 0.f;
        if (k < K && m < M) {
          if (!ADJ) {
            val = w[(int64_t)m * K + k];
          } else {
            const int co = k / 27, t = k - 27 * (k / 27);
            val = w[((int64_t)co * Cin_w + m) * 27 + t];
          }
        }
        ao[j] = bf(val);
      }
      acc[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ao, bo, acc[mt], 0, 0, 0);
    }
  }
  float* yb = y + (int64_t)b * ybs;
#pragma unroll
  for (int mt = 0; mt < MTMAX; ++mt) {
    if (mt >= MT) break;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = mt * 16 + 4 * g + j;
      if (m >= M || !live) continue;
      float* o = yb + (int64_t)m * d.V + v;
      if (!ADJ) {
        float r = acc[mt][j] + (bias ? bias[m] : 0.f);
        if (relu && r < 0.f) r = 0.f;
        *o = r;
      } else {
        *o += acc[mt][j];
      }
    }
  }
}

// Partial weight gradients: part[split][m][n] = sum over this split's voxels of
// dz[b, m, v] x[b, ci(n), v + t(n)], M = Cout rows, N = Cin * 27 columns.
// Block (4 waves) = one 16 x 16 (m, n) tile of one split; the waves take
// interleaved 16-voxel chunks and are summed through LDS in a fixed order.
__global__ void __launch_bounds__(256) conv_wgrad_kernel(const float* __restrict__ x, int64_t xbs,
                                                         int Cin, const float* __restrict__ dz,
                                                         int64_t zbs, int Cout, Dims d, int B,
                                                         int chunks_per_split,
                                                         float* __restrict__ part) {
  __shared__ float red[4][64][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int N = Cin * 27;
  const int NT = (N + 15) / 16;
  const int mt = blockIdx.x / NT, nt = blockIdx.x - (blockIdx.x / NT) * NT;
  const int split = blockIdx.y;
  const int64_t nvox = (int64_t)B * d.V;
  const int64_t nchunks = (nvox + 15) / 16;
  const int m = mt * 16 + i;   // A row of this lane
  const int n = nt * 16 + i;   // B column of this lane
  const int ci = n / 27, t = n - 27 * (n / 27);
  f4 acc = f4{0.f, 0.f, 0.f, 0.f};
  const int64_t c0 = (int64_t)split * chunks_per_split;
  for (int q = wave; q < chunks_per_split; q += 4) {
    const int64_t ch = c0 + q;
    if (ch >= nchunks) break;
    s4 ao, bo;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      // voxel 4 g + j of the chunk; chunks may span samples when V < 16
      const int64_t gv = ch * 16 + 4 * g + j;
      const bool live = gv < nvox;
      const int b = live ? (int)(gv / d.V) : 0;
      const int64_t v = live ? gv - (int64_t)b * d.V : 0;
      ao[j] = bf(m < Cout && live ? dz[(int64_t)b * zbs + (int64_t)m * d.V + v] : 0.f);
      float xv = 0.f;
      if (n < N && live) {
        const int x0 = (int)(v % d.W), y0 = (int)((v / d.W) % d.H);
        const int z0 = (int)(v / ((int64_t)d.W * d.H));
        xv = x[(int64_t)b * xbs + (int64_t)ci * d.V + shifted(d, x0, y0, z0, t, 1)];
      }
      bo[j] = bf(xv);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ao, bo, acc, 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) red[wave][lane][j] = acc[j];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float s = ((red[0][lane][j] + red[1][lane][j]) + red[2][lane][j]) + red[3][lane][j];
      const int mm = mt * 16 + 4 * g + j;
      if (mm < Cout && n < N) part[((int64_t)split * Cout + mm) * N + n] = s;
    }
  }
}

__global__ void wgrad_reduce_kernel(const float* __restrict__ part, int nsplit, int64_t MN,
                                    float* __restrict__ dw) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < MN;
       e += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * MN + e];
    dw[e] += s;
  }
}

// db[m] += sum_{b, v} dz[b, m, v]: one block per channel, fixed order.
__global__ void __launch_bounds__(256) bgrad_kernel(const float* __restrict__ dz, int64_t zbs,
                                                    int64_t V, int B, float* __restrict__ db) {
  __shared__ double red[256];
  const int m = blockIdx.x;
  double s = 0.0;
  for (int b = 0; b < B; ++b)
    for (int64_t v = threadIdx.x; v < V; v += blockDim.x) s += dz[(int64_t)b * zbs + m * V + v];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[m] += (float)red[0];
}

__global__ void relu_bwd_kernel(const float* __restrict__ y, int64_t ybs, float* __restrict__ dy,
                                int64_t dbs, int C, int64_t V, int B) {
  const int64_t per = (int64_t)C * V, total = per * B;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / per);
    const int64_t r = e - b * per;
    if (!(y[b * ybs + r] > 0.f)) dy[b * dbs + r] = 0.f;
  }
}

// Coarse voxel (X, Y, Z) of a fine (D, H, W) grid owns fine voxels (2X + a, ...).
__global__ void pool_fwd_kernel(const float* __restrict__ x, int64_t xbs, float* __restrict__ y,
                                int64_t ybs, int C, Dims f, int B) {
  const int Dc = f.D / 2, Hc = f.H / 2, Wc = f.W / 2;
  const int64_t Vc = (int64_t)Dc * Hc * Wc, per = C * Vc, total = per * B;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / per);
    const int64_t r = e - b * per;
    const int c = (int)(r / Vc);
    const int64_t vc = r - (int64_t)c * Vc;
    const int X = (int)(vc % Wc), Y = (int)((vc / Wc) % Hc), Z = (int)(vc / ((int64_t)Wc * Hc));
    const float* xc = x + b * xbs + (int64_t)c * f.V;
    float s = 0.f;
    for (int a = 0; a < 8; ++a)
      s += xc[((int64_t)(2 * Z + (a >> 2)) * f.H + 2 * Y + ((a >> 1) & 1)) * f.W + 2 * X + (a & 1)];
    y[b * ybs + r] = 0.125f * s;
  }
}

__global__ void pool_bwd_kernel(const float* __restrict__ dy, int64_t ybs, float* __restrict__ dx,
                                int64_t xbs, int C, Dims f, int B) {
  const int Hc = f.H / 2, Wc = f.W / 2;
  const int64_t Vc = (int64_t)(f.D / 2) * Hc * Wc, per = C * f.V, total = per * B;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / per);
    const int64_t r = e - b * per;
    const int c = (int)(r / f.V);
    const int64_t v = r - (int64_t)c * f.V;
    const int xx = (int)(v % f.W), yy = (int)((v / f.W) % f.H), zz = (int)(v / ((int64_t)f.W * f.H));
    const int64_t vc = ((int64_t)(zz >> 1) * Hc + (yy >> 1)) * Wc + (xx >> 1);
    dx[b * xbs + r] += 0.125f * dy[b * ybs + (int64_t)c * Vc + vc];
  }
}

// Nearest-neighbour 2x upsampling from the coarse grid (f = fine dims).
__global__ void up_fwd_kernel(const float* __restrict__ x, int64_t xbs, float* __restrict__ y,
                              int64_t ybs, int C, Dims f, int B) {
  const int Hc = f.H / 2, Wc = f.W / 2;
  const int64_t Vc = (int64_t)(f.D / 2) * Hc * Wc, per = C * f.V, total = per * B;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / per);
    const int64_t r = e - b * per;
    const int c = (int)(r / f.V);
    const int64_t v = r - (int64_t)c * f.V;
    const int xx = (int)(v % f.W), yy = (int)((v / f.W) % f.H), zz = (int)(v / ((int64_t)f.W * f.H));
    const int64_t vc = ((int64_t)(zz >> 1) * Hc + (yy >> 1)) * Wc + (xx >> 1);
    y[b * ybs + r] = x[b * xbs + (int64_t)c * Vc + vc];
  }
}

__global__ void up_bwd_kernel(const float* __restrict__ dy, int64_t ybs, float* __restrict__ dx,
                              int64_t xbs, int C, Dims f, int B) {
  const int Dc = f.D / 2, Hc = f.H / 2, Wc = f.W / 2;
  const int64_t Vc = (int64_t)Dc * Hc * Wc, per = C * Vc, total = per * B;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / per);
    const int64_t r = e - b * per;
    const int c = (int)(r / Vc);
    const int64_t vc = r - (int64_t)c * Vc;
    const int X = (int)(vc % Wc), Y = (int)((vc / Wc) % Hc), Z = (int)(vc / ((int64_t)Wc * Hc));
    const float* dyc = dy + b * ybs + (int64_t)c * f.V;
    float s = 0.f;
    for (int a = 0; a < 8; ++a)
      s += dyc[((int64_t)(2 * Z + (a >> 2)) * f.H + 2 * Y + ((a >> 1) & 1)) * f.W + 2 * X + (a & 1)];
    dx[b * xbs + r] += s;
  }
}

__global__ void fill_f_kernel(float* __restrict__ p, int64_t n, float v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

__global__ void __launch_bounds__(256) mse_kernel(const float* __restrict__ y,
                                                  const float* __restrict__ t, int64_t n,
                                                  float* __restrict__ dy, double* part) {
  __shared__ double red[256];
  double s = 0.0;
  const float sc = 2.0f / (float)n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float dlt = y[e] - t[e];
    dy[e] = sc * dlt;
    s += (double)dlt * (double)dlt;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_part_kernel(const double* part, int nblk, int64_t n, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < nblk; ++k) s += part[k];
    *out = s / (double)n;
  }
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  return (int)(b < 1 ? 1 : b);
}

Dims dims(int D, int H, int W) { return Dims{D, H, W, (int64_t)D * H * W}; }

constexpr int WG_SPLITS = 64;

}  // namespace

// ------------------------------------------------------------------ launchers
void nn_conv_forward(const TView& x, const float* w, const float* bias, const TView& y, int B,
                     int D, int H, int W, bool relu, hipStream_t st) {
  const Dims d = dims(D, H, W);
  const int64_t tot = (int64_t)B * d.V;
  hipLaunchKernelGGL(conv_kernel<false>, dim3((unsigned)(((tot + 15) / 16 + 3) / 4)), dim3(256), 0, st,
                     x.p, x.bstride, x.c, w, bias, y.p, y.bstride, y.c, d, tot, relu ? 1 : 0);
}

void nn_conv_backward_data(const TView& dz, const float* w, const TView& dx, int B, int D, int H,
                           int W, hipStream_t st) {
  const Dims d = dims(D, H, W);
  const int64_t tot = (int64_t)B * d.V;
  hipLaunchKernelGGL(conv_kernel<true>, dim3((unsigned)(((tot + 15) / 16 + 3) / 4)), dim3(256), 0, st,
                     dz.p, dz.bstride, dz.c, w, (const float*)nullptr, dx.p, dx.bstride, dx.c, d,
                     tot, 0);
}

int64_t nn_conv_work_floats(int Cin, int Cout) { return (int64_t)WG_SPLITS * Cout * Cin * 27; }

void nn_conv_backward_weight(const TView& x, const TView& dz, float* dw, float* db, float* work,
                             int B, int D, int H, int W, hipStream_t st) {
  const Dims d = dims(D, H, W);
  const int Cin = x.c, Cout = dz.c, N = Cin * 27;
  const int64_t nchunks = ((int64_t)B * d.V + 15) / 16;
  const int per = (int)((nchunks + WG_SPLITS - 1) / WG_SPLITS);
  const int nsplit = (int)((nchunks + per - 1) / per);
  const int tiles = ((Cout + 15) / 16) * ((N + 15) / 16);
  hipLaunchKernelGGL(conv_wgrad_kernel, dim3(tiles, nsplit), dim3(256), 0, st, x.p, x.bstride, Cin,
                     dz.p, dz.bstride, Cout, d, B, per, work);
  const int64_t MN = (int64_t)Cout * N;
  hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(grid_for(MN)), dim3(256), 0, st, work, nsplit, MN,
                     dw);
  if (db)
    hipLaunchKernelGGL(bgrad_kernel, dim3(Cout), dim3(256), 0, st, dz.p, dz.bstride, d.V, B, db);
}

void nn_relu_backward(const TView& y, const TView& dy, int B, int64_t V, hipStream_t st) {
  hipLaunchKernelGGL(relu_bwd_kernel, dim3(grid_for((int64_t)B * y.c * V)), dim3(256), 0, st, y.p,
                     y.bstride, dy.p, dy.bstride, y.c, V, B);
}
void nn_pool_forward(const TView& x, const TView& y, int B, int D, int H, int W, hipStream_t st) {
  hipLaunchKernelGGL(pool_fwd_kernel, dim3(grid_for((int64_t)B * x.c * D * H * W / 8)), dim3(256),
                     0, st, x.p, x.bstride, y.p, y.bstride, x.c, dims(D, H, W), B);
}
void nn_pool_backward(const TView& dy, const TView& dx, int B, int D, int H, int W,
                      hipStream_t st) {
  hipLaunchKernelGGL(pool_bwd_kernel, dim3(grid_for((int64_t)B * dx.c * D * H * W)), dim3(256), 0,
                     st, dy.p, dy.bstride, dx.p, dx.bstride, dx.c, dims(D, H, W), B);
}
void nn_up_forward(const TView& x, const TView& y, int B, int D, int H, int W, hipStream_t st) {
  hipLaunchKernelGGL(up_fwd_kernel, dim3(grid_for((int64_t)B * x.c * D * H * W)), dim3(256), 0, st,
                     x.p, x.bstride, y.p, y.bstride, x.c, dims(D, H, W), B);
}
void nn_up_backward(const TView& dy, const TView& dx, int B, int D, int H, int W,
                    hipStream_t st) {
  hipLaunchKernelGGL(up_bwd_kernel, dim3(grid_for((int64_t)B * dx.c * D * H * W / 8)), dim3(256),
                     0, st, dy.p, dy.bstride, dx.p, dx.bstride, dx.c, dims(D, H, W), B);
}
void nn_fill(float* p, int64_t n, float v, hipStream_t st) {
  hipLaunchKernelGGL(fill_f_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
}
void nn_mse(const float* y, const float* t, int64_t n, float* dy, double* part, int nblk,
            double* out_dev, hipStream_t st) {
  hipLaunchKernelGGL(mse_kernel, dim3(nblk), dim3(256), 0, st, y, t, n, dy, part);
  hipLaunchKernelGGL(sum_part_kernel, dim3(1), dim3(64), 0, st, part, nblk, n, out_dev);
}
void nn_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
             float eps, float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2,
                     eps, c1, c2);
}

// ------------------------------------------------------------------ the network
Net::Net(int levels, int base, int cin, int cout, hipStream_t st)
    : levels_(levels), base_(base), cin_(cin), cout_(cout), st_(st) {
  auto ch = [&](int l) { return base_ << l; };
  // encoder: two convs per level; decoder: two convs per level above the
  // bottom (input = up(level below) ++ skip); then the linear output conv
  for (int l = 0; l < levels_; ++l) {
    convs_.push_back({l == 0 ? cin_ : ch(l - 1), ch(l), 0, 0, true});
    convs_.push_back({ch(l), ch(l), 0, 0, true});
  }
  for (int l = levels_ - 2; l >= 0; --l) {
    convs_.push_back({ch(l + 1) + ch(l), ch(l), 0, 0, true});
    convs_.push_back({ch(l), ch(l), 0, 0, true});
  }
  convs_.push_back({ch(0), cout_, 0, 0, false});
  int64_t off = 0;
  for (auto& c : convs_) {
    c.woff = off;
    off += (int64_t)c.cout * c.cin * 27;
  }
  for (auto& c : convs_) {
    c.boff = off;
    off += c.cout;
  }
  nparam_ = off;
  int64_t wmax = 0;
  for (auto& c : convs_) wmax = std::max<int64_t>(wmax, nn_conv_work_floats(c.cin, c.cout));
  work_floats_ = wmax;
  ok_ = hipMalloc((void**)&p_, sizeof(float) * nparam_) == hipSuccess &&
        hipMalloc((void**)&g_, sizeof(float) * nparam_) == hipSuccess &&
        hipMalloc((void**)&m_, sizeof(float) * nparam_) == hipSuccess &&
        hipMalloc((void**)&v_, sizeof(float) * nparam_) == hipSuccess &&
        hipMalloc((void**)&work_, sizeof(float) * work_floats_) == hipSuccess;
  if (ok_) {
    nn_fill(g_, nparam_, 0.f, st_);
    nn_fill(m_, nparam_, 0.f, st_);
    nn_fill(v_, nparam_, 0.f, st_);
  }
}

Net::~Net() {
  free_work();
  for (float* q : {p_, g_, m_, v_, work_})
    if (q) (void)hipFree(q);
}

void Net::free_work() {
  (void)hipStreamSynchronize(st_);
  for (float* q : act_)
    if (q) (void)hipFree(q);
  for (float* q : grad_)
    if (q) (void)hipFree(q);
  act_.clear();
  grad_.clear();
  cap_ = 0;
}

void Net::init_params(uint64_t seed) {
  std::vector<float> h(nparam_, 0.f);
  uint64_t ctr = 0;
  auto next = [&]() {  // SplitMix64 (Steele, Lea, Flood 2014) over a counter
    uint64_t z = (seed * 0x9E3779B97F4A7C15ull) ^ (ctr++ + 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return ((z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  };
  for (auto& c : convs_) {
    const double sd = std::sqrt(2.0 / (27.0 * c.cin)) * (c.relu ? 1.0 : 0.1);  // He normal
    for (int64_t e = 0; e < (int64_t)c.cout * c.cin * 27; ++e) {
      const double u1 = next(), u2 = next();
      h[c.woff + e] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
    }
  }
  (void)hipMemcpyAsync(p_, h.data(), sizeof(float) * nparam_, hipMemcpyHostToDevice, st_);
  (void)hipStreamSynchronize(st_);
}

// Activation layout per level l (dims D_l = D >> l, V_l = D_l^3, channels c_l):
//   buffer 4l+0: enc_a  [c_l]         first encoder conv
//   buffer 4l+1: cat    [c_{l+1}+c_l] (up of the level below ++ skip), or the
//                bottom output [c_l] at the last level
//   buffer 4l+2: pool   [c_{l-1}]     pooled skip of level l-1 (l >= 1)
//   buffer 4l+3: dec    [2 c_l]       the two decoder convs (a then b)
std::string Net::ensure(int B, int D) {
  const int64_t need = (int64_t)B * D * D * D;
  if (need <= cap_ && B == B_ && D == D_) return "";
  if (need > cap_) {
    free_work();
    auto ch = [&](int l) { return (int64_t)(base_ << l); };
    for (int l = 0; l < levels_; ++l) {
      const int64_t Vl = need >> (3 * l);
      const int64_t sizes[4] = {ch(l) * Vl, (l + 1 < levels_ ? ch(l + 1) + ch(l) : ch(l)) * Vl,
                                l >= 1 ? ch(l - 1) * Vl : 0, 2 * ch(l) * Vl};
      for (int k = 0; k < 4; ++k) {
        float *a = nullptr, *g = nullptr;
        if (sizes[k] > 0) {
          if (hipMalloc((void**)&a, sizeof(float) * sizes[k]) != hipSuccess ||
              hipMalloc((void**)&g, sizeof(float) * sizes[k]) != hipSuccess)
            return "device allocation of network activations failed";
        }
        act_.push_back(a);
        grad_.push_back(g);
      }
    }
    float* xin = nullptr;  // copy of the input, kept for the first layer's gradient
    if (hipMalloc((void**)&xin, sizeof(float) * cin_ * need) != hipSuccess)
      return "device allocation of network activations failed";
    act_.push_back(xin);
    grad_.push_back(nullptr);
    cap_ = need;
  }
  B_ = B;
  D_ = D;
  return "";
}

std::string Net::forward(const float* x, int B, int D, float* y) {
  if (B < 1 || D < min_dim() || D % dim_multiple())
    return "network input dims must be a multiple of 2^(levels-1), at least 2^levels";
  std::string e = ensure(B, D);
  if (!e.empty()) return e;
  float* xcopy = act_[4 * levels_];
  (void)hipMemcpyAsync(xcopy, x, sizeof(float) * cin_ * (int64_t)B * D * D * D,
                       hipMemcpyDeviceToDevice, st_);
  x_in_ = xcopy;
  y_out_ = y;
  auto ch = [&](int l) { return base_ << l; };
  auto V = [&](int l) { return (int64_t)(D >> l) * (D >> l) * (D >> l); };
  auto catc = [&](int l) { return l + 1 < levels_ ? ch(l + 1) + ch(l) : ch(l); };
  auto encA = [&](int l) { return TView{act_[4 * l], ch(l), ch(l) * V(l)}; };
  auto cat = [&](int l) { return TView{act_[4 * l + 1], catc(l), catc(l) * V(l)}; };
  auto skip = [&](int l) {  // second encoder output: the tail of cat (or the bottom)
    const int off = l + 1 < levels_ ? ch(l + 1) : 0;
    return TView{act_[4 * l + 1] + off * V(l), ch(l), catc(l) * V(l)};
  };
  auto pool = [&](int l) { return TView{act_[4 * l + 2], ch(l - 1), ch(l - 1) * V(l)}; };
  auto decA = [&](int l) { return TView{act_[4 * l + 3], ch(l), 2 * ch(l) * V(l)}; };
  auto decB = [&](int l) { return TView{act_[4 * l + 3] + ch(l) * V(l), ch(l), 2 * ch(l) * V(l)}; };
  int ci = 0;
  for (int l = 0; l < levels_; ++l) {
    const int Dl = D >> l;
    TView in = l == 0 ? TView{const_cast<float*>(x), cin_, cin_ * V(0)} : pool(l);
    if (l >= 1) nn_pool_forward(skip(l - 1), pool(l), B, 2 * Dl, 2 * Dl, 2 * Dl, st_);
    const Conv& a = convs_[ci++];
    nn_conv_forward(in, p_ + a.woff, p_ + a.boff, encA(l), B, Dl, Dl, Dl, true, st_);
    const Conv& b = convs_[ci++];
    nn_conv_forward(encA(l), p_ + b.woff, p_ + b.boff, skip(l), B, Dl, Dl, Dl, true, st_);
  }
  for (int l = levels_ - 2; l >= 0; --l) {
    const int Dl = D >> l;
    TView src = (l + 1 == levels_ - 1) ? skip(l + 1) : decB(l + 1);
    nn_up_forward(src, TView{cat(l).p, ch(l + 1), cat(l).bstride}, B, Dl, Dl, Dl, st_);
    const Conv& a = convs_[ci++];
    nn_conv_forward(cat(l), p_ + a.woff, p_ + a.boff, decA(l), B, Dl, Dl, Dl, true, st_);
    const Conv& b = convs_[ci++];
    nn_conv_forward(decA(l), p_ + b.woff, p_ + b.boff, decB(l), B, Dl, Dl, Dl, true, st_);
  }
  TView top = levels_ > 1 ? decB(0) : skip(0);
  const Conv& o = convs_[ci++];
  nn_conv_forward(top, p_ + o.woff, p_ + o.boff, TView{y, cout_, cout_ * V(0)}, B, D, D, D, false,
                  st_);
  const hipError_t err = hipGetLastError();
  return err == hipSuccess ? "" : std::string("network forward: ") + hipGetErrorString(err);
}

std::string Net::backward(const float* dy) {
  if (!y_out_) return "hmg_nn_backward needs a preceding hmg_nn_forward";
  const int B = B_, D = D_;
  auto ch = [&](int l) { return base_ << l; };
  auto V = [&](int l) { return (int64_t)(D >> l) * (D >> l) * (D >> l); };
  auto catc = [&](int l) { return l + 1 < levels_ ? ch(l + 1) + ch(l) : ch(l); };
  auto vw = [&](const std::vector<float*>& bufs, int k, int64_t off, int c, int64_t bs) {
    return TView{bufs[k] + off, c, bs};
  };
  auto encA = [&](const std::vector<float*>& s, int l) { return vw(s, 4 * l, 0, ch(l), ch(l) * V(l)); };
  auto cat = [&](const std::vector<float*>& s, int l) {
    return vw(s, 4 * l + 1, 0, catc(l), catc(l) * V(l));
  };
  auto skip = [&](const std::vector<float*>& s, int l) {
    const int off = l + 1 < levels_ ? ch(l + 1) : 0;
    return vw(s, 4 * l + 1, off * V(l), ch(l), catc(l) * V(l));
  };
  auto pool = [&](const std::vector<float*>& s, int l) {
    return vw(s, 4 * l + 2, 0, ch(l - 1), ch(l - 1) * V(l));
  };
  auto decA = [&](const std::vector<float*>& s, int l) { return vw(s, 4 * l + 3, 0, ch(l), 2 * ch(l) * V(l)); };
  auto decB = [&](const std::vector<float*>& s, int l) {
    return vw(s, 4 * l + 3, ch(l) * V(l), ch(l), 2 * ch(l) * V(l));
  };
  // every activation gradient accumulates; start from zero
  for (int l = 0; l < levels_; ++l) {
    const int64_t Vl = (int64_t)B * V(l);
    nn_fill(grad_[4 * l], ch(l) * Vl, 0.f, st_);
    nn_fill(grad_[4 * l + 1], catc(l) * Vl, 0.f, st_);
    if (l >= 1) nn_fill(grad_[4 * l + 2], ch(l - 1) * Vl, 0.f, st_);
    nn_fill(grad_[4 * l + 3], 2 * ch(l) * Vl, 0.f, st_);
  }
  // conv backward: relu mask on dz (in place), weight/bias grads, data grad
  auto conv_bwd = [&](const Conv& c, const TView& xin, const TView& yout, const TView& dyout,
                      const TView* dxin, int Dl) {
    if (c.relu) nn_relu_backward(yout, dyout, B, (int64_t)Dl * Dl * Dl, st_);
    nn_conv_backward_weight(xin, dyout, g_ + c.woff, g_ + c.boff, work_, B, Dl, Dl, Dl, st_);
    if (dxin) nn_conv_backward_data(dyout, p_ + c.woff, *dxin, B, Dl, Dl, Dl, st_);
  };
  int ci = (int)convs_.size() - 1;
  // output conv
  {
    TView top = levels_ > 1 ? decB(act_, 0) : skip(act_, 0);
    TView gtop = levels_ > 1 ? decB(grad_, 0) : skip(grad_, 0);
    TView dyv{const_cast<float*>(dy), cout_, cout_ * V(0)};
    TView yv{y_out_, cout_, cout_ * V(0)};
    conv_bwd(convs_[ci--], top, yv, dyv, &gtop, D);
  }
  // decoder, from the top level down the U
  for (int l = 0; l <= levels_ - 2; ++l) {
    const int Dl = D >> l;
    const Conv& b = convs_[ci--];
    const Conv& a = convs_[ci--];
    TView gA = decA(grad_, l), gC = cat(grad_, l);
    conv_bwd(b, decA(act_, l), decB(act_, l), decB(grad_, l), &gA, Dl);
    conv_bwd(a, cat(act_, l), decA(act_, l), gA, &gC, Dl);
    TView gsrc = (l + 1 == levels_ - 1) ? skip(grad_, l + 1) : decB(grad_, l + 1);
    nn_up_backward(TView{gC.p, ch(l + 1), gC.bstride}, gsrc, B, Dl, Dl, Dl, st_);
  }
  // encoder, from the bottom up
  for (int l = levels_ - 1; l >= 0; --l) {
    const int Dl = D >> l;
    const Conv& b = convs_[2 * l + 1];
    const Conv& a = convs_[2 * l];
    TView gA = encA(grad_, l);
    conv_bwd(b, encA(act_, l), skip(act_, l), skip(grad_, l), &gA, Dl);
    if (l == 0) {
      TView xin{const_cast<float*>(x_in_), cin_, cin_ * V(0)};
      conv_bwd(a, xin, encA(act_, 0), gA, nullptr, Dl);
    } else {
      TView gP = pool(grad_, l);
      conv_bwd(a, pool(act_, l), encA(act_, l), gA, &gP, Dl);
      nn_pool_backward(gP, skip(grad_, l - 1), B, 2 * Dl, 2 * Dl, 2 * Dl, st_);
    }
  }
  const hipError_t err = hipGetLastError();
  return err == hipSuccess ? "" : std::string("network backward: ") + hipGetErrorString(err);
}

void Net::zero_grad() { nn_fill(g_, nparam_, 0.f, st_); }

void Net::adam(double lr, double b1, double b2, double eps, int step) {
  const double c1 = 1.0 - std::pow(b1, step), c2 = 1.0 - std::pow(b2, step);
  nn_adam(p_, g_, m_, v_, nparam_, (float)lr, (float)b1, (float)b2, (float)eps, (float)c1,
          (float)c2, st_);
}

}  // namespace hmg

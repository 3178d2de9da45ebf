// Design-space steps of the optimization loop.
//
//   * Symmetry (Sec. 6.1): the density is averaged over a group of symmetries
//     of the cube.  Each group element is a signed permutation of the axes:
//     output axis a takes input axis perm[a], mirrored about the centre when
//     its flip bit is set (reflect3: the 8 mirrorings, reflect6: all 48 signed
//     permutations, rotate3: the 24 of determinant +1).
//   * Trigonometric initialization (Sec. 6.2): y_e = sum_m w_m Q_m(x_e) with
//     Q_n the functions cos / sin (2 pi k xb_i), k = 1..n, of the rotated
//     centre coordinates xb = R (x - 1/2) and their pairwise products (a <= b),
//     then rho = rho_min + Vh / (1 + exp(-k (y - mu))) with mu found by
//     bisection so that the mean density is the volume fraction.
//   * Sensitivity filter (Sec. 5.3): g~_e = sum_f w_ef x_f g_f /
//     (max(1e-3, x_e) sum_f w_ef) with the periodic cone weights.
#include <cmath>

#include "hmg_internal.hpp"

namespace hmg {
namespace {

constexpr int DB = 256;

inline int dblocks(int64_t n) {
  int64_t b = (n + DB - 1) / DB;
  if (b > 4096) b = 4096;
  return (int)(b < 1 ? 1 : b);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

template <int NW>
__device__ __forceinline__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NW; ++i) s += lds[i];
  return s;
}

// ---------------------------------------------------------------- symmetry
// ops[t] = perm[0] | perm[1] << 2 | perm[2] << 4 | flips << 6 for group
// element t; the sum runs over t in order.
__global__ void __launch_bounds__(DB) symmetrize_kernel(Grid g, const float* __restrict__ in,
                                                        float* __restrict__ out, SymOps ops) {
  const double inv = 1.0 / (double)ops.count;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int c[3] = {(int)(i % g.nx), (int)((i / g.nx) % g.ny),
                      (int)(i / ((int64_t)g.nx * g.ny))};
    const int dim[3] = {g.nx, g.ny, g.nz};
    double acc = 0.0;
    for (int t = 0; t < ops.count; ++t) {
      const int op = ops.code[t];
      int im[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int v = c[(op >> (2 * a)) & 3];
        im[a] = ((op >> (6 + a)) & 1) ? dim[a] - 1 - v : v;
      }
      acc += (double)in[im[0] + (int64_t)g.nx * (im[1] + (int64_t)g.ny * im[2])];
    }
    out[i] = (float)(acc * inv);
  }
}

// ---------------------------------------------------------------- initialization
__global__ void __launch_bounds__(DB) trig_field_kernel(Grid g, TrigBasis tb,
                                                        const double* __restrict__ w,
                                                        float* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double x0 = ((double)(i % g.nx) + 0.5) / g.nx - 0.5;
    const double x1 = ((double)((i / g.nx) % g.ny) + 0.5) / g.ny - 0.5;
    const double x2 = ((double)(i / ((int64_t)g.nx * g.ny)) + 0.5) / g.nz - 0.5;
    double xb[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) xb[r] = tb.R[3 * r] * x0 + tb.R[3 * r + 1] * x1 + tb.R[3 * r + 2] * x2;
    double T[6 * TRIG_MAX_FREQ];
    const int nt = 6 * tb.nfreq;
    int m = 0;
    for (int a = 0; a < 3; ++a)
      for (int k = 1; k <= tb.nfreq; ++k) {
        double sn, cs;
        sincos(2.0 * M_PI * k * xb[a], &sn, &cs);
        T[m++] = cs;
        T[m++] = sn;
      }
    double acc = 0.0;
    for (int t = 0; t < nt; ++t) acc += w[t] * T[t];
    int idx = nt;
    for (int a = 0; a < nt; ++a)
      for (int b = a; b < nt; ++b) acc += w[idx++] * (T[a] * T[b]);
    y[i] = (float)acc;
  }
}

// state: [0] lo, [1] hi (bracket of mu), [2] done, [3] mu
__device__ __forceinline__ double sigmoid(double y, double mu, double rho_min, double vh,
                                          double k) {
  return rho_min + vh / (1.0 + exp(-k * (y - mu)));
}

__global__ void __launch_bounds__(DB) sig_partial_kernel(Grid g, const float* __restrict__ y,
                                                         double rho_min, double vh, double k,
                                                         const double* __restrict__ state,
                                                         Partials part) {
  __shared__ double red[DB / 64];
  if (state[2] != 0.0) return;
  const double mu = 0.5 * (state[0] + state[1]);
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += sigmoid((double)y[i], mu, rho_min, vh, k);
  const double v = block_sum<DB / 64>(acc, red);
  if (threadIdx.x == 0) part.buf[blockIdx.x] = v;
}

__global__ void __launch_bounds__(256) sig_step_kernel(Partials part, int nblk, int64_t n,
                                                       double volfrac, double* state) {
  __shared__ double red[4];
  if (state[2] != 0.0) return;
  double a = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) a += part.buf[b];
  const double v = block_sum<4>(a, red);
  if (threadIdx.x == 0) {
    const double mid = 0.5 * (state[0] + state[1]);
    if (v / (double)n > volfrac)
      state[0] = mid;
    else
      state[1] = mid;
    if (state[1] - state[0] <= 1e-14 * fmax(1.0, fabs(mid))) state[2] = 1.0;
    state[3] = 0.5 * (state[0] + state[1]);
  }
}

// Bracket [min y - 40/k, max y + 40/k] from per-block extremes.
__global__ void __launch_bounds__(DB) minmax_partial_kernel(Grid g, const float* __restrict__ y,
                                                            Partials part) {
  __shared__ double lo[DB], hi[DB];
  double a = INFINITY, b = -INFINITY;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    a = fmin(a, (double)y[i]);
    b = fmax(b, (double)y[i]);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int s = DB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + s]);
      hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part.buf[blockIdx.x] = lo[0];
    part.buf[part.stride + blockIdx.x] = hi[0];
  }
}

__global__ void sig_init_kernel(Partials part, int nblk, double k, double* state) {
  if (threadIdx.x != 0) return;
  double a = INFINITY, b = -INFINITY;
  for (int i = 0; i < nblk; ++i) {
    a = fmin(a, part.buf[i]);
    b = fmax(b, part.buf[part.stride + i]);
  }
  state[0] = a - 40.0 / k;
  state[1] = b + 40.0 / k;
  state[2] = 0.0;
  state[3] = 0.5 * (state[0] + state[1]);
}

__global__ void __launch_bounds__(DB) sig_apply_kernel(Grid g, float* __restrict__ y,
                                                       double rho_min, double vh, double k,
                                                       const double* __restrict__ state) {
  const double mu = 0.5 * (state[0] + state[1]);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)sigmoid((double)y[i], mu, rho_min, vh, k);
}

// ---------------------------------------------------------------- sensitivity filter
__global__ void __launch_bounds__(DB) sens_filter_kernel(Grid g, const float* __restrict__ x,
                                                         const float* __restrict__ gin,
                                                         float* __restrict__ out,
                                                         const float* __restrict__ w, int h,
                                                         double floor_x) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int gx = (int)(i % g.nx);
    const int gy = (int)((i / g.nx) % g.ny);
    const int gz = (int)(i / ((int64_t)g.nx * g.ny));
    double acc = 0.0;
    int t = 0;
    for (int dz = -h; dz <= h; ++dz) {
      int z = (gz + dz) % g.nz;
      if (z < 0) z += g.nz;
      for (int dy = -h; dy <= h; ++dy) {
        int yy = (gy + dy) % g.ny;
        if (yy < 0) yy += g.ny;
        const int64_t row = (int64_t)g.nx * (yy + (int64_t)g.ny * z);
        for (int dx = -h; dx <= h; ++dx, ++t) {
          const float wt = w[t];
          if (wt == 0.0f) continue;
          int xx = (gx + dx) % g.nx;
          if (xx < 0) xx += g.nx;
          acc += (double)wt * (double)x[row + xx] * (double)gin[row + xx];
        }
      }
    }
    out[i] = (float)(acc / fmax(floor_x, (double)x[i]));
  }
}

}  // namespace

void symmetrize(const Grid& g, const float* in, float* out, const SymOps& ops, hipStream_t st) {
  hipLaunchKernelGGL(symmetrize_kernel, dim3(dblocks(g.n)), dim3(DB), 0, st, g, in, out, ops);
}

void trig_field(const Grid& g, const TrigBasis& tb, const double* w_dev, float* y,
                hipStream_t st) {
  hipLaunchKernelGGL(trig_field_kernel, dim3(dblocks(g.n)), dim3(DB), 0, st, g, tb, w_dev, y);
}

void sigmoid_project(const Grid& g, float* y, double volfrac, double rho_min, double k,
                     double* state, Partials part, int steps, hipStream_t st) {
  const double vh = std::fmin(1.5 * volfrac, 1.0);
  const int nb = dblocks(g.n);
  hipLaunchKernelGGL(minmax_partial_kernel, dim3(nb), dim3(DB), 0, st, g, y, part);
  hipLaunchKernelGGL(sig_init_kernel, dim3(1), dim3(64), 0, st, part, nb, k, state);
  for (int s = 0; s < steps; ++s) {
    hipLaunchKernelGGL(sig_partial_kernel, dim3(nb), dim3(DB), 0, st, g, y, rho_min, vh, k, state,
                       part);
    hipLaunchKernelGGL(sig_step_kernel, dim3(1), dim3(256), 0, st, part, nb, g.n, volfrac, state);
  }
  hipLaunchKernelGGL(sig_apply_kernel, dim3(dblocks(g.n)), dim3(DB), 0, st, g, y, rho_min, vh, k,
                     state);
}

void sensitivity_filter(const Grid& g, const float* x, const float* gin, float* out,
                        const float* w_dev, int h, hipStream_t st) {
  hipLaunchKernelGGL(sens_filter_kernel, dim3(dblocks(g.n)), dim3(DB), 0, st, g, x, gin, out, w_dev,
                     h, 1e-3);
}

}  // namespace hmg

// Homogenized tensor, element sensitivities, density filter and OC update.
//
// C^H (Sec. 3.2, Eq. elasttensor) and its sensitivities (Eq. ch-sens, read per
// element) both need, per element, the 21 energies
//   E_ij = (chi^i - u^i_e)^T K0 (chi^j - u^j_e).
// They are evaluated in the Walsh-Hadamard mode basis: d_hat^i = H chi^i - H u^i_e,
// E_ij = d_hat^i . (Kt d_hat^j) with the 45-entry Kt (mode 0 drops out, which
// is the translation invariance of C^H).  The paper splits K_e into eight
// 3-row blocks handled by eight warps; here one thread owns one element and
// the per-element sums go to FP64 wavefront and block reductions.
#include "hmg_internal.hpp"

namespace hmg {
namespace {

constexpr int PB = 256;
constexpr int PCAP = 4096;

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

inline int blocks_for(int64_t n) {
  int64_t b = (n + PB - 1) / PB;
  if (b > PCAP) b = PCAP;
  return (int)(b < 1 ? 1 : b);
}

// Kt applied to one mode vector (modes 1..7, component k) -- same pattern as
// the level-0 operator, without the element scale.
template <typename T>
__device__ __forceinline__ void kt_apply(const ModeK<T>& K, const T (&d)[8][3], T (&o)[8][3]) {
  const T sn = K.b * (d[1][0] + d[2][1] + d[4][2]);
  o[1][0] = K.ab * d[1][0] + sn;
  o[2][1] = K.ab * d[2][1] + sn;
  o[4][2] = K.ab * d[4][2] + sn;
  T t = K.cs * (d[1][1] + d[2][0]);
  o[1][1] = t;
  o[2][0] = t;
  t = K.cs * (d[1][2] + d[4][0]);
  o[1][2] = t;
  o[4][0] = t;
  t = K.cs * (d[2][2] + d[4][1]);
  o[2][2] = t;
  o[4][1] = t;
  o[3][0] = K.p * d[3][0] + K.q * d[6][2];
  o[6][2] = K.q * d[3][0] + K.p * d[6][2];
  o[3][1] = K.p * d[3][1] + K.q * d[5][2];
  o[5][2] = K.q * d[3][1] + K.p * d[5][2];
  o[5][0] = K.p * d[5][0] + K.q * d[6][1];
  o[6][1] = K.q * d[5][0] + K.p * d[6][1];
  const T st = K.g * (d[3][2] + d[5][1] + d[6][0]);
  o[3][2] = K.fg * d[3][2] + st;
  o[5][1] = K.fg * d[5][1] + st;
  o[6][0] = K.fg * d[6][0] + st;
  o[7][0] = K.z * d[7][0];
  o[7][1] = K.z * d[7][1];
  o[7][2] = K.z * d[7][2];
  o[0][0] = o[0][1] = o[0][2] = T(0);
}

// d_hat^c for the six cases of element i (modes 0..7; mode 0 unused); u is
// stored as U (the arithmetic type T, or FP16 for the cast of Sec. 4.3).
template <typename T, typename U>
__device__ __forceinline__ void element_dhat(const Grid& g, int64_t i, const U* __restrict__ u,
                                             const LoadTpl<T>& chh, T (&dh)[NCASE][8][3]) {
  const int gx = (int)(i % g.nx);
  const int gy = (int)((i / g.nx) % g.ny);
  const int gz = (int)(i / ((int64_t)g.nx * g.ny));
  const int xp = gx + 1 == g.nx ? 0 : gx + 1;
  const int yp = gy + 1 == g.ny ? 0 : gy + 1;
  const int zp = gz + 1 == g.nz ? 0 : gz + 1;
  int64_t node[8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
    node[a] = ((a & 1) ? xp : gx) + (int64_t)g.nx * (((a & 2) ? yp : gy) + (int64_t)g.ny * ((a & 4) ? zp : gz));
#pragma unroll
  for (int c = 0; c < NCASE; ++c)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T v[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) v[a] = (T)u[(int64_t)(c * 3 + k) * g.n + node[a]];
      // 8-point Walsh-Hadamard transform, bit 0 then 1 then 2
#pragma unroll
      for (int h = 1; h < 8; h <<= 1)
#pragma unroll
        for (int a = 0; a < 8; ++a)
          if (!(a & h)) {
            const T x = v[a], y = v[a + h];
            v[a] = x + y;
            v[a + h] = x - y;
          }
#pragma unroll
      for (int m = 0; m < 8; ++m) dh[c][m][k] = chh.g[c][m][k] - v[m];
    }
}

template <typename T>
__device__ __forceinline__ T mode_dot(const T (&a)[8][3], const T (&b)[8][3]) {
  T s = T(0);
#pragma unroll
  for (int m = 1; m < 8; ++m)
#pragma unroll
    for (int k = 0; k < 3; ++k) s += a[m][k] * b[m][k];
  return s;
}

template <typename T, typename U>
__global__ void __launch_bounds__(PB) elastic_kernel(Grid g, ModeK<T> mk, LoadTpl<T> chh,
                                                     const T* __restrict__ s,
                                                     const U* __restrict__ u, Partials part) {
  __shared__ double red[PB / 64];
  double acc[21];
#pragma unroll
  for (int t = 0; t < 21; ++t) acc[t] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    T dh[NCASE][8][3];
    element_dhat(g, i, u, chh, dh);
    const double se = (double)s[i];
    int t = 0;
#pragma unroll
    for (int j = 0; j < NCASE; ++j) {
      T kd[8][3];
      kt_apply(mk, dh[j], kd);
#pragma unroll
      for (int ii = 0; ii <= j; ++ii) acc[t++] += se * (double)mode_dot(dh[ii], kd);
    }
  }
#pragma unroll
  for (int t = 0; t < 21; ++t) {
    const double v = block_sum<PB / 64>(acc[t], red);
    if (threadIdx.x == 0) part.buf[(int64_t)t * part.stride + blockIdx.x] = v;
  }
}

__global__ void __launch_bounds__(256) elastic_fin_kernel(Partials part, int nblk, int64_t n,
                                                          double* out36) {
  __shared__ double red[4];
  const int t = blockIdx.x;
  double a = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) a += part.buf[(int64_t)t * part.stride + b];
  const double v = block_sum<4>(a, red);
  if (threadIdx.x == 0) {
    // t enumerates (i <= j) with j outer: t = j(j+1)/2 + i
    int j = 0;
    while ((j + 1) * (j + 2) / 2 <= t) ++j;
    const int i = t - j * (j + 1) / 2;
    out36[i * 6 + j] = v / (double)n;
    out36[j * 6 + i] = v / (double)n;
  }
}

template <typename T, typename U>
__global__ void __launch_bounds__(PB) sens_kernel(Grid g, ModeK<T> mk, LoadTpl<T> chh,
                                                  const T* __restrict__ rho,
                                                  const U* __restrict__ u,
                                                  const double* __restrict__ w21, double coef,
                                                  double penal, float* __restrict__ out) {
  double w[21];
#pragma unroll
  for (int t = 0; t < 21; ++t) w[t] = w21[t];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    T dh[NCASE][8][3];
    element_dhat(g, i, u, chh, dh);
    double acc = 0.0;
    int t = 0;
#pragma unroll
    for (int j = 0; j < NCASE; ++j) {
      T kd[8][3];
      kt_apply(mk, dh[j], kd);
#pragma unroll
      for (int ii = 0; ii <= j; ++ii) {
        if (w[t] != 0.0) acc += w[t] * (double)mode_dot(dh[ii], kd);
        ++t;
      }
    }
    const double r = (double)rho[i];
    const double dp = (penal == 3.0) ? r * r : (penal == 1.0 ? 1.0 : pow(r, penal - 1.0));
    out[i] = (float)(coef * dp * acc);
  }
}

// ---------------------------------------------------------------- filter
__global__ void __launch_bounds__(PB) filter_kernel(Grid g, const float* __restrict__ in,
                                                    float* __restrict__ out,
                                                    const float* __restrict__ w, int h) {
  const int span = 2 * h + 1;
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
        int y = (gy + dy) % g.ny;
        if (y < 0) y += g.ny;
        const int64_t row = (int64_t)g.nx * (y + (int64_t)g.ny * z);
        for (int dx = -h; dx <= h; ++dx, ++t) {
          const float wt = w[t];
          if (wt == 0.0f) continue;
          int x = (gx + dx) % g.nx;
          if (x < 0) x += g.nx;
          acc += (double)wt * (double)in[row + x];
        }
      }
    }
    (void)span;
    out[i] = (float)acc;
  }
}

// ---------------------------------------------------------------- OC
// state: [0] lo = log lambda lower, [1] hi, [2] done flag, [3] final lambda
__device__ __forceinline__ double oc_x(double x, double g, double lam, double move, double damp,
                                       double xmin) {
  const double B = fmax(0.0, -g) / lam;
  const double c = (damp == 0.5) ? x * sqrt(B) : x * pow(B, damp);
  const double lo = fmax(xmin, x - move), hi = fmin(1.0, x + move);
  return fmin(fmax(c, lo), hi);
}

__global__ void __launch_bounds__(PB) oc_partial_kernel(Grid g, const float* __restrict__ x,
                                                        const float* __restrict__ dfdx, double move,
                                                        double damp, double xmin,
                                                        const double* __restrict__ state,
                                                        Partials part) {
  __shared__ double red[PB / 64];
  if (state[2] != 0.0) return;
  const double lam = exp(0.5 * (state[0] + state[1]));
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += oc_x(x[i], dfdx[i], lam, move, damp, xmin);
  const double v = block_sum<PB / 64>(acc, red);
  if (threadIdx.x == 0) part.buf[blockIdx.x] = v;
}

__global__ void __launch_bounds__(256) oc_step_kernel(Partials part, int nblk, int64_t n,
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
    // Once the next midpoint rounds to an end of the bracket, every further
    // step leaves lambda = exp(next) (the bracket stays or collapses onto that
    // end), so the search stops there with the same lambda; for |log lambda|
    // above ~8 the width test alone never fires (adjacent doubles are wider).
    const double next = 0.5 * (state[0] + state[1]);
    if (state[1] - state[0] < 1e-15 || next == state[0] || next == state[1]) state[2] = 1.0;
    state[3] = exp(0.5 * (state[0] + state[1]));
  }
}

__global__ void oc_init_kernel(double* state) {
  if (threadIdx.x == 0) {
    state[0] = log(1e-40);
    state[1] = log(1e40);
    state[2] = 0.0;
    state[3] = exp(0.5 * (state[0] + state[1]));
  }
}

__global__ void __launch_bounds__(PB) oc_apply_kernel(Grid g, float* __restrict__ x,
                                                      const float* __restrict__ dfdx, double move,
                                                      double damp, double xmin,
                                                      const double* __restrict__ state) {
  const double lam = exp(0.5 * (state[0] + state[1]));
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = (float)oc_x(x[i], dfdx[i], lam, move, damp, xmin);
}

}  // namespace

template <typename T, typename U>
void elastic_partials(const Grid& g, const ModeK<T>& mk, const LoadTpl<T>& chihat, const T* s,
                      const U* u, Partials part, int* nblk_out, hipStream_t st) {
  const int nb = blocks_for(g.n);
  hipLaunchKernelGGL((elastic_kernel<T, U>), dim3(nb), dim3(PB), 0, st, g, mk, chihat, s, u, part);
  *nblk_out = nb;
}
void elastic_finalize(const Partials& part, int nblk, int64_t n, double* out36, hipStream_t st) {
  hipLaunchKernelGGL(elastic_fin_kernel, dim3(21), dim3(256), 0, st, part, nblk, n, out36);
}
template <typename T, typename U>
void sensitivity(const Grid& g, const ModeK<T>& mk, const LoadTpl<T>& chihat, const T* rho,
                 const U* u, const double* w21_dev, double coef, double penal, float* out,
                 hipStream_t st) {
  hipLaunchKernelGGL((sens_kernel<T, U>), dim3(blocks_for(g.n)), dim3(PB), 0, st, g, mk, chihat, rho, u,
                     w21_dev, coef, penal, out);
}
void density_filter(const Grid& g, const float* in, float* out, const float* w_dev, int h,
                    hipStream_t st) {
  hipLaunchKernelGGL(filter_kernel, dim3(blocks_for(g.n)), dim3(PB), 0, st, g, in, out, w_dev, h);
}
void oc_partial(const Grid& g, const float* x, const float* dfdx, double move, double damp,
                double xmin, const double* state, Partials part, int* nblk_out, hipStream_t st) {
  const int nb = blocks_for(g.n);
  hipLaunchKernelGGL(oc_partial_kernel, dim3(nb), dim3(PB), 0, st, g, x, dfdx, move, damp, xmin,
                     state, part);
  *nblk_out = nb;
}
void oc_step(const Partials& part, int nblk, int64_t n, double volfrac, double* state,
             hipStream_t st) {
  hipLaunchKernelGGL(oc_step_kernel, dim3(1), dim3(256), 0, st, part, nblk, n, volfrac, state);
}
void oc_apply(const Grid& g, float* x, const float* dfdx, double move, double damp, double xmin,
              const double* state, hipStream_t st) {
  hipLaunchKernelGGL(oc_apply_kernel, dim3(blocks_for(g.n)), dim3(PB), 0, st, g, x, dfdx, move,
                     damp, xmin, state);
}
void oc_init(double* state, hipStream_t st) {
  hipLaunchKernelGGL(oc_init_kernel, dim3(1), dim3(64), 0, st, state);
}

#define HMG_INST(T, U)                                                                          \
  template void elastic_partials<T, U>(const Grid&, const ModeK<T>&, const LoadTpl<T>&, const T*, \
                                       const U*, Partials, int*, hipStream_t);                    \
  template void sensitivity<T, U>(const Grid&, const ModeK<T>&, const LoadTpl<T>&, const T*,      \
                                  const U*, const double*, double, double, float*, hipStream_t);
HMG_INST(float, float)
HMG_INST(double, double)
HMG_INST(float, f16)
#undef HMG_INST

}  // namespace hmg

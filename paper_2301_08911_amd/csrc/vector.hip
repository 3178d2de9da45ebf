// Pointwise PCG kernels on the fine grid and the small finalizer kernels that
// turn deterministic per-block partial sums into the FP64 scalars of the six
// CG recurrences (dot products, step lengths, convergence state).
#include <type_traits>

#include "hmg_internal.hpp"

namespace hmg {
namespace {

constexpr int VB = 256;       // threads per block of the pointwise kernels
constexpr int VCAP = 4096;    // cap on their grid (grid-stride loops)

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

template <typename T>
__device__ __forceinline__ double to_d(T v) {
  return (double)(typename Acc<T>::type)v;
}

__device__ __forceinline__ bool case_on(const double* scal, int c) {
  return scal == nullptr || scal[S_ACTIVE * 8 + c] != 0.0;
}

// Sums NV per-thread values over the block in a fixed order; out[j] valid in
// thread 0 only.
template <int NV>
__device__ __forceinline__ void block_sum_multi(double (&v)[NV], double* lds /* [VB/64][NV] */) {
#pragma unroll
  for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < NV; ++j) lds[w * NV + j] = v[j];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      double s = 0.0;
      for (int i = 0; i < VB / 64; ++i) s += lds[i * NV + j];
      v[j] = s;
    }
}

// r -= alpha q for load case c, with partials of ||r||^2 and of sum r per
// component.  The single-cell solver advances the iterate every fourth
// iteration: the four direction buffers of the matvec still hold p_{k-3} ..
// p_k, so XMODE 4 adds alpha_{k-3} p_{k-3} + .. + alpha_k p_k and XMODE 0
// leaves x alone (44 and 12 bytes per DOF instead of 32 and 32); XMODE 1 and
// 3 fold two and three directions, XMODE 2 is the plain x += alpha_k p_k of
// the batched solver.  pend[j] is the (j+1)-th newest pending direction, with
// its alpha in slot S_XALPHA + j.  One load case per block row: a thread
// streams the three components of one case, which keeps its registers (and the
// number of concurrent streams per wave) small.
template <typename T>
struct Pending {
  const T* d[3];
};
template <typename T, int XMODE>
__device__ __forceinline__ void update_case(const Grid& g, double* __restrict__ x,
                                            const Pending<T> pend, const T* __restrict__ p,
                                            T* __restrict__ r, const T* __restrict__ q,
                                            const double* scal, const Partials& part, int c) {
  __shared__ double red[(VB / 64) * 4];
  if (!case_on(scal, c)) {
    if (threadIdx.x == 0) {
      part.buf[(S_RR * 8 + c) * part.stride + blockIdx.x] = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        part.buf[((S_MEAN0 + k) * 8 + c) * part.stride + blockIdx.x] = 0.0;
    }
    return;
  }
  const double al64 = scal[S_ALPHA * 8 + c];
  constexpr int NP = XMODE == 1 ? 1 : (XMODE == 3 ? 2 : (XMODE == 4 ? 3 : 0));  // pending folded
  double xa[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < NP; ++j) xa[j] = scal[(S_XALPHA + j) * 8 + c];
  const T al = (T)al64;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // ||r||^2, sum r per component
  const int64_t n = g.n;
  const int64_t base = (int64_t)c * 3 * n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int64_t o = base + (int64_t)k * n + i;
      if constexpr (NP > 0) {
        // oldest direction first
        double dx = xa[NP - 1] * (double)pend.d[NP - 1][o];
#pragma unroll
        for (int j = NP - 2; j >= 0; --j) dx += xa[j] * (double)pend.d[j][o];
        x[o] += dx + al64 * (double)p[o];
      }
      if (XMODE == 2) x[o] += al64 * (double)p[o];
      const T rv = r[o] - al * q[o];
      r[o] = rv;
      acc[0] += (double)rv * (double)rv;
      acc[1 + k] += (double)rv;
    }
  }
  block_sum_multi<4>(acc, red);
  if (threadIdx.x == 0) {
    part.buf[(S_RR * 8 + c) * part.stride + blockIdx.x] = acc[0];
#pragma unroll
    for (int k = 0; k < 3; ++k)
      part.buf[((S_MEAN0 + k) * 8 + c) * part.stride + blockIdx.x] = acc[1 + k];
  }
}

template <typename T, int XMODE>
__global__ void __launch_bounds__(VB) update2_kernel(Grid g, double* __restrict__ x,
                                                     const Pending<T> pend,
                                                     const T* __restrict__ p, T* __restrict__ r,
                                                     const T* __restrict__ q, const double* scal,
                                                     Partials part) {
  update_case<T, XMODE>(g, x, pend, p, r, q, scal, part, blockIdx.y);
}

// x += sum_j S_XALPHA+j pend[j] over the NP directions still owed to the
// iterate, for the active cases (one case per blockIdx.y).
template <typename T, int NP>
__global__ void __launch_bounds__(VB) flush_x_kernel(Grid g, double* __restrict__ x,
                                                     const Pending<T> pend, const double* scal) {
  const int c = blockIdx.y;
  if (!case_on(scal, c)) return;
  double xa[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) xa[j] = scal[(S_XALPHA + j) * 8 + c];
  const int64_t n = g.n;
  const int64_t base = (int64_t)c * 3 * n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int64_t o = base + (int64_t)k * n + i;
      double dx = xa[NP - 1] * (double)pend.d[NP - 1][o];
#pragma unroll
      for (int j = NP - 2; j >= 0; --j) dx += xa[j] * (double)pend.d[j][o];
      x[o] += dx;
    }
}

__global__ void __launch_bounds__(VB) update_batched_kernel(const PwBatchCell* __restrict__ cells) {
  // blockIdx.y = cell * NCASE + load case; x += alpha p every iteration
  const PwBatchCell& ce = cells[blockIdx.y / NCASE];
  update_case<float, 2>(ce.g, ce.x, Pending<float>{}, ce.p, ce.r, ce.q, ce.scal, ce.part,
                        blockIdx.y % NCASE);
}

// z = Dinv (r - m), m the per-component mean in `mean` (slots S_MEAN*, may be NULL).
template <typename R, typename D, typename Z>
__device__ __forceinline__ void jacobi0_body(const Grid& g, const R* __restrict__ r,
                                             const D* __restrict__ dinv, Z* __restrict__ z,
                                             const double* scal, const double* mean) {
  using A = typename Acc<Z>::type;
  bool on[NCASE];
#pragma unroll
  for (int c = 0; c < NCASE; ++c) on[c] = case_on(scal, c);
  const int64_t n = g.n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const A dxx = (A)dinv[i], dyy = (A)dinv[n + i], dzz = (A)dinv[2 * n + i];
    const A dxy = (A)dinv[3 * n + i], dyz = (A)dinv[4 * n + i], dxz = (A)dinv[5 * n + i];
#pragma unroll
    for (int c = 0; c < NCASE; ++c) {
      if (!on[c]) continue;
      double m0 = 0.0, m1 = 0.0, m2 = 0.0;
      if (mean) {
        m0 = mean[S_MEAN0 * 8 + c];
        m1 = mean[S_MEAN1 * 8 + c];
        m2 = mean[S_MEAN2 * 8 + c];
      }
      const A r0 = (A)(to_d(r[(int64_t)(c * 3 + 0) * n + i]) - m0);
      const A r1 = (A)(to_d(r[(int64_t)(c * 3 + 1) * n + i]) - m1);
      const A r2 = (A)(to_d(r[(int64_t)(c * 3 + 2) * n + i]) - m2);
      z[(int64_t)(c * 3 + 0) * n + i] = (Z)(dxx * r0 + dxy * r1 + dxz * r2);
      z[(int64_t)(c * 3 + 1) * n + i] = (Z)(dxy * r0 + dyy * r1 + dyz * r2);
      z[(int64_t)(c * 3 + 2) * n + i] = (Z)(dxz * r0 + dyz * r1 + dzz * r2);
    }
  }
}

template <typename R, typename D, typename Z>
__global__ void __launch_bounds__(VB) jacobi0_kernel(Grid g, const R* __restrict__ r,
                                                     const D* __restrict__ dinv, Z* __restrict__ z,
                                                     const double* scal, const double* mean) {
  jacobi0_body<R, D, Z>(g, r, dinv, z, scal, mean);
}

template <typename T>
__global__ void fill_kernel(T* __restrict__ a, int64_t count, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

template <typename T>
__global__ void scale_kernel(T* __restrict__ a, int64_t count, double f) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = (T)(to_d(a[i]) * f);
}

template <typename T>
__global__ void add_to_kernel(double* __restrict__ x, const T* __restrict__ z, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] += to_d(z[i]);
}

template <typename T>
__global__ void box_mean_kernel(Grid gf, const T* __restrict__ in, int f, float* __restrict__ out) {
  const int nx = gf.nx / f, ny = gf.ny / f, nz = gf.nz / f;
  const int64_t nc = (int64_t)nx * ny * nz;
  const double inv = 1.0 / ((double)f * f * f);
  for (int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; I < nc;
       I += (int64_t)gridDim.x * blockDim.x) {
    const int X = (int)(I % nx), Y = (int)((I / nx) % ny), Z = (int)(I / ((int64_t)nx * ny));
    double s = 0.0;
    for (int c = 0; c < f; ++c)
      for (int b = 0; b < f; ++b)
        for (int a = 0; a < f; ++a)
          s += to_d(in[(int64_t)(Z * f + c) * gf.nx * gf.ny + (int64_t)(Y * f + b) * gf.nx + X * f + a]);
    out[I] = (float)(s * inv);
  }
}

template <typename T>
__global__ void pattern_kernel(T* __restrict__ a, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t h = (uint32_t)i * 2654435761u;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    a[i] = (T)(typename Acc<T>::type)((double)(h >> 8) * (1.0 / 8388608.0) - 1.0);
  }
}

template <typename S, typename D>
__global__ void convert_kernel(D* __restrict__ d, const S* __restrict__ s, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    if constexpr (std::is_same<D, f16>::value)
      d[i] = (D)to_d(s[i]);  // one rounding, straight from double
    else
      d[i] = (D)(typename Acc<D>::type)to_d(s[i]);
  }
}

template <typename T>
__global__ void copy_kernel(T* __restrict__ d, const T* __restrict__ s, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

template <typename TA, typename TB>
__global__ void __launch_bounds__(VB) dot_kernel(Grid g, const TA* __restrict__ a,
                                                 const TB* __restrict__ b, const double* scal,
                                                 Partials part, int slot) {
  __shared__ double red[VB / 64];
  double acc[NCASE];
#pragma unroll
  for (int c = 0; c < NCASE; ++c) acc[c] = 0.0;
  const int64_t n = g.n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
#pragma unroll
    for (int c = 0; c < NCASE; ++c) {
      if (!case_on(scal, c)) continue;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int64_t o = (int64_t)(c * 3 + k) * n + i;
        acc[c] += to_d(a[o]) * to_d(b[o]);
      }
    }
#pragma unroll
  for (int c = 0; c < NCASE; ++c) {
    const double t = block_sum<VB / 64>(acc[c], red);
    if (threadIdx.x == 0) part.buf[(slot * 8 + c) * part.stride + blockIdx.x] = t;
  }
}

template <typename T>
__global__ void __launch_bounds__(VB) mean_partial_kernel(Grid g, const T* __restrict__ a,
                                                          Partials part) {
  __shared__ double red[VB / 64];
  const int64_t n = g.n;
  for (int ck = 0; ck < NCASE * 3; ++ck) {
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
      acc += to_d(a[(int64_t)ck * n + i]);
    const double t = block_sum<VB / 64>(acc, red);
    const int c = ck / 3, k = ck % 3;
    if (threadIdx.x == 0) part.buf[((S_MEAN0 + k) * 8 + c) * part.stride + blockIdx.x] = t;
  }
}

template <typename T>
__global__ void mean_subtract_kernel(Grid g, T* __restrict__ a, const double* scal) {
  const int64_t n = g.n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
#pragma unroll
    for (int c = 0; c < NCASE; ++c)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int64_t o = (int64_t)(c * 3 + k) * n + i;
        a[o] = a[o] - (T)scal[(S_MEAN0 + k) * 8 + c];
      }
}

// ---------------------------------------------------------------- finalizers
// One block per case; fixed summation order, so results are reproducible.
__global__ void __launch_bounds__(256) fin_sum_kernel(Partials part, int slot, int nblk,
                                                      double* scal, int all) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  if (!all && scal[S_ACTIVE * 8 + c] == 0.0) return;
  double a = 0.0;
  const double* src = part.buf + (int64_t)(slot * 8 + c) * part.stride;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) a += src[i];
  const double t = block_sum<4>(a, red);
  if (threadIdx.x == 0) scal[slot * 8 + c] = t;
}

__global__ void fin_init_kernel(double* scal, double eps_abs, double tol) {
  const int c = threadIdx.x;
  if (c >= NCASE) return;
  const double fn = sqrt(scal[S_FF * 8 + c]);
  const double rn = sqrt(scal[S_RR * 8 + c]);
  const bool trivial = fn <= eps_abs;
  const double th = fmax(tol * fn, eps_abs);
  scal[S_TRIVIAL * 8 + c] = trivial ? 1.0 : 0.0;
  scal[S_THRESH * 8 + c] = th;
  scal[S_ACTIVE * 8 + c] = (!trivial && rn > th) ? 1.0 : 0.0;
  scal[S_ALPHA * 8 + c] = 0.0;
  scal[S_BETA * 8 + c] = 0.0;
  scal[S_RZ * 8 + c] = 0.0;
}

__global__ void fin_alpha_kernel(double* scal) {
  const int c = threadIdx.x;
  if (c >= NCASE) return;
  const double pq = scal[S_PQ * 8 + c];
  const bool on = scal[S_ACTIVE * 8 + c] != 0.0 && pq != 0.0;
  const double a = on ? scal[S_RZ * 8 + c] / pq : 0.0;
  scal[S_ALPHA * 8 + c] = a;
}

__global__ void fin_beta_kernel(double* scal, int pr) {
  const int c = threadIdx.x;
  if (c >= NCASE) return;
  if (scal[S_ACTIVE * 8 + c] == 0.0) return;
  const double rz = scal[S_RZ * 8 + c], rzn = scal[S_RZNEW * 8 + c];
  const bool restart = scal[S_RESTART * 8 + c] != 0.0;
  double beta = 0.0;
  if (rz != 0.0 && !restart) {
    if (pr && scal[S_REPLACED * 8 + c] == 0.0) {
      // (r_new - r_old).z_new = -alpha q.z_new; negative values restart
      beta = -scal[S_ALPHA * 8 + c] * scal[S_QZ * 8 + c] / rz;
      if (beta < 0.0) beta = 0.0;
    } else {
      beta = rzn / rz;
    }
  }
  scal[S_BETA * 8 + c] = beta;
  scal[S_RZ * 8 + c] = rzn;
  scal[S_RESTART * 8 + c] = 0.0;
  scal[S_REPLACED * 8 + c] = 0.0;
}

__global__ void fin_mean_kernel(Partials part, int nblk, int64_t n, double* scal) {
  __shared__ double red[4];
  const int c = blockIdx.x % NCASE, k = blockIdx.x / NCASE;
  double a = 0.0;
  const double* src = part.buf + (int64_t)((S_MEAN0 + k) * 8 + c) * part.stride;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) a += src[i];
  const double t = block_sum<4>(a, red);
  if (threadIdx.x == 0) scal[(S_MEAN0 + k) * 8 + c] = t / (double)n;
}

__global__ void all_active_kernel(double* scal) {
  const int c = threadIdx.x;
  if (c < 8) {
    scal[S_ACTIVE * 8 + c] = 1.0;
    scal[S_BETA * 8 + c] = 0.0;
    scal[S_ALPHA * 8 + c] = 0.0;
    scal[S_RESTART * 8 + c] = 0.0;
    scal[S_REPLACED * 8 + c] = 0.0;
  }
}

template <typename T>
__global__ void __launch_bounds__(VB) sum_kernel(const T* __restrict__ a, int64_t n, Partials part) {
  __shared__ double red[VB / 64];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += (double)a[i];
  const double t = block_sum<VB / 64>(acc, red);
  if (threadIdx.x == 0) part.buf[blockIdx.x] = t;
}

__global__ void __launch_bounds__(256) sum_fin_kernel(Partials part, int nblk, double* out) {
  __shared__ double red[4];
  double a = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) a += part.buf[i];
  const double t = block_sum<4>(a, red);
  if (threadIdx.x == 0) out[0] = t;
}

inline int blocks_for(int64_t n) {
  int64_t b = (n + VB - 1) / VB;
  if (b > VCAP) b = VCAP;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

int vec_blocks(const Grid& g) { return blocks_for(g.n); }

void update_batched(const PwBatchCell* cells_dev, int ncells, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(update_batched_kernel, dim3(nblk, ncells * NCASE), dim3(VB), 0, st, cells_dev);
}
int vec_blocks_for(int64_t n) { return blocks_for(n); }

template <typename S, typename D>
void vec_convert(D* dst, const S* src, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL((convert_kernel<S, D>), dim3(blocks_for(count)), dim3(VB), 0, st, dst, src,
                     count);
}
template void vec_convert<float, double>(double*, const float*, int64_t, hipStream_t);
template void vec_convert<double, float>(float*, const double*, int64_t, hipStream_t);
template void vec_convert<double, double>(double*, const double*, int64_t, hipStream_t);
template void vec_convert<float, float>(float*, const float*, int64_t, hipStream_t);
template void vec_convert<float, bf16>(bf16*, const float*, int64_t, hipStream_t);
template void vec_convert<bf16, float>(float*, const bf16*, int64_t, hipStream_t);
template void vec_convert<bf16, double>(double*, const bf16*, int64_t, hipStream_t);
template void vec_convert<double, f16>(f16*, const double*, int64_t, hipStream_t);

template <typename T>
void vec_update_r4(const Grid& g, double* x, const T* const* pend, int npend, const T* p, T* r,
                   const T* q, const double* scal, Partials part, int* nblk_out, hipStream_t st) {
  const int nb = blocks_for(g.n);
  Pending<T> pd{};
  for (int j = 0; j < npend; ++j) pd.d[j] = pend[j];
  switch (npend) {
    case 0:
      hipLaunchKernelGGL((update2_kernel<T, 0>), dim3(nb, NCASE), dim3(VB), 0, st, g, x, pd, p, r,
                         q, scal, part);
      break;
    case 1:
      hipLaunchKernelGGL((update2_kernel<T, 1>), dim3(nb, NCASE), dim3(VB), 0, st, g, x, pd, p, r,
                         q, scal, part);
      break;
    case 2:
      hipLaunchKernelGGL((update2_kernel<T, 3>), dim3(nb, NCASE), dim3(VB), 0, st, g, x, pd, p, r,
                         q, scal, part);
      break;
    default:
      hipLaunchKernelGGL((update2_kernel<T, 4>), dim3(nb, NCASE), dim3(VB), 0, st, g, x, pd, p, r,
                         q, scal, part);
  }
  *nblk_out = nb;
}
template <typename T>
void vec_flush_x(const Grid& g, double* x, const T* const* pend, int npend, const double* scal,
                 hipStream_t st) {
  Pending<T> pd{};
  for (int j = 0; j < npend; ++j) pd.d[j] = pend[j];
  const dim3 grid(blocks_for(g.n), NCASE);
  if (npend == 1)
    hipLaunchKernelGGL((flush_x_kernel<T, 1>), grid, dim3(VB), 0, st, g, x, pd, scal);
  else if (npend == 2)
    hipLaunchKernelGGL((flush_x_kernel<T, 2>), grid, dim3(VB), 0, st, g, x, pd, scal);
  else if (npend == 3)
    hipLaunchKernelGGL((flush_x_kernel<T, 3>), grid, dim3(VB), 0, st, g, x, pd, scal);
}
template void vec_update_r4<float>(const Grid&, double*, const float* const*, int, const float*,
                                   float*, const float*, const double*, Partials, int*,
                                   hipStream_t);
template void vec_update_r4<double>(const Grid&, double*, const double* const*, int,
                                    const double*, double*, const double*, const double*, Partials,
                                    int*, hipStream_t);
template void vec_flush_x<float>(const Grid&, double*, const float* const*, int, const double*,
                                 hipStream_t);
template void vec_flush_x<double>(const Grid&, double*, const double* const*, int, const double*,
                                  hipStream_t);

template <typename R, typename D, typename Z>
void vec_jacobi0(const Grid& g, const R* r, const D* dinv, Z* z, const double* scal,
                 const double* mean, hipStream_t st) {
  hipLaunchKernelGGL((jacobi0_kernel<R, D, Z>), dim3(blocks_for(g.n)), dim3(VB), 0, st, g, r,
                     dinv, z, scal, mean);
}
template void vec_jacobi0<float, float, float>(const Grid&, const float*, const float*, float*,
                                               const double*, const double*, hipStream_t);
template void vec_jacobi0<double, double, double>(const Grid&, const double*, const double*,
                                                  double*, const double*, const double*,
                                                  hipStream_t);
template void vec_jacobi0<float, float, bf16>(const Grid&, const float*, const float*, bf16*,
                                              const double*, const double*, hipStream_t);
template void vec_jacobi0<bf16, bf16, bf16>(const Grid&, const bf16*, const bf16*, bf16*,
                                            const double*, const double*, hipStream_t);
template void vec_jacobi0<bf16, float, bf16>(const Grid&, const bf16*, const float*, bf16*,
                                             const double*, const double*, hipStream_t);

template <typename T>
void vec_fill(T* a, int64_t count, T v, hipStream_t st) {
  hipLaunchKernelGGL(fill_kernel<T>, dim3(blocks_for(count)), dim3(VB), 0, st, a, count, v);
}
template <typename T>
void vec_scale(T* a, int64_t count, double factor, hipStream_t st) {
  hipLaunchKernelGGL(scale_kernel<T>, dim3(blocks_for(count)), dim3(VB), 0, st, a, count, factor);
}
template <typename T>
void vec_add_to(double* x, const T* z, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(add_to_kernel<T>, dim3(blocks_for(count)), dim3(VB), 0, st, x, z, count);
}
template <typename T>
void vec_box_mean(const Grid& gf, const T* in, int f, float* out, hipStream_t st) {
  hipLaunchKernelGGL(box_mean_kernel<T>, dim3(blocks_for(gf.n / ((int64_t)f * f * f))), dim3(VB), 0,
                     st, gf, in, f, out);
}
template <typename T>
void vec_pattern(T* a, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(pattern_kernel<T>, dim3(blocks_for(count)), dim3(VB), 0, st, a, count);
}
template <typename T>
void vec_copy(T* d, const T* s, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(copy_kernel<T>, dim3(blocks_for(count)), dim3(VB), 0, st, d, s, count);
}
template <typename TA, typename TB>
void vec_dot_cases(const Grid& g, const TA* a, const TB* b, const double* scal, Partials part,
                   int slot, int* nblk_out, hipStream_t st) {
  const int nb = blocks_for(g.n);
  hipLaunchKernelGGL((dot_kernel<TA, TB>), dim3(nb), dim3(VB), 0, st, g, a, b, scal, part, slot);
  *nblk_out = nb;
}
template void vec_dot_cases<double, float>(const Grid&, const double*, const float*,
                                           const double*, Partials, int, int*, hipStream_t);
template void vec_dot_cases<float, bf16>(const Grid&, const float*, const bf16*, const double*,
                                         Partials, int, int*, hipStream_t);
template <typename T>
void vec_mean_partial(const Grid& g, const T* a, Partials part, int* nblk_out, hipStream_t st) {
  const int nb = blocks_for(g.n);
  hipLaunchKernelGGL(mean_partial_kernel<T>, dim3(nb), dim3(VB), 0, st, g, a, part);
  *nblk_out = nb;
}
template <typename T>
void vec_mean_subtract(const Grid& g, T* a, const double* scal, hipStream_t st) {
  hipLaunchKernelGGL(mean_subtract_kernel<T>, dim3(blocks_for(g.n)), dim3(VB), 0, st, g, a, scal);
}

template <typename T>
void vec_sum_scalar(const T* a, int64_t n, double* out_dev, Partials part, hipStream_t st) {
  const int nb = blocks_for(n);
  hipLaunchKernelGGL(sum_kernel<T>, dim3(nb), dim3(VB), 0, st, a, n, part);
  hipLaunchKernelGGL(sum_fin_kernel, dim3(1), dim3(256), 0, st, part, nb, out_dev);
}

void fin_sum(const Partials& part, int slot, int nblk, double* scal, bool all_cases,
             hipStream_t st) {
  hipLaunchKernelGGL(fin_sum_kernel, dim3(NCASE), dim3(256), 0, st, part, slot, nblk, scal,
                     all_cases ? 1 : 0);
}
void fin_init(double* scal, double eps_abs, double tol, hipStream_t st) {
  hipLaunchKernelGGL(fin_init_kernel, dim3(1), dim3(64), 0, st, scal, eps_abs, tol);
}
void fin_alpha(double* scal, hipStream_t st) {
  hipLaunchKernelGGL(fin_alpha_kernel, dim3(1), dim3(64), 0, st, scal);
}
void fin_beta(double* scal, bool polak_ribiere, hipStream_t st) {
  hipLaunchKernelGGL(fin_beta_kernel, dim3(1), dim3(64), 0, st, scal, polak_ribiere ? 1 : 0);
}
void fin_mean(const Partials& part, int nblk, int64_t n, double* scal, hipStream_t st) {
  hipLaunchKernelGGL(fin_mean_kernel, dim3(NCASE * 3), dim3(256), 0, st, part, nblk, n, scal);
}
void scal_set_all_active(double* scal, hipStream_t st) {
  hipLaunchKernelGGL(all_active_kernel, dim3(1), dim3(64), 0, st, scal);
}

#define HMG_INST(T)                                                                             \
  template void vec_fill<T>(T*, int64_t, T, hipStream_t);                                       \
  template void vec_scale<T>(T*, int64_t, double, hipStream_t);                                 \
  template void vec_add_to<T>(double*, const T*, int64_t, hipStream_t);                         \
  template void vec_box_mean<T>(const Grid&, const T*, int, float*, hipStream_t);               \
  template void vec_pattern<T>(T*, int64_t, hipStream_t);                                       \
  template void vec_copy<T>(T*, const T*, int64_t, hipStream_t);                                \
  template void vec_dot_cases<T, T>(const Grid&, const T*, const T*, const double*, Partials, int,\
                                 int*, hipStream_t);                                            \
  template void vec_mean_partial<T>(const Grid&, const T*, Partials, int*, hipStream_t);        \
  template void vec_mean_subtract<T>(const Grid&, T*, const double*, hipStream_t);        \
  template void vec_sum_scalar<T>(const T*, int64_t, double*, Partials, hipStream_t);
HMG_INST(float)
HMG_INST(double)
HMG_INST(bf16)
#undef HMG_INST

}  // namespace hmg

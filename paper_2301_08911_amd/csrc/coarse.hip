// Coarse multigrid levels: stored 27-point 3x3 stencils, grid transfers,
// Galerkin assembly and the FP64 direct solve on the coarsest grid.
//
// Sec. 3.3: trilinear interpolation I and restriction R = I^T, Galerkin
// K_{l+1} = R K_l I, V-cycle of Alg. 1.  Sec. 4.2: the second level is
// assembled from the densities (Eq. st-level-2, st-assemb-w), deeper levels from
// the stencil of the finer level; the null-space component is removed before
// the coarsest solve.
//
// Stencil layout (coefficient-major, coalesced over vertices):
//   st[((d*3 + p)*3 + q) * n + v],  d = (dx+1) + 3 (dy+1) + 9 (dz+1).
#include "hmg_internal.hpp"

namespace hmg {
namespace {

__host__ __device__ inline int modp(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

inline int pw_blocks(int64_t n, int tpb, int cap) {
  int64_t b = (n + tpb - 1) / tpb;
  if (b > cap) b = cap;
  return (int)(b < 1 ? 1 : b);
}

// Conversions between the storage type and FP64 / the arithmetic type.
template <typename T>
__device__ __forceinline__ double to_d(T v) {
  return (double)(typename Acc<T>::type)v;
}
template <typename T>
__device__ __forceinline__ T from_d(double v) {
  return (T)(typename Acc<T>::type)v;
}

__device__ __forceinline__ bool case_on(const double* scal, int c) {
  return scal == nullptr || scal[S_ACTIVE * 8 + c] != 0.0;
}

// MODE 0: out = K u.  MODE 1: out = (r - m) - K u.  MODE 2: out = u + Dinv ((r - m) - K u).
// m is the per-component mean of r (slots S_MEAN* of `mean`, FP64).
template <typename T, typename W, int MODE>
__global__ void stencil_kernel(Grid g, const W* __restrict__ st, const T* __restrict__ u,
                               const T* __restrict__ r, const W* __restrict__ dinv,
                               T* __restrict__ out, const double* scal, const double* mean) {
  using A = typename Acc<T>::type;
  bool on[NCASE];
#pragma unroll
  for (int c = 0; c < NCASE; ++c) on[c] = case_on(scal, c);
  const int64_t n = g.n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int gx = (int)(i % g.nx);
    const int gy = (int)((i / g.nx) % g.ny);
    const int gz = (int)(i / ((int64_t)g.nx * g.ny));
    int xs[3] = {gx == 0 ? g.nx - 1 : gx - 1, gx, gx + 1 == g.nx ? 0 : gx + 1};
    int ys[3] = {gy == 0 ? g.ny - 1 : gy - 1, gy, gy + 1 == g.ny ? 0 : gy + 1};
    int zs[3] = {gz == 0 ? g.nz - 1 : gz - 1, gz, gz + 1 == g.nz ? 0 : gz + 1};
    A acc[NCASE][3];
#pragma unroll
    for (int c = 0; c < NCASE; ++c) acc[c][0] = acc[c][1] = acc[c][2] = A(0);
    for (int d = 0; d < 27; ++d) {
      const int dx = d % 3, dy = (d / 3) % 3, dz = d / 9;
      const int64_t w = xs[dx] + (int64_t)g.nx * (ys[dy] + (int64_t)g.ny * zs[dz]);
      A K[9];
#pragma unroll
      for (int t = 0; t < 9; ++t) K[t] = (A)st[(int64_t)(d * 9 + t) * n + i];
#pragma unroll
      for (int c = 0; c < NCASE; ++c) {
        if (!on[c]) continue;
        const A u0 = (A)u[(int64_t)(c * 3 + 0) * n + w];
        const A u1 = (A)u[(int64_t)(c * 3 + 1) * n + w];
        const A u2 = (A)u[(int64_t)(c * 3 + 2) * n + w];
        acc[c][0] += K[0] * u0 + K[1] * u1 + K[2] * u2;
        acc[c][1] += K[3] * u0 + K[4] * u1 + K[5] * u2;
        acc[c][2] += K[6] * u0 + K[7] * u1 + K[8] * u2;
      }
    }
    A D[6];
    if (MODE == 2) {
#pragma unroll
      for (int t = 0; t < 6; ++t) D[t] = (A)dinv[(int64_t)t * n + i];
    }
#pragma unroll
    for (int c = 0; c < NCASE; ++c) {
      if (!on[c]) continue;
      if (MODE == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) out[(int64_t)(c * 3 + k) * n + i] = (T)acc[c][k];
      } else {
        A res[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
          res[k] = (A)(to_d(r[(int64_t)(c * 3 + k) * n + i]) - mean[(S_MEAN0 + k) * 8 + c]) -
                   acc[c][k];
        if (MODE == 1) {
#pragma unroll
          for (int k = 0; k < 3; ++k) out[(int64_t)(c * 3 + k) * n + i] = (T)res[k];
        } else {
          const A z0 = (A)u[(int64_t)(c * 3 + 0) * n + i] + (D[0] * res[0] + D[3] * res[1] + D[5] * res[2]);
          const A z1 = (A)u[(int64_t)(c * 3 + 1) * n + i] + (D[3] * res[0] + D[1] * res[1] + D[4] * res[2]);
          const A z2 = (A)u[(int64_t)(c * 3 + 2) * n + i] + (D[5] * res[0] + D[4] * res[1] + D[2] * res[2]);
          out[(int64_t)(c * 3 + 0) * n + i] = (T)z0;
          out[(int64_t)(c * 3 + 1) * n + i] = (T)z1;
          out[(int64_t)(c * 3 + 2) * n + i] = (T)z2;
        }
      }
    }
  }
}

// rc[V] = sum_{a in {-1,0,1}^3} w(a) tf[2V + a], w(a) = prod (a_k == 0 ? 1 : 1/2)
template <typename T>
__global__ void restrict_kernel(Grid gf, Grid gc, const T* __restrict__ tf, T* __restrict__ rc,
                                const double* scal) {
  bool on[NCASE];
#pragma unroll
  for (int c = 0; c < NCASE; ++c) on[c] = case_on(scal, c);
  using A = typename Acc<T>::type;
  for (int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; I < gc.n;
       I += (int64_t)gridDim.x * blockDim.x) {
    const int X = (int)(I % gc.nx);
    const int Y = (int)((I / gc.nx) % gc.ny);
    const int Z = (int)(I / ((int64_t)gc.nx * gc.ny));
    int xs[3] = {modp(2 * X - 1, gf.nx), 2 * X, 2 * X + 1};
    int ys[3] = {modp(2 * Y - 1, gf.ny), 2 * Y, 2 * Y + 1};
    int zs[3] = {modp(2 * Z - 1, gf.nz), 2 * Z, 2 * Z + 1};
    A acc[NCASE][3];
#pragma unroll
    for (int c = 0; c < NCASE; ++c) acc[c][0] = acc[c][1] = acc[c][2] = A(0);
    for (int a = 0; a < 27; ++a) {
      const int ax = a % 3, ay = (a / 3) % 3, az = a / 9;
      const A w = A((ax == 1 ? 1.0 : 0.5) * (ay == 1 ? 1.0 : 0.5) * (az == 1 ? 1.0 : 0.5));
      const int64_t f = xs[ax] + (int64_t)gf.nx * (ys[ay] + (int64_t)gf.ny * zs[az]);
#pragma unroll
      for (int c = 0; c < NCASE; ++c) {
        if (!on[c]) continue;
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[c][k] += w * (A)tf[(int64_t)(c * 3 + k) * gf.n + f];
      }
    }
#pragma unroll
    for (int c = 0; c < NCASE; ++c) {
      if (!on[c]) continue;
#pragma unroll
      for (int k = 0; k < 3; ++k) rc[(int64_t)(c * 3 + k) * gc.n + I] = (T)acc[c][k];
    }
  }
}

// zf[v] (+)= sum over the coarse vertices of v's cell of trilinear weights * ec
template <typename T, typename C>
__global__ void prolong_kernel(Grid gf, Grid gc, T* __restrict__ zf, const C* __restrict__ ec,
                               const double* scal, int overwrite) {
  bool on[NCASE];
#pragma unroll
  for (int c = 0; c < NCASE; ++c) on[c] = case_on(scal, c);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < gf.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int gx = (int)(i % gf.nx);
    const int gy = (int)((i / gf.nx) % gf.ny);
    const int gz = (int)(i / ((int64_t)gf.nx * gf.ny));
    const int X0 = gx >> 1, Y0 = gy >> 1, Z0 = gz >> 1;
    const int X1 = (gx & 1) ? (X0 + 1 == gc.nx ? 0 : X0 + 1) : X0;
    const int Y1 = (gy & 1) ? (Y0 + 1 == gc.ny ? 0 : Y0 + 1) : Y0;
    const int Z1 = (gz & 1) ? (Z0 + 1 == gc.nz ? 0 : Z0 + 1) : Z0;
    using A = typename Acc<T>::type;
    const int nt = 1 << ((gx & 1) + (gy & 1) + (gz & 1));
    const A w = A(1.0) / A(nt);
    int64_t idx[8];
    int m = 0;
    for (int cz = 0; cz < ((gz & 1) ? 2 : 1); ++cz)
      for (int cy = 0; cy < ((gy & 1) ? 2 : 1); ++cy)
        for (int cx = 0; cx < ((gx & 1) ? 2 : 1); ++cx)
          idx[m++] = (cx ? X1 : X0) + (int64_t)gc.nx * ((cy ? Y1 : Y0) + (int64_t)gc.ny * (cz ? Z1 : Z0));
#pragma unroll
    for (int c = 0; c < NCASE; ++c) {
      if (!on[c]) continue;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const C* e = ec + (int64_t)(c * 3 + k) * gc.n;
        A v = A(0);
        for (int t = 0; t < m; ++t) v += (A)e[idx[t]];
        T* o = zf + (int64_t)(c * 3 + k) * gf.n + i;
        *o = (T)(overwrite ? w * v : (A)*o + w * v);
      }
    }
  }
}

// First coarse level from the densities.  Coarse vertex V is local node A of
// the coarse element with origin V - A; that element holds the 8 fine elements
// 2(V - A) + sigma, each contributing s * (W_sigma^T K0 W_sigma)[A, A + D].
template <typename S, typename T>
__global__ void galerkin_first_kernel(Grid gf, Grid gc, const S* __restrict__ s,
                                      const double* __restrict__ msig, T* __restrict__ st) {
  const int d = blockIdx.y;
  const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
  for (int64_t V = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; V < gc.n;
       V += (int64_t)gridDim.x * blockDim.x) {
    const int X = (int)(V % gc.nx);
    const int Y = (int)((V / gc.nx) % gc.ny);
    const int Z = (int)(V / ((int64_t)gc.nx * gc.ny));
    double blk[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int A = 0; A < 8; ++A) {
      const int A0 = A & 1, A1 = (A >> 1) & 1, A2 = A >> 2;
      const int B0 = A0 + dx, B1 = A1 + dy, B2 = A2 + dz;
      if (B0 < 0 || B0 > 1 || B1 < 0 || B1 > 1 || B2 < 0 || B2 > 1) continue;
      const int B = B0 + 2 * B1 + 4 * B2;
      const int CX = modp(X - A0, gc.nx), CY = modp(Y - A1, gc.ny), CZ = modp(Z - A2, gc.nz);
      for (int sg = 0; sg < 8; ++sg) {
        const int64_t e = (2 * CX + (sg & 1)) +
                          (int64_t)gf.nx * ((2 * CY + ((sg >> 1) & 1)) +
                                            (int64_t)gf.ny * (2 * CZ + (sg >> 2)));
        const double se = (double)s[e];
        const double* M = msig + (int64_t)sg * 576;
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
          for (int q = 0; q < 3; ++q) blk[p * 3 + q] += se * M[(3 * A + p) * 24 + 3 * B + q];
      }
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) st[(int64_t)(d * 9 + t) * gc.n + V] = from_d<T>(blk[t]);
  }
}

// K_{l+1}[V, V+D] = sum_a sum_b w(a) w(b) K_l[2V + a, 2V + a + d'], d' = 2D + b - a.
template <typename T>
__global__ void galerkin_next_kernel(Grid gf, Grid gc, const T* __restrict__ stf,
                                     T* __restrict__ stc) {
  const int d = blockIdx.y;
  const int Dx = d % 3 - 1, Dy = (d / 3) % 3 - 1, Dz = d / 9 - 1;
  for (int64_t V = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; V < gc.n;
       V += (int64_t)gridDim.x * blockDim.x) {
    const int X = (int)(V % gc.nx);
    const int Y = (int)((V / gc.nx) % gc.ny);
    const int Z = (int)(V / ((int64_t)gc.nx * gc.ny));
    double blk[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < 27; ++a) {
      const int ax = a % 3 - 1, ay = (a / 3) % 3 - 1, az = a / 9 - 1;
      const double wa = (ax ? 0.5 : 1.0) * (ay ? 0.5 : 1.0) * (az ? 0.5 : 1.0);
      const int64_t i = modp(2 * X + ax, gf.nx) +
                        (int64_t)gf.nx * (modp(2 * Y + ay, gf.ny) + (int64_t)gf.ny * modp(2 * Z + az, gf.nz));
      for (int b = 0; b < 27; ++b) {
        const int bx = b % 3 - 1, by = (b / 3) % 3 - 1, bz = b / 9 - 1;
        const int px = 2 * Dx + bx - ax, py = 2 * Dy + by - ay, pz = 2 * Dz + bz - az;
        if (px < -1 || px > 1 || py < -1 || py > 1 || pz < -1 || pz > 1) continue;
        const double w = wa * (bx ? 0.5 : 1.0) * (by ? 0.5 : 1.0) * (bz ? 0.5 : 1.0);
        const int dp = (px + 1) + 3 * (py + 1) + 9 * (pz + 1);
#pragma unroll
        for (int t = 0; t < 9; ++t) blk[t] += w * to_d(stf[(int64_t)(dp * 9 + t) * gf.n + i]);
      }
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) stc[(int64_t)(d * 9 + t) * gc.n + V] = from_d<T>(blk[t]);
  }
}

// omega * inverse of the centre block (d = 13), stored as xx, yy, zz, xy, yz, xz.
template <typename T>
__global__ void dinv_stencil_kernel(Grid g, const T* __restrict__ st, double omega,
                                    T* __restrict__ dinv) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double a[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) a[t] = to_d(st[(int64_t)(13 * 9 + t) * g.n + i]);
    const double a00 = a[0], a11 = a[4], a22 = a[8];
    const double a01 = 0.5 * (a[1] + a[3]), a12 = 0.5 * (a[5] + a[7]), a02 = 0.5 * (a[2] + a[6]);
    const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22;
    const double c02 = a01 * a12 - a02 * a11, c11 = a00 * a22 - a02 * a02;
    const double c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
    const double f = omega / (a00 * c00 + a01 * c01 + a02 * c02);
    dinv[i] = from_d<T>(f * c00);
    dinv[g.n + i] = from_d<T>(f * c11);
    dinv[2 * g.n + i] = from_d<T>(f * c22);
    dinv[3 * g.n + i] = from_d<T>(f * c01);
    dinv[4 * g.n + i] = from_d<T>(f * c12);
    dinv[5 * g.n + i] = from_d<T>(f * c02);
  }
}

// Dense coarsest matrix (row per thread), then vertex 0 pinned to the identity.
template <typename T>
__global__ void dense_kernel(Grid g, const T* __restrict__ st, double* __restrict__ A) {
  const int64_t N = 3 * g.n;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < g.n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int gx = (int)(v % g.nx);
    const int gy = (int)((v / g.nx) % g.ny);
    const int gz = (int)(v / ((int64_t)g.nx * g.ny));
    for (int p = 0; p < 3; ++p)
      for (int64_t j = 0; j < N; ++j) A[(3 * v + p) * N + j] = 0.0;
    for (int d = 0; d < 27; ++d) {
      const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
      const int64_t w = modp(gx + dx, g.nx) +
                        (int64_t)g.nx * (modp(gy + dy, g.ny) + (int64_t)g.ny * modp(gz + dz, g.nz));
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q)
          A[(3 * v + p) * N + 3 * w + q] += to_d(st[(int64_t)(d * 9 + p * 3 + q) * g.n + v]);
    }
  }
}

__global__ void pin_kernel(int64_t N, double* __restrict__ A) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N;
       j += (int64_t)gridDim.x * blockDim.x)
    for (int p = 0; p < 3; ++p) {
      const double v = (j == p) ? 1.0 : 0.0;
      A[p * N + j] = v;
      A[j * N + p] = v;
    }
}

// In-place Gauss-Jordan inverse of an SPD matrix (no pivoting), one workgroup.
// colk is a scratch column of length N in global memory.
__global__ void __launch_bounds__(1024) gj_kernel(int N, double* __restrict__ A,
                                                  double* __restrict__ colk) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  for (int k = 0; k < N; ++k) {
    const double piv = 1.0 / A[(int64_t)k * N + k];
    for (int i = tid; i < N; i += nt) colk[i] = A[(int64_t)i * N + k];
    __syncthreads();
    for (int j = tid; j < N; j += nt)
      A[(int64_t)k * N + j] = (j == k) ? piv : A[(int64_t)k * N + j] * piv;
    __syncthreads();
    for (int i = wave; i < N; i += nw) {
      if (i == k) continue;
      const double f = colk[i];
      double* row = A + (int64_t)i * N;
      const double* rk = A + (int64_t)k * N;
      for (int j = lane; j < N; j += 64) row[j] = (j == k) ? -f * piv : row[j] - f * rk[j];
    }
    __syncthreads();
  }
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Fixed-order block sum, result returned to every thread.
__device__ double block_allsum(double v, double* lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += lds[i];
  return s;
}

// One workgroup per case: project the RHS to zero mean per component, apply
// the inverse of the vertex-0-pinned matrix, project the result to zero mean.
template <typename R, typename T>
__global__ void __launch_bounds__(1024) coarse_solve_kernel(Grid g, const double* __restrict__ Ainv,
                                                            const R* __restrict__ r, T* __restrict__ z,
                                                            const double* scal) {
  extern __shared__ double sh[];
  __shared__ double red[16];
  const int c = blockIdx.x;
  if (!case_on(scal, c)) return;
  const int n = (int)g.n, N = 3 * n;
  double* rl = sh;
  double* zl = sh + N;
  double m[3];
  for (int k = 0; k < 3; ++k) {
    double a = 0.0;
    for (int v = threadIdx.x; v < n; v += blockDim.x) {
      const double x = to_d(r[(int64_t)(c * 3 + k) * n + v]);
      rl[3 * v + k] = x;
      a += x;
    }
    m[k] = block_allsum(a, red) / n;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) rl[i] = (i < 3) ? 0.0 : rl[i] - m[i % 3];
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    double a = 0.0;
    for (int j = 0; j < N; ++j) a += Ainv[(int64_t)j * N + i] * rl[j];  // symmetric: column i
    zl[i] = a;
  }
  __syncthreads();
  for (int k = 0; k < 3; ++k) {
    double a = 0.0;
    for (int v = threadIdx.x; v < n; v += blockDim.x) a += zl[3 * v + k];
    m[k] = block_allsum(a, red) / n;
  }
  for (int k = 0; k < 3; ++k)
    for (int v = threadIdx.x; v < n; v += blockDim.x)
      z[(int64_t)(c * 3 + k) * n + v] = from_d<T>(zl[3 * v + k] - m[k]);
}

}  // namespace

template <typename T, typename W>
void kc_apply(const Grid& g, const W* st, const T* u, T* y, hipStream_t s) {
  hipLaunchKernelGGL((stencil_kernel<T, W, 0>), dim3(pw_blocks(g.n, 256, 8192)), dim3(256), 0, s,
                     g, st, u, (const T*)nullptr, (const W*)nullptr, y, (const double*)nullptr,
                     (const double*)nullptr);
}
template <typename T, typename W>
void kc_residual(const Grid& g, const W* st, const T* z, const T* r, T* t, const double* scal,
                 const double* mean, hipStream_t s) {
  hipLaunchKernelGGL((stencil_kernel<T, W, 1>), dim3(pw_blocks(g.n, 256, 8192)), dim3(256), 0, s,
                     g, st, z, r, (const W*)nullptr, t, scal, mean);
}
template <typename T, typename W>
void kc_smooth(const Grid& g, const W* st, const T* z, const T* r, const W* dinv, T* zout,
               const double* scal, const double* mean, hipStream_t s) {
  hipLaunchKernelGGL((stencil_kernel<T, W, 2>), dim3(pw_blocks(g.n, 256, 8192)), dim3(256), 0, s,
                     g, st, z, r, dinv, zout, scal, mean);
}
template <typename T>
void restrict_to(const Grid& gf, const Grid& gc, const T* tf, T* rc, const double* scal,
                 hipStream_t s) {
  hipLaunchKernelGGL(restrict_kernel<T>, dim3(pw_blocks(gc.n, 256, 8192)), dim3(256), 0, s, gf, gc,
                     tf, rc, scal);
}
template <typename T, typename C>
void prolong_add(const Grid& gf, const Grid& gc, T* zf, const C* ec, const double* scal,
                 bool overwrite, hipStream_t s) {
  hipLaunchKernelGGL((prolong_kernel<T, C>), dim3(pw_blocks(gf.n, 256, 8192)), dim3(256), 0, s, gf, gc,
                     zf, ec, scal, overwrite ? 1 : 0);
}
template <typename S, typename T>
void galerkin_first(const Grid& gf, const Grid& gc, const S* s, const double* msig_dev, T* st,
                    hipStream_t stm) {
  hipLaunchKernelGGL((galerkin_first_kernel<S, T>), dim3(pw_blocks(gc.n, 256, 4096), 27), dim3(256), 0,
                     stm, gf, gc, s, msig_dev, st);
}
template <typename T>
void galerkin_next(const Grid& gf, const Grid& gc, const T* stf, T* stc, hipStream_t stm) {
  hipLaunchKernelGGL(galerkin_next_kernel<T>, dim3(pw_blocks(gc.n, 256, 4096), 27), dim3(256), 0,
                     stm, gf, gc, stf, stc);
}
template <typename T>
void dinv_from_stencil(const Grid& g, const T* st, double omega, T* dinv, hipStream_t stm) {
  hipLaunchKernelGGL(dinv_stencil_kernel<T>, dim3(pw_blocks(g.n, 256, 8192)), dim3(256), 0, stm, g,
                     st, omega, dinv);
}
template <typename T>
void dense_from_stencil(const Grid& g, const T* st, double* A, hipStream_t stm) {
  hipLaunchKernelGGL(dense_kernel<T>, dim3(pw_blocks(g.n, 64, 4096)), dim3(64), 0, stm, g, st, A);
  hipLaunchKernelGGL(pin_kernel, dim3(pw_blocks(3 * g.n, 256, 4096)), dim3(256), 0, stm,
                     (int64_t)(3 * g.n), A);
}
void gauss_jordan_inverse(int N, double* A, hipStream_t stm) {
  // scratch column lives right after the matrix (allocated by the caller)
  hipLaunchKernelGGL(gj_kernel, dim3(1), dim3(1024), 0, stm, N, A, A + (int64_t)N * N);
}
template <typename R, typename T>
void coarse_solve(const Grid& g, const double* Ainv, const R* r, T* z, const double* scal,
                  hipStream_t stm) {
  const size_t shm = sizeof(double) * 6 * g.n;
  hipLaunchKernelGGL((coarse_solve_kernel<R, T>), dim3(NCASE), dim3(1024), shm, stm, g, Ainv, r, z,
                     scal);
}

#define HMG_INSTKC(T, W)                                                                         \
  template void kc_apply<T, W>(const Grid&, const W*, const T*, T*, hipStream_t);                 \
  template void kc_residual<T, W>(const Grid&, const W*, const T*, const T*, T*, const double*,   \
                                  const double*, hipStream_t);                                      \
  template void kc_smooth<T, W>(const Grid&, const W*, const T*, const T*, const W*, T*,          \
                                const double*, const double*, hipStream_t);
HMG_INSTKC(float, float)
HMG_INSTKC(double, double)
HMG_INSTKC(bf16, bf16)
HMG_INSTKC(bf16, float)
#undef HMG_INSTKC
#define HMG_INST(T)                                                                               \
  template void restrict_to<T>(const Grid&, const Grid&, const T*, T*, const double*, hipStream_t); \
  template void prolong_add<T, T>(const Grid&, const Grid&, T*, const T*, const double*, bool,    \
                               hipStream_t);                                                        \
  template void galerkin_next<T>(const Grid&, const Grid&, const T*, T*, hipStream_t);            \
  template void dinv_from_stencil<T>(const Grid&, const T*, double, T*, hipStream_t);             \
  template void dense_from_stencil<T>(const Grid&, const T*, double*, hipStream_t);               \
  template void coarse_solve<T, T>(const Grid&, const double*, const T*, T*, const double*,       \
                                   hipStream_t);
HMG_INST(float)
HMG_INST(double)
HMG_INST(bf16)
#undef HMG_INST
template void galerkin_first<float, float>(const Grid&, const Grid&, const float*, const double*,
                                           float*, hipStream_t);
template void galerkin_first<double, double>(const Grid&, const Grid&, const double*,
                                             const double*, double*, hipStream_t);
template void prolong_add<bf16, float>(const Grid&, const Grid&, bf16*, const float*,
                                       const double*, bool, hipStream_t);
template void coarse_solve<bf16, float>(const Grid&, const double*, const bf16*, float*,
                                        const double*, hipStream_t);
template void prolong_add<float, bf16>(const Grid&, const Grid&, float*, const bf16*,
                                       const double*, bool, hipStream_t);
template void coarse_solve<float, bf16>(const Grid&, const double*, const float*, bf16*,
                                        const double*, hipStream_t);
template void galerkin_first<float, bf16>(const Grid&, const Grid&, const float*, const double*,
                                          bf16*, hipStream_t);

}  // namespace hmg

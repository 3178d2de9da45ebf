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

// Rounded (bf16) stencils: a translation t of the whole grid (or of a stiff
// island floating in Emin-void) costs no energy, so the 27 blocks of a row sum
// to zero, and rounding each block on its own breaks that.  The centre block
// is therefore never taken from storage: it is the negated sum of the 26
// stored off-centre blocks (in FP64), and the operator is applied in the
// difference form sum_{d != 0} K_d (u_{v+d} - u_v), which keeps every such
// translation in the null space exactly.  Stencils of wider types keep their
// stored centre.
template <typename W>
constexpr bool kCentreFromSum = std::is_same<W, bf16>::value;

template <typename W>
__device__ __forceinline__ void centre_block(const W* __restrict__ st, int64_t n, int64_t v,
                                             double (&c)[9]) {
  if (kCentreFromSum<W>) {
#pragma unroll
    for (int t = 0; t < 9; ++t) c[t] = 0.0;
    for (int d = 0; d < 27; ++d) {
      if (d == 13) continue;
#pragma unroll
      for (int t = 0; t < 9; ++t) c[t] -= to_d(st[(int64_t)(d * 9 + t) * n + v]);
    }
  } else {
#pragma unroll
    for (int t = 0; t < 9; ++t) c[t] = to_d(st[(int64_t)(13 * 9 + t) * n + v]);
  }
}

// Two consecutive values of a row (the even one first): one aligned load or
// store of 2 * sizeof(T) bytes.  Rows start at even offsets (every grid that
// is coarsened has even extents), so 2X is always pair-aligned.
template <typename T>
struct alignas(2 * sizeof(T)) Pair {
  T v[2];
};

// Stored stencil coefficients are read once per pass and never again by any
// block, while the vectors they multiply are read by the 27 neighbouring
// vertices; the coefficient loads are therefore non-temporal (streaming), so
// that they do not push the neighbours' vector lines out of L2.  At 256^3 this
// took the level-1 residual pass from 27.5 to 24.7 GB of reads (5.4 -> 4.9 ms).
// The prolongation reads its fine field once the same way, keeping the coarse
// values that eight fine vertices share (4.3 -> 4.1 ms at level 1 -> 0).
template <typename W>
__device__ __forceinline__ W ld_coef(const W* p) {
  if constexpr (sizeof(W) == 2)
    return __builtin_bit_cast(
        W, __builtin_nontemporal_load(reinterpret_cast<const unsigned short*>(p)));
  else
    return __builtin_nontemporal_load(p);
}
template <typename W>
__device__ __forceinline__ Pair<W> ld_coef_pair(const W* p) {
  if constexpr (sizeof(W) == 2) {
    return __builtin_bit_cast(
        Pair<W>, __builtin_nontemporal_load(reinterpret_cast<const unsigned int*>(p)));
  } else {
    typedef W w2 __attribute__((ext_vector_type(2)));
    const w2 v = __builtin_nontemporal_load(reinterpret_cast<const w2*>(p));
    Pair<W> r;
    r.v[0] = v.x;
    r.v[1] = v.y;
    return r;
  }
}

// Row r of a launch over `rows` rows: consecutive block indices go to
// different XCDs, so hand each XCD a contiguous range of rows (neighbouring
// rows share their coarse or fine partner rows in that XCD's L2).
__device__ __forceinline__ int xcd_row(int rows) {
  const int b = blockIdx.x;
  if (rows % 8 != 0) return b;
  return (b & 7) * (rows >> 3) + (b >> 3);
}

inline int row_threads(int nx) { return nx >= 256 ? 256 : (nx > 64 ? 128 : 64); }

// MODE 0: out = K u.  MODE 1: out = (r - m) - K u.  MODE 2: out = u + Dinv ((r - m) - K u).
// m is the per-component mean of r (slots S_MEAN* of `mean`, FP64).
//
// One block per grid row (y, z), a thread per x.  The 27 neighbour offsets
// are 32-bit (a level holds fewer than 2^31 vertices) on top of uniform
// component base pointers.  Every case is computed whether active or not, so
// that no load waits behind a branch; the sums of an inactive case depend on
// its own (stale) buffers only and are never stored.  The stencil stream, read
// once for all six cases, dominates the traffic either way.
template <typename T, typename W, int MODE>
__global__ void stencil_kernel(Grid g, const W* __restrict__ st, const T* __restrict__ u,
                               const T* __restrict__ r, const W* __restrict__ dinv,
                               T* __restrict__ out, const double* scal, const double* mean) {
  using A = typename Acc<T>::type;
  bool on[NCASE];
#pragma unroll
  for (int c = 0; c < NCASE; ++c) on[c] = case_on(scal, c);
  const int n = (int)g.n;
  const int row = xcd_row(g.ny * g.nz);
  const int gy = row % g.ny, gz = row / g.ny;
  for (int gx = threadIdx.x; gx < g.nx; gx += blockDim.x) {
    const int i = row * g.nx + gx;
    A acc[NCASE][3];
#pragma unroll
    for (int c = 0; c < NCASE; ++c) acc[c][0] = acc[c][1] = acc[c][2] = A(0);
    A uc[NCASE][3];  // u at v, subtracted in the difference form
#pragma unroll
    for (int c = 0; c < NCASE; ++c)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        uc[c][k] = kCentreFromSum<W> ? (A)(u + (size_t)(c * 3 + k) * n)[i] : A(0);
    // neighbour rows (dy, dz), then the three x offsets of each row
    for (int a = 0; a < 9; ++a) {
      int y = gy + a % 3 - 1, z = gz + a / 3 - 1;
      y = y < 0 ? y + g.ny : (y == g.ny ? 0 : y);
      z = z < 0 ? z + g.nz : (z == g.nz ? 0 : z);
      const int rb = g.nx * (y + g.ny * z);
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        if (kCentreFromSum<W> && a == 4 && dx == 1) continue;
        int x = gx + dx - 1;
        x = x < 0 ? x + g.nx : (x == g.nx ? 0 : x);
        const int w = rb + x;
        const W* sd = st + (size_t)((3 * a + dx) * 9) * n;
        A K[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) K[t] = (A)ld_coef(sd + (size_t)t * n + i);
#pragma unroll
        for (int c = 0; c < NCASE; ++c) {
          const A u0 = (A)(u + (size_t)(c * 3 + 0) * n)[w] - uc[c][0];
          const A u1 = (A)(u + (size_t)(c * 3 + 1) * n)[w] - uc[c][1];
          const A u2 = (A)(u + (size_t)(c * 3 + 2) * n)[w] - uc[c][2];
          acc[c][0] += K[0] * u0 + K[1] * u1 + K[2] * u2;
          acc[c][1] += K[3] * u0 + K[4] * u1 + K[5] * u2;
          acc[c][2] += K[6] * u0 + K[7] * u1 + K[8] * u2;
        }
      }
    }
    A D[6];
    if (MODE == 2) {
#pragma unroll
      for (int t = 0; t < 6; ++t) D[t] = (A)(dinv + (size_t)t * n)[i];
    }
#pragma unroll
    for (int c = 0; c < NCASE; ++c) {
      if (!on[c]) continue;
      if (MODE == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) (out + (size_t)(c * 3 + k) * n)[i] = (T)acc[c][k];
      } else {
        A res[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
          res[k] = (A)(to_d((r + (size_t)(c * 3 + k) * n)[i]) - mean[(S_MEAN0 + k) * 8 + c]) -
                   acc[c][k];
        if (MODE == 1) {
#pragma unroll
          for (int k = 0; k < 3; ++k) (out + (size_t)(c * 3 + k) * n)[i] = (T)res[k];
        } else {
          const A z0 = (A)(u + (size_t)(c * 3 + 0) * n)[i] + (D[0] * res[0] + D[3] * res[1] + D[5] * res[2]);
          const A z1 = (A)(u + (size_t)(c * 3 + 1) * n)[i] + (D[3] * res[0] + D[1] * res[1] + D[4] * res[2]);
          const A z2 = (A)(u + (size_t)(c * 3 + 2) * n)[i] + (D[5] * res[0] + D[4] * res[1] + D[2] * res[2]);
          (out + (size_t)(c * 3 + 0) * n)[i] = (T)z0;
          (out + (size_t)(c * 3 + 1) * n)[i] = (T)z1;
          (out + (size_t)(c * 3 + 2) * n)[i] = (T)z2;
        }
      }
    }
  }
}

// The same three modes for a pair of vertices (x0, x0 + 1) per thread, used
// for FP32 and bf16 stencils on rows of even length.  The
// two vertices share their neighbour columns: per neighbour row and component
// one paired load (x0, x0 + 1) and two single loads (x0 - 1, x0 + 2) replace
// six loads, and every stencil coefficient of the pair is one paired load.
// Rounded stencils skip the centre block and use the difference form.
template <typename T, typename W, int MODE>
__global__ void __launch_bounds__(256)
stencil2_kernel(Grid g, const W* __restrict__ st, const T* __restrict__ u, const T* __restrict__ r,
                const W* __restrict__ dinv, T* __restrict__ out, const double* scal,
                const double* mean) {
  using A = typename Acc<T>::type;
  bool on[NCASE];
#pragma unroll
  for (int c = 0; c < NCASE; ++c) on[c] = case_on(scal, c);
  const int n = (int)g.n;
  const int row = xcd_row(g.ny * g.nz);
  const int gy = row % g.ny, gz = row / g.ny;
  const int np = g.nx >> 1;
  for (int px = threadIdx.x; px < np; px += blockDim.x) {
    const int x0 = 2 * px;
    const int i = row * g.nx + x0;  // vertex A; vertex B = i + 1
    A acc[2][NCASE][3];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < NCASE; ++c) acc[h][c][0] = acc[h][c][1] = acc[h][c][2] = A(0);
    const int xm = x0 == 0 ? g.nx - 1 : x0 - 1;
    const int xp = x0 + 2 == g.nx ? 0 : x0 + 2;
    constexpr bool kDiff = kCentreFromSum<W>;
    A uc[2][NCASE][3];  // u at the pair, subtracted in the difference form
    if (kDiff) {
#pragma unroll
      for (int c = 0; c < NCASE; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const Pair<T> own = *reinterpret_cast<const Pair<T>*>(u + (size_t)(c * 3 + k) * n + i);
          uc[0][c][k] = (A)own.v[0];
          uc[1][c][k] = (A)own.v[1];
        }
    }
    for (int a = 0; a < 9; ++a) {
      int y = gy + a % 3 - 1, z = gz + a / 3 - 1;
      y = y < 0 ? y + g.ny : (y == g.ny ? 0 : y);
      z = z < 0 ? z + g.nz : (z == g.nz ? 0 : z);
      const int rb = g.nx * (y + g.ny * z);
      // coefficients of both vertices for the three x offsets of this row (a
      // rounded stencil's centre block is zero here: the difference form)
      A K[3][2][9];
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const W* sd = st + (size_t)((3 * a + dx) * 9) * n;
        const bool skip = kDiff && a == 4 && dx == 1;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          Pair<W> kp;
          if (skip) {
            kp.v[0] = kp.v[1] = W(0.0f);
          } else {
            kp = ld_coef_pair<W>(sd + (size_t)t * n + i);
          }
          K[dx][0][t] = (A)kp.v[0];
          K[dx][1][t] = (A)kp.v[1];
        }
      }
#pragma unroll
      for (int c = 0; c < NCASE; ++c) {
        A uu[4][3];  // columns x0 - 1, x0, x0 + 1, x0 + 2
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T* uk = u + (size_t)(c * 3 + k) * n + rb;
          const Pair<T> mid = *reinterpret_cast<const Pair<T>*>(uk + x0);
          uu[0][k] = (A)uk[xm];
          uu[1][k] = (A)mid.v[0];
          uu[2][k] = (A)mid.v[1];
          uu[3][k] = (A)uk[xp];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) {
            const A* Kd = K[dx][h];
            A v[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) v[k] = kDiff ? uu[h + dx][k] - uc[h][c][k] : uu[h + dx][k];
            acc[h][c][0] += Kd[0] * v[0] + Kd[1] * v[1] + Kd[2] * v[2];
            acc[h][c][1] += Kd[3] * v[0] + Kd[4] * v[1] + Kd[5] * v[2];
            acc[h][c][2] += Kd[6] * v[0] + Kd[7] * v[1] + Kd[8] * v[2];
          }
      }
    }
    A D[2][6];
    if (MODE == 2) {
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const Pair<W> dp = *reinterpret_cast<const Pair<W>*>(dinv + (size_t)t * n + i);
        D[0][t] = (A)dp.v[0];
        D[1][t] = (A)dp.v[1];
      }
    }
#pragma unroll
    for (int c = 0; c < NCASE; ++c) {
      if (!on[c]) continue;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        Pair<T>* o = reinterpret_cast<Pair<T>*>(out + (size_t)(c * 3 + k) * n + i);
        if (MODE == 0) {
          Pair<T> w;
          w.v[0] = (T)acc[0][c][k];
          w.v[1] = (T)acc[1][c][k];
          *o = w;
        }
      }
      if (MODE != 0) {
        A res[2][3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const Pair<T> rp = *reinterpret_cast<const Pair<T>*>(r + (size_t)(c * 3 + k) * n + i);
          const double m = mean[(S_MEAN0 + k) * 8 + c];
          res[0][k] = (A)(to_d(rp.v[0]) - m) - acc[0][c][k];
          res[1][k] = (A)(to_d(rp.v[1]) - m) - acc[1][c][k];
        }
        if (MODE == 1) {
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            Pair<T> w;
            w.v[0] = (T)res[0][k];
            w.v[1] = (T)res[1][k];
            *reinterpret_cast<Pair<T>*>(out + (size_t)(c * 3 + k) * n + i) = w;
          }
        } else {
          A zz[2][3];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const A* Dh = D[h];
            zz[h][0] = Dh[0] * res[h][0] + Dh[3] * res[h][1] + Dh[5] * res[h][2];
            zz[h][1] = Dh[3] * res[h][0] + Dh[1] * res[h][1] + Dh[4] * res[h][2];
            zz[h][2] = Dh[5] * res[h][0] + Dh[4] * res[h][1] + Dh[2] * res[h][2];
          }
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const Pair<T> up = *reinterpret_cast<const Pair<T>*>(u + (size_t)(c * 3 + k) * n + i);
            Pair<T> w;
            w.v[0] = (T)((A)up.v[0] + zz[0][k]);
            w.v[1] = (T)((A)up.v[1] + zz[1][k]);
            *reinterpret_cast<Pair<T>*>(out + (size_t)(c * 3 + k) * n + i) = w;
          }
        }
      }
    }
  }
}

// Restriction R = P^T (unscaled weights, Sec. 3.3):
//   rc[V] = sum_{a in {-1,0,1}^3} w(a) tf[2V + a],  w(a) = prod_k (a_k == 0 ? 1 : 1/2).
// One block per coarse row Y, chunk of lz coarse planes and load case
// (blockIdx.y); a thread per coarse X reads the pair (2X, 2X+1) and the value
// 2X-1 of the fine rows 2Y+{-1,0,1} of the case's three components.  The block
// marches Z through its chunk: fine plane 2Z+1 (weight 1/2 for Z) is also plane
// 2(Z+1)-1 of the next coarse plane, so its weighted row sum is kept and each
// step after the first reads two fine planes instead of three.
template <typename T>
__global__ void restrict_kernel(Grid gf, Grid gc, const T* __restrict__ tf, T* __restrict__ rc,
                                const double* scal, int lz) {
  using A = typename Acc<T>::type;
  const int c = blockIdx.y;
  if (!case_on(scal, c)) return;
  const int nzc = (gc.nz + lz - 1) / lz;
  const int item = xcd_row(gc.ny * nzc);
  const int Y = item % gc.ny, Z0 = (item / gc.ny) * lz;
  const int Z1 = min(Z0 + lz, gc.nz);
  const int ys[3] = {Y == 0 ? gf.ny - 1 : 2 * Y - 1, 2 * Y, 2 * Y + 1};
  const int64_t fplane = (int64_t)gf.nx * gf.ny;
  for (int X = threadIdx.x; X < gc.nx; X += blockDim.x) {
    const int xm = X == 0 ? gf.nx - 1 : 2 * X - 1;
    // y- and x-weighted sum of fine plane z of component k at (2X, 2Y)
    auto plane_sum = [&](int k, int z) {
      const T* f = tf + (int64_t)(c * 3 + k) * gf.n + fplane * z;
      A rowsum[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int64_t fb = (int64_t)gf.nx * ys[a];
        const Pair<T> p = *reinterpret_cast<const Pair<T>*>(f + fb + 2 * X);
        rowsum[a] = (A)p.v[0] + A(0.5) * ((A)p.v[1] + (A)f[fb + xm]);
      }
      return rowsum[1] + A(0.5) * (rowsum[0] + rowsum[2]);
    };
    A kept[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) kept[k] = plane_sum(k, Z0 == 0 ? gf.nz - 1 : 2 * Z0 - 1);
    for (int Z = Z0; Z < Z1; ++Z) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const A s0 = kept[k], s1 = plane_sum(k, 2 * Z), s2 = plane_sum(k, 2 * Z + 1);
        // weights 1/2, 1, 1/2 along z
        A s = A(0);
        s += A(0.5) * s0;
        s += A(1) * s1;
        s += A(0.5) * s2;
        rc[(int64_t)(c * 3 + k) * gc.n + (int64_t)gc.nx * (Y + (int64_t)gc.ny * Z) + X] = (T)s;
        kept[k] = s2;
      }
    }
  }
}

// Trilinear prolongation P: zf (+)= P ec.  A fine vertex takes the mean of the
// coarse vertices of its coarse cell that it lies between: 1, 2, 4 or 8 of
// them by the parities of its coordinates.  One block per fine row (y, z) and
// load case (blockIdx.y); a thread per coarse X writes the fine pair
// (2X, 2X+1) of the case's three components.  The four coarse rows
// (Y0|Y1) x (Z0|Z1) are always summed, with Y1 = Y0 (Z1 = Z0) for an even y
// (z): the duplicated terms double exactly, so the quarter of the sum is the
// mean without any branch.
template <typename T, typename C, bool OVERWRITE>
__global__ void prolong_kernel(Grid gf, Grid gc, T* __restrict__ zf, const C* __restrict__ ec,
                               const double* scal) {
  using A = typename Acc<T>::type;
  const int c = blockIdx.y;
  if (!case_on(scal, c)) return;
  const int row = xcd_row(gf.ny * gf.nz);
  const int y = row % gf.ny, z = row / gf.ny;
  const int Y0 = y >> 1, Z0 = z >> 1;
  const int Y1 = (y & 1) ? (Y0 + 1 == gc.ny ? 0 : Y0 + 1) : Y0;
  const int Z1 = (z & 1) ? (Z0 + 1 == gc.nz ? 0 : Z0 + 1) : Z0;
  const int64_t cr[4] = {(int64_t)gc.nx * (Y0 + (int64_t)gc.ny * Z0),
                         (int64_t)gc.nx * (Y1 + (int64_t)gc.ny * Z0),
                         (int64_t)gc.nx * (Y0 + (int64_t)gc.ny * Z1),
                         (int64_t)gc.nx * (Y1 + (int64_t)gc.ny * Z1)};
  const int64_t fbase = (int64_t)row * gf.nx;
  for (int X = threadIdx.x; X < gc.nx; X += blockDim.x) {
    const int X1 = X + 1 == gc.nx ? 0 : X + 1;
    {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const C* e = ec + (int64_t)(c * 3 + k) * gc.n;
        const A s0 = ((A)e[cr[0] + X] + (A)e[cr[1] + X]) + ((A)e[cr[2] + X] + (A)e[cr[3] + X]);
        const A s1 = ((A)e[cr[0] + X1] + (A)e[cr[1] + X1]) + ((A)e[cr[2] + X1] + (A)e[cr[3] + X1]);
        const A v0 = A(0.25) * s0, v1 = A(0.125) * (s0 + s1);
        Pair<T>* o = reinterpret_cast<Pair<T>*>(zf + (int64_t)(c * 3 + k) * gf.n + fbase + 2 * X);
        Pair<T> p;
        if (OVERWRITE) {
          p.v[0] = (T)v0;
          p.v[1] = (T)v1;
        } else {
          p = ld_coef_pair<T>(reinterpret_cast<const T*>(o));  // read once: streaming
          p.v[0] = (T)((A)p.v[0] + v0);
          p.v[1] = (T)((A)p.v[1] + v1);
        }
        *o = p;
      }
    }
  }
}

// Non-dyadic first step (Sec. 4.2): the coarse grid is 4 times coarser per
// axis and the trilinear weights along an axis are (4 - |a|)/4, |a| <= 3
// (Eq. st-assemb-w with the coarse element 4 fine cells long).
__device__ __forceinline__ double w4(int a) { return (4 - (a < 0 ? -a : a)) * 0.25; }

// Restriction R = P^T for the factor-4 step: rc[V] = sum_a w4(a) tf[4V + a]
// over a in {-3..3}^3.  A thread per coarse vertex and load case; the fine
// rows 4Y + ay, 4Z + az are visited in turn.
template <typename T>
__global__ void restrict4_kernel(Grid gf, Grid gc, const T* __restrict__ tf, T* __restrict__ rc,
                                 const double* scal) {
  using A = typename Acc<T>::type;
  const int c = blockIdx.y;
  if (!case_on(scal, c)) return;
  for (int64_t V = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; V < gc.n;
       V += (int64_t)gridDim.x * blockDim.x) {
    const int X = (int)(V % gc.nx);
    const int Y = (int)((V / gc.nx) % gc.ny);
    const int Z = (int)(V / ((int64_t)gc.nx * gc.ny));
    A acc[3] = {A(0), A(0), A(0)};
    for (int az = -3; az <= 3; ++az) {
      const int z = modp(4 * Z + az, gf.nz);
      for (int ay = -3; ay <= 3; ++ay) {
        const int y = modp(4 * Y + ay, gf.ny);
        const A wyz = (A)(w4(ay) * w4(az));
        const int64_t rb = (int64_t)gf.nx * (y + (int64_t)gf.ny * z);
#pragma unroll
        for (int ax = -3; ax <= 3; ++ax) {
          const int x = modp(4 * X + ax, gf.nx);
          const A w = wyz * (A)w4(ax);
#pragma unroll
          for (int k = 0; k < 3; ++k) acc[k] += w * (A)tf[(int64_t)(c * 3 + k) * gf.n + rb + x];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) rc[(int64_t)(c * 3 + k) * gc.n + V] = (T)acc[k];
  }
}

// Prolongation P for the factor-4 step: fine coordinate 4X + r takes coarse X
// with weight (4 - r)/4 and X + 1 with r/4, axis by axis.  A thread per fine
// vertex and load case.
template <typename T, typename C, bool OVERWRITE>
__global__ void prolong4_kernel(Grid gf, Grid gc, T* __restrict__ zf, const C* __restrict__ ec,
                                const double* scal) {
  using A = typename Acc<T>::type;
  const int c = blockIdx.y;
  if (!case_on(scal, c)) return;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < gf.n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(v % gf.nx);
    const int y = (int)((v / gf.nx) % gf.ny);
    const int z = (int)(v / ((int64_t)gf.nx * gf.ny));
    const int X0 = x >> 2, Y0 = y >> 2, Z0 = z >> 2;
    const int rx = x & 3, ry = y & 3, rz = z & 3;
    const int X1 = X0 + 1 == gc.nx ? 0 : X0 + 1;
    const int Y1 = Y0 + 1 == gc.ny ? 0 : Y0 + 1;
    const int Z1 = Z0 + 1 == gc.nz ? 0 : Z0 + 1;
    const A wx[2] = {A(4 - rx) * A(0.25), A(rx) * A(0.25)};
    const A wy[2] = {A(4 - ry) * A(0.25), A(ry) * A(0.25)};
    const A wz[2] = {A(4 - rz) * A(0.25), A(rz) * A(0.25)};
    const int Xs[2] = {X0, X1}, Ys[2] = {Y0, Y1}, Zs[2] = {Z0, Z1};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const C* e = ec + (int64_t)(c * 3 + k) * gc.n;
      A acc = A(0);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int qx = q & 1, qy = (q >> 1) & 1, qz = q >> 2;
        acc += wx[qx] * wy[qy] * wz[qz] *
               (A)e[Xs[qx] + (int64_t)gc.nx * (Ys[qy] + (int64_t)gc.ny * Zs[qz])];
      }
      T* o = zf + (int64_t)(c * 3 + k) * gf.n + v;
      *o = OVERWRITE ? (T)acc : (T)((A)*o + acc);
    }
  }
}

// First coarse level from the densities, for a coarse grid F = 2 or 4 times
// coarser per axis.  Coarse vertex V is local node A of the coarse element with
// origin V - A; that element holds the F^3 fine elements F(V - A) + sigma, each
// contributing s * (W_sigma^T K0 W_sigma)[A, A + D] (msig: F^3 matrices 24x24).
template <typename S, typename T>
__global__ void galerkin_first_kernel(Grid gf, Grid gc, const S* __restrict__ s,
                                      const double* __restrict__ msig, T* __restrict__ st) {
  const int F = gf.nx / gc.nx;
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
      for (int sg = 0; sg < F * F * F; ++sg) {
        const int sx = sg % F, sy = (sg / F) % F, sz = sg / (F * F);
        const int64_t e = (F * CX + sx) +
                          (int64_t)gf.nx * ((F * CY + sy) + (int64_t)gf.ny * (F * CZ + sz));
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
        if (kCentreFromSum<T> && dp == 13) {
          double cb[9];
          centre_block(stf, gf.n, i, cb);
#pragma unroll
          for (int t = 0; t < 9; ++t) blk[t] += w * cb[t];
          continue;
        }
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
    centre_block(st, g.n, i, a);
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

__global__ void zero_kernel(int64_t count, double* __restrict__ A) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    A[i] = 0.0;
}

// Dense coarsest matrix (the three rows of a vertex per thread, added into a
// cleared matrix), then vertex 0 pinned to the identity.
template <typename T>
__global__ void dense_kernel(Grid g, const T* __restrict__ st, double* __restrict__ A) {
  const int64_t N = 3 * g.n;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < g.n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int gx = (int)(v % g.nx);
    const int gy = (int)((v / g.nx) % g.ny);
    const int gz = (int)(v / ((int64_t)g.nx * g.ny));
    for (int d = 0; d < 27; ++d) {
      const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
      const int64_t w = modp(gx + dx, g.nx) +
                        (int64_t)g.nx * (modp(gy + dy, g.ny) + (int64_t)g.ny * modp(gz + dz, g.nz));
      double b[9];
      if (d == 13) {
        centre_block(st, g.n, v, b);
      } else {
#pragma unroll
        for (int t = 0; t < 9; ++t) b[t] = to_d(st[(int64_t)(d * 9 + t) * g.n + v]);
      }
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) A[(3 * v + p) * N + 3 * w + q] += b[p * 3 + q];
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

// Blocked Gauss-Jordan inverse for the larger coarsest grids, one panel of
// GJ_B pivots at a time.  With the panel's rows and columns K and the rest I:
//   A[K,K] <- P^-1,  A[K,I] <- P^-1 A[K,I],  A[I,K] <- -A[I,K] P^-1,
//   A[I,I] <- A[I,I] - A[I,K] P^-1 A[K,I]      (P = A[K,K]),
// which after the last panel leaves the inverse in A (no pivoting: A is SPD).
constexpr int GJ_B = 32;

// P^-1 of the panel's diagonal block (b <= GJ_B) by unblocked GJ in LDS.
__global__ void __launch_bounds__(1024) gj_panel_inverse_kernel(int N, const double* __restrict__ A,
                                                                int k0, int b,
                                                                double* __restrict__ Pi) {
  __shared__ double P[GJ_B][GJ_B + 1];
  __shared__ double col[GJ_B], rowk[GJ_B];
  const int t = threadIdx.x, r = t / GJ_B, c = t % GJ_B;
  if (r < b && c < b) P[r][c] = A[(int64_t)(k0 + r) * N + k0 + c];
  __syncthreads();
  for (int k = 0; k < b; ++k) {
    const double piv = 1.0 / P[k][k];
    if (t < b) {
      col[t] = P[t][k];
      rowk[t] = P[k][t];
    }
    __syncthreads();
    if (r < b && c < b) {
      if (r == k)
        P[r][c] = (c == k) ? piv : rowk[c] * piv;
      else
        P[r][c] = (c == k) ? -col[r] * piv : P[r][c] - col[r] * piv * rowk[c];
    }
    __syncthreads();
  }
  // entries beyond a ragged last panel are zero (the row-panel kernel sums
  // over all GJ_B columns)
  Pi[r * GJ_B + c] = (r < b && c < b) ? P[r][c] : 0.0;
}

// Save the old column panel: Cs[i][m] = A[i][k0 + m].
__global__ void gj_save_columns_kernel(int N, const double* __restrict__ A, int k0, int b,
                                       double* __restrict__ Cs) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)N * GJ_B;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / GJ_B), m = (int)(e % GJ_B);
    Cs[e] = m < b ? A[(int64_t)i * N + k0 + m] : 0.0;
  }
}

// Row panel: A[K, j] <- P^-1 A[K, j] (j outside K), A[K, K] <- P^-1.
__global__ void gj_row_panel_kernel(int N, double* __restrict__ A, int k0, int b,
                                    const double* __restrict__ Pi) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x) {
    if (j >= k0 && j < k0 + b) {
      for (int m = 0; m < b; ++m) A[(int64_t)(k0 + m) * N + j] = Pi[m * GJ_B + (j - k0)];
      continue;
    }
    double old[GJ_B];
#pragma unroll
    for (int l = 0; l < GJ_B; ++l) old[l] = l < b ? A[(int64_t)(k0 + l) * N + j] : 0.0;
    for (int m = 0; m < b; ++m) {
      double a = 0.0;
#pragma unroll
      for (int l = 0; l < GJ_B; ++l) a += Pi[m * GJ_B + l] * old[l];
      A[(int64_t)(k0 + m) * N + j] = a;
    }
  }
}

// Trailing update of the rows outside K, a 64 x 64 tile per block (4 x 4 per
// thread): A[i][j] <- [j outside K] A[i][j] - sum_m Cs[i][m] A[k0 + m][j].
// For j in K the row panel holds P^-1, giving -A[I,K] P^-1.
__global__ void __launch_bounds__(256) gj_update_kernel(int N, double* __restrict__ A, int k0,
                                                        int b, const double* __restrict__ Cs) {
  __shared__ double Ct[64][GJ_B + 1];
  __shared__ double Rt[GJ_B][64 + 1];
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int t = threadIdx.x;
  for (int e = t; e < 64 * GJ_B; e += 256) {
    const int ii = e / GJ_B, m = e % GJ_B;
    Ct[ii][m] = (i0 + ii < N) ? Cs[(int64_t)(i0 + ii) * GJ_B + m] : 0.0;
  }
  for (int e = t; e < GJ_B * 64; e += 256) {
    const int m = e / 64, jj = e % 64;
    Rt[m][jj] = (m < b && j0 + jj < N) ? A[(int64_t)(k0 + m) * N + j0 + jj] : 0.0;
  }
  __syncthreads();
  const int tx = t % 16, ty = t / 16;
  double acc[4][4] = {};
  for (int m = 0; m < GJ_B; ++m) {
    double cv[4], rv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) cv[a] = Ct[ty * 4 + a][m];
#pragma unroll
    for (int q = 0; q < 4; ++q) rv[q] = Rt[m][tx * 4 + q];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[a][q] += cv[a] * rv[q];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = i0 + ty * 4 + a;
    if (i >= N || (i >= k0 && i < k0 + b)) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + tx * 4 + q;
      if (j >= N) continue;
      double* aij = A + (int64_t)i * N + j;
      *aij = ((j >= k0 && j < k0 + b) ? 0.0 : *aij) - acc[a][q];
    }
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

// Coarsest solve for grids whose right-hand sides do not fit in LDS, in three
// passes over global scratch (same steps as coarse_solve_kernel):
// (1) the projected right-hand side X[c][i], zero at the pinned vertex;
template <typename R>
__global__ void __launch_bounds__(1024) cs_rhs_kernel(Grid g, const R* __restrict__ r,
                                                      double* __restrict__ X, const double* scal) {
  __shared__ double red[16];
  const int c = blockIdx.x;
  if (!case_on(scal, c)) return;
  const int n = (int)g.n, N = 3 * n;
  for (int k = 0; k < 3; ++k) {
    double a = 0.0;
    for (int v = threadIdx.x; v < n; v += blockDim.x) a += to_d(r[(int64_t)(c * 3 + k) * n + v]);
    const double m = block_allsum(a, red) / n;
    for (int v = threadIdx.x; v < n; v += blockDim.x)
      X[(int64_t)c * N + 3 * v + k] =
          (v == 0) ? 0.0 : to_d(r[(int64_t)(c * 3 + k) * n + v]) - m;
  }
}

// (2) partial products Zp[jc][c][i] = sum over the jc-th slice of j of
// Ainv[j][i] X[c][j] (column i of the symmetric inverse, as the LDS form
// reads it), a thread per i, the slice of X staged in LDS;
constexpr int CS_SLICES = 16;
__global__ void __launch_bounds__(256) cs_gemv_kernel(int N, const double* __restrict__ Ainv,
                                                      const double* __restrict__ X,
                                                      double* __restrict__ Zp,
                                                      const double* scal) {
  extern __shared__ double xs[];  // [NCASE][len]
  const int jc = blockIdx.y;
  const int ja = (int)((int64_t)N * jc / CS_SLICES), jb = (int)((int64_t)N * (jc + 1) / CS_SLICES);
  const int len = jb - ja;
  bool on[NCASE];
#pragma unroll
  for (int c = 0; c < NCASE; ++c) on[c] = case_on(scal, c);
  for (int e = threadIdx.x; e < NCASE * len; e += blockDim.x) {
    const int c = e / len, j = e % len;
    xs[e] = on[c] ? X[(int64_t)c * N + ja + j] : 0.0;
  }
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double acc[NCASE] = {};
  for (int j = 0; j < len; ++j) {
    const double a = Ainv[(int64_t)(ja + j) * N + i];
#pragma unroll
    for (int c = 0; c < NCASE; ++c) acc[c] += a * xs[c * len + j];
  }
#pragma unroll
  for (int c = 0; c < NCASE; ++c) Zp[((int64_t)jc * NCASE + c) * N + i] = acc[c];
}

// (3) the slices summed in order, the result projected to zero mean per
// component and stored.
template <typename T>
__global__ void __launch_bounds__(1024) cs_finish_kernel(Grid g, const double* __restrict__ Zp,
                                                         T* __restrict__ z, const double* scal) {
  __shared__ double red[16];
  const int c = blockIdx.x;
  if (!case_on(scal, c)) return;
  const int n = (int)g.n, N = 3 * n;
  auto zval = [&](int i) {
    double a = 0.0;
    for (int jc = 0; jc < CS_SLICES; ++jc) a += Zp[((int64_t)jc * NCASE + c) * N + i];
    return a;
  };
  for (int k = 0; k < 3; ++k) {
    double a = 0.0;
    for (int v = threadIdx.x; v < n; v += blockDim.x) a += zval(3 * v + k);
    const double m = block_allsum(a, red) / n;
    for (int v = threadIdx.x; v < n; v += blockDim.x)
      z[(int64_t)(c * 3 + k) * n + v] = from_d<T>(zval(3 * v + k) - m);
  }
}

}  // namespace

// Paired-vertex stencil passes: FP32 or bf16 stencils with FP32 or bf16 vectors, and
// an even row.
template <typename T, typename W>
inline bool use_pairs(const Grid& g) {
  return (std::is_same<T, float>::value || std::is_same<T, bf16>::value) &&
         (std::is_same<W, float>::value || std::is_same<W, bf16>::value) && g.nx % 2 == 0;
}
template <typename T, typename W>
void kc_apply(const Grid& g, const W* st, const T* u, T* y, hipStream_t s) {
  if (use_pairs<T, W>(g))
    hipLaunchKernelGGL((stencil2_kernel<T, W, 0>), dim3(g.ny * g.nz), dim3(row_threads(g.nx / 2)),
                       0, s, g, st, u, (const T*)nullptr, (const W*)nullptr, y,
                       (const double*)nullptr, (const double*)nullptr);
  else
    hipLaunchKernelGGL((stencil_kernel<T, W, 0>), dim3(g.ny * g.nz), dim3(row_threads(g.nx)), 0, s,
                       g, st, u, (const T*)nullptr, (const W*)nullptr, y, (const double*)nullptr,
                       (const double*)nullptr);
}
template <typename T, typename W>
void kc_residual(const Grid& g, const W* st, const T* z, const T* r, T* t, const double* scal,
                 const double* mean, hipStream_t s) {
  if (use_pairs<T, W>(g))
    hipLaunchKernelGGL((stencil2_kernel<T, W, 1>), dim3(g.ny * g.nz), dim3(row_threads(g.nx / 2)),
                       0, s, g, st, z, r, (const W*)nullptr, t, scal, mean);
  else
    hipLaunchKernelGGL((stencil_kernel<T, W, 1>), dim3(g.ny * g.nz), dim3(row_threads(g.nx)), 0, s,
                       g, st, z, r, (const W*)nullptr, t, scal, mean);
}
template <typename T, typename W>
void kc_smooth(const Grid& g, const W* st, const T* z, const T* r, const W* dinv, T* zout,
               const double* scal, const double* mean, hipStream_t s) {
  if (use_pairs<T, W>(g))
    hipLaunchKernelGGL((stencil2_kernel<T, W, 2>), dim3(g.ny * g.nz), dim3(row_threads(g.nx / 2)),
                       0, s, g, st, z, r, dinv, zout, scal, mean);
  else
    hipLaunchKernelGGL((stencil_kernel<T, W, 2>), dim3(g.ny * g.nz), dim3(row_threads(g.nx)), 0, s,
                       g, st, z, r, dinv, zout, scal, mean);
}

inline bool factor4(const Grid& gf, const Grid& gc) { return gf.nx == 4 * gc.nx; }

template <typename T>
void restrict_to(const Grid& gf, const Grid& gc, const T* tf, T* rc, const double* scal,
                 hipStream_t s) {
  if (factor4(gf, gc)) {
    hipLaunchKernelGGL(restrict4_kernel<T>, dim3(pw_blocks(gc.n, 256, 4096), NCASE), dim3(256), 0,
                       s, gf, gc, tf, rc, scal);
    return;
  }
  // z-chunks of up to 8 coarse planes while each case keeps at least 4096 blocks
  int lz = 8;
  while (lz > 1 && gc.ny * ((gc.nz + lz - 1) / lz) < 4096) lz >>= 1;
  hipLaunchKernelGGL(restrict_kernel<T>, dim3(gc.ny * ((gc.nz + lz - 1) / lz), NCASE),
                     dim3(row_threads(gc.nx)), 0, s, gf, gc, tf, rc, scal, lz);
}
template <typename T, typename C>
void prolong_add(const Grid& gf, const Grid& gc, T* zf, const C* ec, const double* scal,
                 bool overwrite, hipStream_t s) {
  if (factor4(gf, gc)) {
    if (overwrite)
      hipLaunchKernelGGL((prolong4_kernel<T, C, true>), dim3(pw_blocks(gf.n, 256, 8192), NCASE),
                         dim3(256), 0, s, gf, gc, zf, ec, scal);
    else
      hipLaunchKernelGGL((prolong4_kernel<T, C, false>), dim3(pw_blocks(gf.n, 256, 8192), NCASE),
                         dim3(256), 0, s, gf, gc, zf, ec, scal);
    return;
  }
  if (overwrite)
    hipLaunchKernelGGL((prolong_kernel<T, C, true>), dim3(gf.ny * gf.nz, NCASE),
                       dim3(row_threads(gc.nx)), 0, s, gf, gc, zf, ec, scal);
  else
    hipLaunchKernelGGL((prolong_kernel<T, C, false>), dim3(gf.ny * gf.nz, NCASE),
                       dim3(row_threads(gc.nx)), 0, s, gf, gc, zf, ec, scal);
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
  const int64_t N = 3 * g.n;
  hipLaunchKernelGGL(zero_kernel, dim3(pw_blocks(N * N, 256, 8192)), dim3(256), 0, stm, N * N, A);
  hipLaunchKernelGGL(dense_kernel<T>, dim3(pw_blocks(g.n, 64, 4096)), dim3(64), 0, stm, g, st, A);
  hipLaunchKernelGGL(pin_kernel, dim3(pw_blocks(3 * g.n, 256, 4096)), dim3(256), 0, stm,
                     (int64_t)(3 * g.n), A);
}

// Coarsest grids of up to SMALL_COARSE_DOF unknowns use the one-workgroup
// inverse and keep their right-hand sides in LDS; larger ones (up to
// MAX_COARSE_DOF) the blocked inverse and the three-pass solve.
constexpr int SMALL_COARSE_DOF = 3072;

int64_t coarse_scratch_doubles(int N) {
  return (int64_t)N * GJ_B + GJ_B * GJ_B + (int64_t)NCASE * N * (1 + CS_SLICES);
}

void gauss_jordan_inverse(int N, double* A, hipStream_t stm) {
  // scratch lives right after the matrix (coarse_scratch_doubles, allocated by the caller)
  double* scr = A + (int64_t)N * N;
  if (N <= SMALL_COARSE_DOF) {
    hipLaunchKernelGGL(gj_kernel, dim3(1), dim3(1024), 0, stm, N, A, scr);
    return;
  }
  double* Cs = scr;
  double* Pi = scr + (int64_t)N * GJ_B;
  const dim3 tiles((N + 63) / 64, (N + 63) / 64);
  for (int k0 = 0; k0 < N; k0 += GJ_B) {
    const int b = std::min(GJ_B, N - k0);
    hipLaunchKernelGGL(gj_panel_inverse_kernel, dim3(1), dim3(GJ_B * GJ_B), 0, stm, N, A, k0, b,
                       Pi);
    hipLaunchKernelGGL(gj_save_columns_kernel, dim3(pw_blocks((int64_t)N * GJ_B, 256, 4096)),
                       dim3(256), 0, stm, N, A, k0, b, Cs);
    hipLaunchKernelGGL(gj_row_panel_kernel, dim3((N + 255) / 256), dim3(256), 0, stm, N, A, k0, b,
                       Pi);
    hipLaunchKernelGGL(gj_update_kernel, tiles, dim3(256), 0, stm, N, A, k0, b, Cs);
  }
}
template <typename R, typename T>
void coarse_solve(const Grid& g, const double* Ainv, const R* r, T* z, const double* scal,
                  hipStream_t stm) {
  const int N = (int)(3 * g.n);
  if (N <= SMALL_COARSE_DOF) {
    const size_t shm = sizeof(double) * 6 * g.n;
    hipLaunchKernelGGL((coarse_solve_kernel<R, T>), dim3(NCASE), dim3(1024), shm, stm, g, Ainv, r,
                       z, scal);
    return;
  }
  double* X = const_cast<double*>(Ainv) + (int64_t)N * N + (int64_t)N * GJ_B + GJ_B * GJ_B;
  double* Zp = X + (int64_t)NCASE * N;
  hipLaunchKernelGGL((cs_rhs_kernel<R>), dim3(NCASE), dim3(1024), 0, stm, g, r, X, scal);
  const size_t shm = sizeof(double) * NCASE * ((N + CS_SLICES - 1) / CS_SLICES);
  hipLaunchKernelGGL(cs_gemv_kernel, dim3((N + 255) / 256, CS_SLICES), dim3(256), shm, stm, N,
                     Ainv, X, Zp, scal);
  hipLaunchKernelGGL((cs_finish_kernel<T>), dim3(NCASE), dim3(1024), 0, stm, g, Zp, z, scal);
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

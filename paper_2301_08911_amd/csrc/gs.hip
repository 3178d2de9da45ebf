// Eight-colour symmetric block Gauss-Seidel smoothing (Sec. 4.1 vertex
// subsets, Sec. 4.2 Eq. st-assemb-gs / st-gs-relx).
//
// Vertex (x, y, z) has colour (x mod 2) + 2 (y mod 2) + 4 (z mod 2).  No two
// vertices of one colour are neighbours in the 27-point stencil, so a colour
// is relaxed in parallel: at each of its vertices
//   S_v u_v = (f - m)_v - M_v,   i.e.  u_v += S_v^-1 ((f - m)_v - [K u]_v),
// with S_v the 3x3 diagonal block of row v and m the per-component mean of
// the level's right-hand side (the translation null space, removed before
// smoothing as on every level).  A forward sweep takes colours 0..7 and a
// backward sweep 7..0, so a V-cycle with forward pre- and backward
// post-smoothing is a symmetric preconditioner.
//
// Colours 2k and 2k+1 differ only in the x parity: both lie on the grid rows
// whose (y mod 2, z mod 2) is (k & 1, k >> 1), here called rows of pair k.  A
// vertex of colour 2k+1 has exactly two neighbours of colour 2k, (x - 1, y, z)
// and (x + 1, y, z), both on its own row, and rows of one pair are two apart,
// so no row of a pair reads another row of the same pair.  One launch
// therefore relaxes both colours of a pair: every block takes whole rows,
// relaxes the first x parity, keeps the new values in LDS, and after a
// barrier relaxes the second parity against them.  A sweep is four launches.
//
// Level 0 is matrix free: [K u]_v = sum over the 8 incident elements e of
// s_e K0[7 - e, :] u_e (Eq. st-assemb), S_v = sum_e s_e K0[7 - e, 7 - e]
// (Eq. st-assemb-gs), evaluated per vertex from the 27 neighbour values.
// Coarse levels read their stored 27-point stencils, six load cases per read.
//
// A forward sweep from zero ("fresh") knows which rows still hold zero: at
// pair k, rows of pairs > k and the old values of its own rows.  It skips
// their loads, so the first sweep needs no cleared buffer.
#include <algorithm>

#include "hmg_internal.hpp"

namespace hmg {
namespace {

constexpr int GS_THREADS = 256;
constexpr int GS_ITEMS0 = 1024;  // vertex pairs held in LDS per step, level 0 (one case)
constexpr int GS_ITEMSC = 256;   // coarse levels (six cases per item)

template <typename T>
__device__ __forceinline__ double to_d(T v) {
  return (double)(typename Acc<T>::type)v;
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ bool case_on(const double* scal, int c) {
  return scal == nullptr || scal[S_ACTIVE * 8 + c] != 0.0;
}

// Pair of the row at offset (dy, dz) from a row of pair k.
__device__ __forceinline__ int row_pair(int k, int dy, int dz) {
  return ((k & 1) ^ (dy != 0 ? 1 : 0)) + 2 * ((k >> 1) ^ (dz != 0 ? 1 : 0));
}

// Inverse of the symmetric block (xx, yy, zz, xy, yz, xz), same order out.
template <typename A>
__device__ __forceinline__ void sym3_inverse(const A (&S)[6], A (&D)[6]) {
  const A a = S[0], b = S[1], c = S[2], d = S[3], e = S[4], f = S[5];
  const A c00 = b * c - e * e, c01 = f * e - d * c, c02 = d * e - b * f;
  const A id = A(1) / (a * c00 + d * c01 + f * c02);
  D[0] = c00 * id;
  D[1] = (a * c - f * f) * id;
  D[2] = (a * b - d * d) * id;
  D[3] = c01 * id;
  D[4] = (d * f - a * e) * id;
  D[5] = c02 * id;
}

template <typename A>
__device__ __forceinline__ void block_apply(const A (&D)[6], A r0, A r1, A r2, A (&o)[3]) {
  o[0] = D[0] * r0 + D[3] * r1 + D[5] * r2;
  o[1] = D[3] * r0 + D[1] * r1 + D[4] * r2;
  o[2] = D[5] * r0 + D[4] * r1 + D[2] * r2;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ __forceinline__ double block_total(double v, double* lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < GS_THREADS / 64; ++i) s += lds[i];
  return s;
}

// ------------------------------------------------------------------ level 0
// The ten distinct magnitudes of K0 (see k0_sel); every loop below that
// touches K0 is unrolled, so each entry is one of these kernel-argument
// scalars with a constant sign.
template <typename T>
struct K0Vals {
  T v[10];
};

template <typename T>
__device__ __forceinline__ T k0e(const K0Vals<T>& kv, int a, int i, int b, int j) {
  const int sel = k0_sel(a, i, b, j);
  return (sel & 1) ? -kv.v[sel >> 1] : kv.v[sel >> 1];
}

// New value z_v + S_v^-1 ((r - m)_v - [K z]_v) at one vertex.  `plane(p, pl)`
// fills pl[(dx + 1) + 3 (dy + 1)][k] with z at offset (dx, dy, p - 1).  The
// incident element e = e0 + 2 e1 + 4 e2 has its origin at
// v + (e0 - 1, e1 - 1, e2 - 1), holds v as local node 7 - e and its node b at
// offset (e0 + b0 - 1, e1 + b1 - 1, e2 + b2 - 1); sv[e] is its scale.  The
// three neighbour planes are visited in turn, so only one is live.
template <typename T, class Plane>
__device__ __forceinline__ void gs0_vertex(const K0Vals<T>& kv, const T (&sv)[8], Plane&& plane,
                                           T r0, T r1, T r2, T (&out)[3]) {
  T w[8][3];
#pragma unroll
  for (int e = 0; e < 8; ++e) w[e][0] = w[e][1] = w[e][2] = T(0);
  T centre[3];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    T pl[9][3];
    plane(p, pl);
    if (p == 1)
#pragma unroll
      for (int k = 0; k < 3; ++k) centre[k] = pl[4][k];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int a = 7 - e, e0 = e & 1, e1 = (e >> 1) & 1, b2 = p - (e >> 2);
      if (b2 < 0 || b2 > 1) continue;
#pragma unroll
      for (int b01 = 0; b01 < 4; ++b01) {
        const int b = b01 + 4 * b2;
        const T* u = pl[(e0 + (b01 & 1)) + 3 * (e1 + (b01 >> 1))];
#pragma unroll
        for (int i = 0; i < 3; ++i)
          w[e][i] += k0e(kv, a, i, b, 0) * u[0] + k0e(kv, a, i, b, 1) * u[1] +
                     k0e(kv, a, i, b, 2) * u[2];
      }
    }
  }
  T y[3] = {T(0), T(0), T(0)};
  T S[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int a = 7 - e;
#pragma unroll
    for (int i = 0; i < 3; ++i) y[i] += sv[e] * w[e][i];
    S[0] += sv[e] * k0e(kv, a, 0, a, 0);
    S[1] += sv[e] * k0e(kv, a, 1, a, 1);
    S[2] += sv[e] * k0e(kv, a, 2, a, 2);
    S[3] += sv[e] * k0e(kv, a, 0, a, 1);
    S[4] += sv[e] * k0e(kv, a, 1, a, 2);
    S[5] += sv[e] * k0e(kv, a, 0, a, 2);
  }
  T D[6];
  sym3_inverse(S, D);
  T dz[3];
  block_apply(D, r0 - y[0], r1 - y[1], r2 - y[2], dz);
#pragma unroll
  for (int k = 0; k < 3; ++k) out[k] = centre[k] + dz[k];
}

// Pair k of one load case (blockIdx.y) on rows [blockIdx.x * rpb, ... + rpb).
// first: x parity relaxed first (0 in a forward sweep, 1 in a backward one).
// s the element scales, r the level's right-hand side, mean its per-component
// means (S_MEAN* slots, or null), z relaxed in place, q optional, scal the
// active cases (or null).  With dot set, the block partials of (r - m).z
// (S_RZNEW) and q.z (S_QZ) over the vertices it finishes go to column
// k * gridDim.x + blockIdx.x.
template <typename T>
__global__ void __launch_bounds__(GS_THREADS)
gs0_pair_kernel(Grid g, K0Vals<T> kv, const T* __restrict__ s, const T* __restrict__ r,
                const double* __restrict__ mean, T* __restrict__ z, const T* __restrict__ q,
                const double* __restrict__ scal, Partials part, int dot, int k, int first,
                int fresh, int rpb) {
  __shared__ T nw[GS_ITEMS0][3];
  __shared__ double red[GS_THREADS / 64];
  const int c = blockIdx.y;
  const int np = g.nx >> 1, hy = g.ny >> 1;
  const int rows = hy * (g.nz >> 1);
  const int rs = max(1, GS_ITEMS0 / np);
  const int rb0 = blockIdx.x * rpb, rb1 = min(rows, rb0 + rpb);
  const int64_t n = g.n;
  const bool on = case_on(scal, c);
  double acc_rz = 0.0, acc_qz = 0.0;
  if (on) {
    double m[3] = {0.0, 0.0, 0.0};
    if (mean)
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) m[kk] = mean[(S_MEAN0 + kk) * 8 + c];
    T* zc[3];
    const T* rc[3];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      zc[kk] = z + (int64_t)(c * 3 + kk) * n;
      rc[kk] = r + (int64_t)(c * 3 + kk) * n;
    }
    const int py = k & 1, pz = k >> 1;
    for (int rb = rb0; rb < rb1; rb += rs) {
      const int nitems = min(rs, rb1 - rb) * np;
#pragma unroll 1
      for (int step = 0; step < 2; ++step) {
        const int xpar = step == 0 ? first : 1 - first;
#pragma unroll 1
        for (int w = threadIdx.x; w < nitems; w += GS_THREADS) {
          const int j = rb + w / np, px = w % np;
          const int y = 2 * (j % hy) + py, zz = 2 * (j / hy) + pz;
          const int x = 2 * px + xpar;
          const int xs[3] = {x == 0 ? g.nx - 1 : x - 1, x, x + 1 == g.nx ? 0 : x + 1};
          // LDS items of the own-row neighbours (x - 1, x + 1) in the second step
          const int wl = w - px + (first == 0 ? px : (px == 0 ? np - 1 : px - 1));
          const int wr = w - px + (first == 0 ? (px + 1 == np ? 0 : px + 1) : px);
          auto plane = [&](int p, T(&pl)[9][3]) {
            const int dz = p - 1;
            const int zq = wrap(zz + dz, g.nz);
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
              const int yy = wrap(y + dy, g.ny);
              const int64_t rbase = (int64_t)g.nx * (yy + (int64_t)g.ny * zq);
              const bool own = dy == 0 && dz == 0;
              const bool zero = fresh && (own || row_pair(k, dy, dz) > k);
#pragma unroll
              for (int dx = 0; dx < 3; ++dx) {
                T* o = pl[dx + 3 * (dy + 1)];
                if (own && dx != 1 && step == 1) {
                  const int wi = dx == 0 ? wl : wr;
#pragma unroll
                  for (int kk = 0; kk < 3; ++kk) o[kk] = nw[wi][kk];
                } else if (zero) {
#pragma unroll
                  for (int kk = 0; kk < 3; ++kk) o[kk] = T(0);
                } else {
#pragma unroll
                  for (int kk = 0; kk < 3; ++kk) o[kk] = zc[kk][rbase + xs[dx]];
                }
              }
            }
          };
          T sv[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int ex = (e & 1) ? x : xs[0];
            const int ey = ((e >> 1) & 1) ? y : wrap(y - 1, g.ny);
            const int ez = (e >> 2) ? zz : wrap(zz - 1, g.nz);
            sv[e] = s[ex + (int64_t)g.nx * (ey + (int64_t)g.ny * ez)];
          }
          const int64_t v = x + (int64_t)g.nx * (y + (int64_t)g.ny * zz);
          const T r0 = (T)((double)rc[0][v] - m[0]);
          const T r1 = (T)((double)rc[1][v] - m[1]);
          const T r2 = (T)((double)rc[2][v] - m[2]);
          T out[3];
          gs0_vertex<T>(kv, sv, plane, r0, r1, r2, out);
#pragma unroll
          for (int kk = 0; kk < 3; ++kk) zc[kk][v] = out[kk];
          if (step == 0)
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) nw[w][kk] = out[kk];
          if (dot) {
            acc_rz += (double)r0 * (double)out[0] + (double)r1 * (double)out[1] +
                      (double)r2 * (double)out[2];
            if (q)
#pragma unroll
              for (int kk = 0; kk < 3; ++kk)
                acc_qz += (double)q[(int64_t)(c * 3 + kk) * n + v] * (double)out[kk];
          }
        }
        __syncthreads();
      }
    }
  }
  if (dot) {
    const int col = k * gridDim.x + blockIdx.x;
    const double t0 = block_total(acc_rz, red);
    if (threadIdx.x == 0) part.buf[(int64_t)(S_RZNEW * 8 + c) * part.stride + col] = t0;
    if (q) {
      const double t1 = block_total(acc_qz, red);
      if (threadIdx.x == 0) part.buf[(int64_t)(S_QZ * 8 + c) * part.stride + col] = t1;
    }
  }
}

// ------------------------------------------------------------- coarse levels
// Stored stencils st[((d*3 + p)*3 + q) * n + v] and block inverses
// dinv[t * n + v], t = (xx, yy, zz, xy, yz, xz) of S_v^-1 (undamped).  Rounded
// (bf16) stencils use the centre block implied by the row sum and apply the
// operator in difference form, as the other coarse kernels do.
template <typename V, typename W>
__global__ void __launch_bounds__(GS_THREADS)
gsc_pair_kernel(Grid g, const W* __restrict__ st, const W* __restrict__ dinv,
                const V* __restrict__ r, const double* __restrict__ mean, V* z,
                const double* __restrict__ scal, int k, int first, int fresh, int rpb) {
  using A = typename Acc<V>::type;
  constexpr bool kDiff = std::is_same<W, bf16>::value;
  __shared__ A nw[GS_ITEMSC][NCASE][3];
  bool on[NCASE];
#pragma unroll
  for (int c = 0; c < NCASE; ++c) on[c] = case_on(scal, c);
  const int np = g.nx >> 1, hy = g.ny >> 1;
  const int rows = hy * (g.nz >> 1);
  const int rs = max(1, GS_ITEMSC / np);
  const int rb0 = blockIdx.x * rpb, rb1 = min(rows, rb0 + rpb);
  const int n = (int)g.n;
  const int py = k & 1, pz = k >> 1;
  for (int rb = rb0; rb < rb1; rb += rs) {
    const int nitems = min(rs, rb1 - rb) * np;
#pragma unroll 1
    for (int step = 0; step < 2; ++step) {
      const int xpar = step == 0 ? first : 1 - first;
      const int w = threadIdx.x;
      if (w < nitems) {
        const int j = rb + w / np, px = w % np;
        const int y = 2 * (j % hy) + py, zz = 2 * (j / hy) + pz;
        const int x = 2 * px + xpar;
        const int v = x + g.nx * (y + g.ny * zz);
        const int xs[3] = {x == 0 ? g.nx - 1 : x - 1, x, x + 1 == g.nx ? 0 : x + 1};
        const int wl = w - px + (first == 0 ? px : (px == 0 ? np - 1 : px - 1));
        const int wr = w - px + (first == 0 ? (px + 1 == np ? 0 : px + 1) : px);
        A uc[NCASE][3];
#pragma unroll
        for (int c = 0; c < NCASE; ++c)
#pragma unroll
          for (int kk = 0; kk < 3; ++kk)
            uc[c][kk] = fresh ? A(0) : (A)z[(int64_t)(c * 3 + kk) * n + v];
        A acc[NCASE][3];
#pragma unroll
        for (int c = 0; c < NCASE; ++c) acc[c][0] = acc[c][1] = acc[c][2] = A(0);
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy) {
            const int yy = wrap(y + dy, g.ny), zq = wrap(zz + dz, g.nz);
            const int rbase = g.nx * (yy + g.ny * zq);
            const bool own = dy == 0 && dz == 0;
            const bool zero = fresh && (own || row_pair(k, dy, dz) > k);
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
              const int d = dx + 3 * (dy + 1) + 9 * (dz + 1);
              if (kDiff && d == 13) continue;
              const bool from_lds = own && dx != 1 && step == 1;
              if (zero && !from_lds && !(own && dx == 1 && !kDiff)) continue;
              A K[9];
#pragma unroll
              for (int t = 0; t < 9; ++t) K[t] = (A)st[(int64_t)(d * 9 + t) * n + v];
#pragma unroll
              for (int c = 0; c < NCASE; ++c) {
                A u[3];
                if (from_lds) {
                  const int wi = dx == 0 ? wl : wr;
#pragma unroll
                  for (int kk = 0; kk < 3; ++kk) u[kk] = nw[wi][c][kk];
                } else if (own && dx == 1) {
#pragma unroll
                  for (int kk = 0; kk < 3; ++kk) u[kk] = uc[c][kk];
                } else if (zero) {
#pragma unroll
                  for (int kk = 0; kk < 3; ++kk) u[kk] = A(0);
                } else {
#pragma unroll
                  for (int kk = 0; kk < 3; ++kk)
                    u[kk] = (A)z[(int64_t)(c * 3 + kk) * n + rbase + xs[dx]];
                }
                if (kDiff)
#pragma unroll
                  for (int kk = 0; kk < 3; ++kk) u[kk] -= uc[c][kk];
                acc[c][0] += K[0] * u[0] + K[1] * u[1] + K[2] * u[2];
                acc[c][1] += K[3] * u[0] + K[4] * u[1] + K[5] * u[2];
                acc[c][2] += K[6] * u[0] + K[7] * u[1] + K[8] * u[2];
              }
            }
          }
        A D[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) D[t] = (A)dinv[(int64_t)t * n + v];
#pragma unroll
        for (int c = 0; c < NCASE; ++c) {
          A res[3];
#pragma unroll
          for (int kk = 0; kk < 3; ++kk)
            res[kk] = (A)(to_d(r[(int64_t)(c * 3 + kk) * n + v]) -
                          (mean ? mean[(S_MEAN0 + kk) * 8 + c] : 0.0)) -
                      acc[c][kk];
          A dzv[3];
          block_apply(D, res[0], res[1], res[2], dzv);
#pragma unroll
          for (int kk = 0; kk < 3; ++kk) {
            const V nv = (V)(uc[c][kk] + dzv[kk]);
            if (on[c]) z[(int64_t)(c * 3 + kk) * n + v] = nv;
            if (step == 0) nw[w][c][kk] = (A)nv;
          }
        }
      }
      __syncthreads();
    }
  }
}

int gs_rows(const Grid& g) { return (g.ny / 2) * (g.nz / 2); }

// Rows per block: whole LDS steps, at most `cap` blocks per case.
int gs_rows_per_block(const Grid& g, int items, int cap) {
  const int np = g.nx / 2;
  const int rs = std::max(1, items / np);
  const int rows = gs_rows(g);
  const int steps = std::max(1, (rows + rs * cap - 1) / (rs * cap));
  return rs * steps;
}

}  // namespace

bool gs_supported(const Grid& g) {
  return g.nx % 2 == 0 && g.ny % 2 == 0 && g.nz % 2 == 0 && g.nx / 2 <= GS_ITEMS0 && g.nx >= 2;
}

int gs0_blocks_per_case(const Grid& g) {
  const int rpb = gs_rows_per_block(g, GS_ITEMS0, 1024);
  return (gs_rows(g) + rpb - 1) / rpb;
}

template <typename T>
void gs0_sweep(const Grid& g, const double* k0v, const T* s, const T* r, const double* mean, T* z,
               const T* q, const double* scal, Partials part, bool forward, bool fresh,
               int* nblk_out, hipStream_t st) {
  K0Vals<T> kv;
  for (int i = 0; i < 10; ++i) kv.v[i] = (T)k0v[i];
  const int rpb = gs_rows_per_block(g, GS_ITEMS0, 1024);
  const int nblk = (gs_rows(g) + rpb - 1) / rpb;
  for (int i = 0; i < 4; ++i) {
    const int k = forward ? i : 3 - i;
    hipLaunchKernelGGL(gs0_pair_kernel<T>, dim3(nblk, NCASE), dim3(GS_THREADS), 0, st, g, kv, s, r,
                       mean, z, q, scal, part, nblk_out ? 1 : 0, k, forward ? 0 : 1,
                       (forward && fresh) ? 1 : 0, rpb);
  }
  if (nblk_out) *nblk_out = 4 * nblk;
}

template <typename V, typename W>
void gsc_sweep(const Grid& g, const W* stc, const W* dinv, const V* r, const double* mean, V* z,
               const double* scal, bool forward, bool fresh, hipStream_t st) {
  const int rpb = gs_rows_per_block(g, GS_ITEMSC, 2048);
  const int nblk = (gs_rows(g) + rpb - 1) / rpb;
  for (int i = 0; i < 4; ++i) {
    const int k = forward ? i : 3 - i;
    hipLaunchKernelGGL((gsc_pair_kernel<V, W>), dim3(nblk), dim3(GS_THREADS), 0, st, g, stc, dinv,
                       r, mean, z, scal, k, forward ? 0 : 1, (forward && fresh) ? 1 : 0, rpb);
  }
}

template void gs0_sweep<float>(const Grid&, const double*, const float*, const float*,
                               const double*, float*, const float*, const double*, Partials, bool,
                               bool, int*, hipStream_t);
template void gs0_sweep<double>(const Grid&, const double*, const double*, const double*,
                                const double*, double*, const double*, const double*, Partials,
                                bool, bool, int*, hipStream_t);
template void gsc_sweep<float, float>(const Grid&, const float*, const float*, const float*,
                                      const double*, float*, const double*, bool, bool,
                                      hipStream_t);
template void gsc_sweep<double, double>(const Grid&, const double*, const double*, const double*,
                                        const double*, double*, const double*, bool, bool,
                                        hipStream_t);
template void gsc_sweep<bf16, float>(const Grid&, const float*, const float*, const bf16*,
                                     const double*, bf16*, const double*, bool, bool, hipStream_t);
template void gsc_sweep<bf16, bf16>(const Grid&, const bf16*, const bf16*, const bf16*,
                                    const double*, bf16*, const double*, bool, bool, hipStream_t);

}  // namespace hmg

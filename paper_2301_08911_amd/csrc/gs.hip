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
#include <type_traits>
#include <utility>

#include "hmg_internal.hpp"

namespace hmg {
namespace {

constexpr int GS_THREADS = 256;
constexpr int GS_ITEMSC = 256;   // vertex pairs per LDS step (one per thread, six cases each)

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

// Offset visited i-th: each neighbour row (dy, dz) in turn, its centre column
// dx = 1 first, then dx = 0 and dx = 2 (d = dx + 3 (dy + 1) + 9 (dz + 1)).
__host__ __device__ constexpr int row_centre_first(int i) {
  return 3 * (i / 3) + (i % 3 == 0 ? 1 : (i % 3 == 1 ? 0 : 2));
}

template <class F, int... I>
__device__ __forceinline__ void static_for27_impl(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, row_centre_first(I)>{}), ...);
}
// f(std::integral_constant<int, d>) for the 27 offsets d, row by row, the
// centre column of each row first.
template <class F>
__device__ __forceinline__ void static_for27(F& f) {
  static_for27_impl(f, std::make_integer_sequence<int, 27>{});
}

template <typename T>
struct alignas(2 * sizeof(T)) VPair {
  T a, b;
};

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

// Block (blockIdx.x, blockIdx.y) -> (row block bx, load case c).  Workgroups go
// to the 8 XCDs round robin; consecutive logical blocks are gathered on one
// XCD, so the row blocks of neighbouring z-planes, which read each other's
// neighbour rows, share that XCD's L2.
__device__ __forceinline__ void xcd_block(int& c, int& bx) {
  const int nbx = gridDim.x;
  const int tot = nbx * gridDim.y;
  const int lin = blockIdx.x + nbx * blockIdx.y;
  const int q = tot >> 3, rem = tot & 7, xcd = lin & 7;
  const int logical = xcd * q + (xcd < rem ? xcd : rem) + (lin >> 3);
  c = logical / nbx;
  bx = logical - c * nbx;
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

// ------------------------------------------------------- six cases per thread
// Stencil sources of the generic pair kernel below.  block<d>() gives the 3x3
// coefficient block of row v towards neighbour v + d (d = dx + 3 dy + 9 dz
// with offsets in 0..2), inv() the inverse of the diagonal block S_v.

// Level 0, matrix free (Eq. st-assemb): the block towards offset d collects
// s_e K0[7 - e, b] over the incident elements e that hold v + d as their node
// b (1, 2, 4 or 8 of them); it is formed once and applied to all six cases.
template <typename T>
struct SrcLevel0 {
  static constexpr bool kDiff = false;
  K0Vals<T> kv;
  const T* __restrict__ s;
  Grid g;
  struct Loc {
    T sv[8];
  };
  __device__ __forceinline__ void load(int x, int y, int zz, int64_t, Loc& L) const {
    const int xm = x == 0 ? g.nx - 1 : x - 1;
    const int ym = wrap(y - 1, g.ny), zm = wrap(zz - 1, g.nz);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int ex = (e & 1) ? x : xm, ey = ((e >> 1) & 1) ? y : ym, ez = (e >> 2) ? zz : zm;
      L.sv[e] = s[ex + (int64_t)g.nx * (ey + (int64_t)g.ny * ez)];
    }
  }
  template <int D>
  __device__ __forceinline__ void block(const Loc& L, T (&K)[9]) const {
    constexpr int d0 = D % 3, d1 = (D / 3) % 3, d2 = D / 9;
#pragma unroll
    for (int t = 0; t < 9; ++t) K[t] = T(0);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int b0 = d0 - (e & 1), b1 = d1 - ((e >> 1) & 1), b2 = d2 - (e >> 2);
      if (b0 < 0 || b0 > 1 || b1 < 0 || b1 > 1 || b2 < 0 || b2 > 1) continue;
      const int a = 7 - e, b = b0 + 2 * b1 + 4 * b2;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) K[i * 3 + j] += L.sv[e] * k0e(kv, a, i, b, j);
    }
  }
  __device__ __forceinline__ void inv(const Loc&, const T (&Kc)[9], int64_t, T (&D)[6]) const {
    const T S[6] = {Kc[0], Kc[4], Kc[8], Kc[1], Kc[5], Kc[2]};
    sym3_inverse(S, D);
  }
};

// Coarse levels: stored stencils st[((d*3 + p)*3 + q) * n + v] and block
// inverses dinv[t * n + v], t = (xx, yy, zz, xy, yz, xz) of S_v^-1.  Rounded
// (bf16) stencils use the centre block implied by the row sum and apply the
// operator in difference form, as the other coarse kernels do.
template <typename W>
struct SrcStored {
  static constexpr bool kDiff = std::is_same<W, bf16>::value;
  const W* __restrict__ st;
  const W* __restrict__ dinv;
  int64_t n;
  struct Loc {
    int64_t v;
  };
  __device__ __forceinline__ void load(int, int, int, int64_t v, Loc& L) const { L.v = v; }
  template <int D, typename A>
  __device__ __forceinline__ void block(const Loc& L, A (&K)[9]) const {
#pragma unroll
    for (int t = 0; t < 9; ++t) K[t] = (A)st[(int64_t)(D * 9 + t) * n + L.v];
  }
  template <typename A>
  __device__ __forceinline__ void inv(const Loc& L, const A (&)[9], int64_t, A (&D)[6]) const {
#pragma unroll
    for (int t = 0; t < 6; ++t) D[t] = (A)dinv[(int64_t)t * n + L.v];
  }
};

// One colour pair (rows of pair k) of all six load cases: a thread per vertex
// pair, the first x parity, an LDS barrier, then the second.  With `dot`, the
// block partials of (r - m).z (S_RZNEW) and q.z (S_QZ) of the finished rows
// go to column k * gridDim.x + bx of `part`.
template <typename V, class Src, int first>
__global__ void __launch_bounds__(GS_THREADS)
gs_pair_kernel(Grid g, Src src, const V* __restrict__ r, const double* __restrict__ mean,
               V* __restrict__ z, const V* __restrict__ q, const double* __restrict__ scal,
               Partials part, int dot, int k, int fresh, int rpb) {
  using A = typename Acc<V>::type;
  constexpr bool kDiff = Src::kDiff;
  __shared__ A nw[GS_ITEMSC][NCASE][3];
  __shared__ double red[GS_THREADS / 64];
  bool on[NCASE];
#pragma unroll
  for (int c = 0; c < NCASE; ++c) on[c] = case_on(scal, c);
  const int np = g.nx >> 1, hy = g.ny >> 1;
  const int rows = hy * (g.nz >> 1);
  const int rs = max(1, GS_ITEMSC / np);
  int c0, bx;
  xcd_block(c0, bx);
  const int rb0 = bx * rpb, rb1 = min(rows, rb0 + rpb);
  const int64_t n = g.n;
  const int py = k & 1, pz = k >> 1;
  double acc_rz[NCASE], acc_qz[NCASE];
#pragma unroll
  for (int c = 0; c < NCASE; ++c) acc_rz[c] = acc_qz[c] = 0.0;
  for (int rb = rb0; rb < rb1; rb += rs) {
    const int nitems = min(rs, rb1 - rb) * np;
    // both steps unrolled: the x parity is a compile-time constant in each
#pragma unroll
    for (int step = 0; step < 2; ++step) {
      const int xpar = step == 0 ? first : 1 - first;
      const int w = threadIdx.x;
      if (w < nitems) {
        const int j = rb + w / np, px = w % np;
        const int y = 2 * (j % hy) + py, zz = 2 * (j / hy) + pz;
        const int x = 2 * px + xpar;
        const int64_t v = x + (int64_t)g.nx * (y + (int64_t)g.ny * zz);
        const int xs[3] = {x == 0 ? g.nx - 1 : x - 1, x, x + 1 == g.nx ? 0 : x + 1};
        // LDS items of the own-row neighbours (x - 1, x + 1) in the second step
        const int wl = w - px + (first == 0 ? px : (px == 0 ? np - 1 : px - 1));
        const int wr = w - px + (first == 0 ? (px + 1 == np ? 0 : px + 1) : px);
        typename Src::Loc loc;
        src.load(x, y, zz, v, loc);
        A uc[NCASE][3];
#pragma unroll
        for (int c = 0; c < NCASE; ++c)
#pragma unroll
          for (int kk = 0; kk < 3; ++kk)
            uc[c][kk] = fresh ? A(0) : (A)z[(int64_t)(c * 3 + kk) * n + v];
        A acc[NCASE][3];
#pragma unroll
        for (int c = 0; c < NCASE; ++c) acc[c][0] = acc[c][1] = acc[c][2] = A(0);
        A Kc[9];
        // In a neighbour row (not the own row) the centre column is read as
        // the aligned pair (x - xpar, x - xpar + 1), which also holds the
        // column on the other side of x from the pair's start: x + 1 for an
        // even x, x - 1 for an odd one.  That value is kept for the row's next
        // offset, and only the remaining column is a single load: two loads
        // per row and component instead of three.
        A kept[NCASE][3];
        const int pb = x - xpar;
        // the 27 offsets; d is a compile-time constant in every iteration
        auto visit = [&](auto dconst) {
          constexpr int d = decltype(dconst)::value;
          constexpr int dx = d % 3, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
          constexpr bool own = dy == 0 && dz == 0;
          if (kDiff && d == 13) return;
          const bool from_lds = own && dx != 1 && step == 1;
          const bool zero = fresh && (own || row_pair(k, dy, dz) > k);
          A K[9];
          src.template block<d>(loc, K);
          if (d == 13)
#pragma unroll
            for (int t = 0; t < 9; ++t) Kc[t] = K[t];
          if (zero && !from_lds && !(own && dx == 1)) return;
          const int64_t rbase =
              (int64_t)g.nx * (wrap(y + dy, g.ny) + (int64_t)g.ny * wrap(zz + dz, g.nz));
          // the kept pair half is the x - 1 column for an odd x, x + 1 for an even x
          const bool use_kept = !own && dx != 1 && (dx == 0) == (xpar == 1);
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
            } else if (!own && dx == 1) {
#pragma unroll
              for (int kk = 0; kk < 3; ++kk) {
                const VPair<V> pr =
                    *reinterpret_cast<const VPair<V>*>(z + (int64_t)(c * 3 + kk) * n + rbase + pb);
                u[kk] = (A)(xpar ? pr.b : pr.a);
                kept[c][kk] = (A)(xpar ? pr.a : pr.b);
              }
            } else if (use_kept) {
#pragma unroll
              for (int kk = 0; kk < 3; ++kk) u[kk] = kept[c][kk];
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
        };
        static_for27(visit);
        A D[6];
        src.inv(loc, Kc, v, D);
#pragma unroll
        for (int c = 0; c < NCASE; ++c) {
          A rv[3], res[3];
#pragma unroll
          for (int kk = 0; kk < 3; ++kk) {
            rv[kk] = (A)(to_d(r[(int64_t)(c * 3 + kk) * n + v]) -
                         (mean ? mean[(S_MEAN0 + kk) * 8 + c] : 0.0));
            res[kk] = rv[kk] - acc[c][kk];
          }
          A dzv[3];
          block_apply(D, res[0], res[1], res[2], dzv);
#pragma unroll
          for (int kk = 0; kk < 3; ++kk) {
            const V nv = (V)(uc[c][kk] + dzv[kk]);
            if (on[c]) z[(int64_t)(c * 3 + kk) * n + v] = nv;
            if (step == 0) nw[w][c][kk] = (A)nv;
            if (dot) {
              acc_rz[c] += (double)rv[kk] * (double)(A)nv;
              if (q) acc_qz[c] += (double)(A)q[(int64_t)(c * 3 + kk) * n + v] * (double)(A)nv;
            }
          }
        }
      }
      __syncthreads();
    }
  }
  if (dot) {
    const int col = k * gridDim.x + bx;
#pragma unroll
    for (int c = 0; c < NCASE; ++c) {
      const double t0 = block_total(acc_rz[c], red);
      if (threadIdx.x == 0) part.buf[(int64_t)(S_RZNEW * 8 + c) * part.stride + col] = t0;
      if (q) {
        const double t1 = block_total(acc_qz[c], red);
        if (threadIdx.x == 0) part.buf[(int64_t)(S_QZ * 8 + c) * part.stride + col] = t1;
      }
    }
  }
}

int gs_rows(const Grid& g) { return (g.ny / 2) * (g.nz / 2); }

// Rows per block: whole LDS steps, at most `cap` blocks.
int gs_rows_per_block(const Grid& g, int items, int cap) {
  const int np = g.nx / 2;
  const int rs = std::max(1, items / np);
  const int rows = gs_rows(g);
  const int steps = std::max(1, (rows + rs * cap - 1) / (rs * cap));
  return rs * steps;
}

constexpr int GS_BLOCK_CAP = 4096;

}  // namespace

bool gs_supported(const Grid& g) {
  return g.nx % 2 == 0 && g.ny % 2 == 0 && g.nz % 2 == 0 && g.nx / 2 <= GS_ITEMSC && g.nx >= 2;
}

int gs0_blocks_per_case(const Grid& g) {
  const int rpb = gs_rows_per_block(g, GS_ITEMSC, GS_BLOCK_CAP);
  return (gs_rows(g) + rpb - 1) / rpb;
}

template <typename T>
void gs0_sweep(const Grid& g, const double* k0v, const T* s, const T* r, const double* mean, T* z,
               const T* q, const double* scal, Partials part, bool forward, bool fresh,
               int* nblk_out, hipStream_t st) {
  SrcLevel0<T> src;
  for (int i = 0; i < 10; ++i) src.kv.v[i] = (T)k0v[i];
  src.s = s;
  src.g = g;
  const int rpb = gs_rows_per_block(g, GS_ITEMSC, GS_BLOCK_CAP);
  const int nblk = (gs_rows(g) + rpb - 1) / rpb;
  for (int i = 0; i < 4; ++i) {
    const int k = forward ? i : 3 - i;
    if (forward)
      hipLaunchKernelGGL((gs_pair_kernel<T, SrcLevel0<T>, 0>), dim3(nblk), dim3(GS_THREADS), 0, st,
                         g, src, r, mean, z, q, scal, part, nblk_out ? 1 : 0, k, fresh ? 1 : 0,
                         rpb);
    else
      hipLaunchKernelGGL((gs_pair_kernel<T, SrcLevel0<T>, 1>), dim3(nblk), dim3(GS_THREADS), 0, st,
                         g, src, r, mean, z, q, scal, part, nblk_out ? 1 : 0, k, 0, rpb);
  }
  if (nblk_out) *nblk_out = 4 * nblk;
}

template <typename V, typename W>
void gsc_sweep(const Grid& g, const W* stc, const W* dinv, const V* r, const double* mean, V* z,
               const double* scal, bool forward, bool fresh, hipStream_t st) {
  const SrcStored<W> src{stc, dinv, g.n};
  const int rpb = gs_rows_per_block(g, GS_ITEMSC, GS_BLOCK_CAP);
  const int nblk = (gs_rows(g) + rpb - 1) / rpb;
  for (int i = 0; i < 4; ++i) {
    const int k = forward ? i : 3 - i;
    if (forward)
      hipLaunchKernelGGL((gs_pair_kernel<V, SrcStored<W>, 0>), dim3(nblk), dim3(GS_THREADS), 0, st,
                         g, src, r, mean, z, (const V*)nullptr, scal, Partials{}, 0, k,
                         fresh ? 1 : 0, rpb);
    else
      hipLaunchKernelGGL((gs_pair_kernel<V, SrcStored<W>, 1>), dim3(nblk), dim3(GS_THREADS), 0, st,
                         g, src, r, mean, z, (const V*)nullptr, scal, Partials{}, 0, k, 0, rpb);
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

// Level-0 (finest grid) kernels: the matrix-free SIMP-weighted stiffness
// operator and everything fused around it.
//
// Operator (Sec. 4.2, Eq. st-assemb):  [K u]_v = sum_{e ∋ v} s_e K0[loc_e(v), :] u_e.
// The paper evaluates it vertex by vertex with one warp per incident element;
// here it is evaluated element by element in the Walsh-Hadamard mode basis of
// the 8 nodal values, where K0 has 45 nonzeros instead of 576:
//   u_hat = H u_e (separable butterflies), w_hat = s_e Kt u_hat, y_e = H w_hat.
// A workgroup owns a tile of 63 x 15 (FP64: 63 x 7) vertex columns and marches
// along z.  The vertex plane (tile plus a one-vertex halo) is staged in LDS; each thread owns
// one element column, forms the x/y butterflies from LDS and the z butterfly
// in registers against the previous plane, and keeps the z-half of its output
// that belongs to the next vertex plane in registers.  Lanes run along x, so
// the x-neighbour part of the vertex gather is a cross-lane move (DPP); only
// the y-neighbour part goes through LDS.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "hmg_internal.hpp"

namespace hmg {
namespace {

// Tile of a level-0 pass: TXE element columns (one wavefront) by TYE element
// rows (one wavefront each).  Every element of a tile is computed, but only
// the vertices whose eight elements all lie in it are owned, so taller tiles
// recompute and re-fetch less of their halo: FP32 passes use 16 rows (1024
// threads), FP64 passes 8 (their register budget allows no more waves).
template <typename T>
struct TileShape {
  static constexpr int TXE = 64;
  static constexpr int TYE = sizeof(T) == 4 ? 16 : 8;
  static constexpr int OX = TXE - 1, OY = TYE - 1;  // owned vertex columns per tile
  static constexpr int PX = TXE + 1, PY = TYE + 1;  // staged vertex plane
  static constexpr int NTHR = TXE * TYE;
  static constexpr int NVTX = PY * PX;                    // vertices of a staged plane
  static constexpr int NSLOT = (NVTX + NTHR - 1) / NTHR;  // plane vertices per thread
};

struct TileGeom {
  int ntx, nty, nzc, lz, ntiles;
};

__host__ __device__ inline int modp(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

template <typename T>
TileGeom tile_geom(const Grid& g, int lz_req = 0) {
  using S = TileShape<T>;
  TileGeom t;
  t.ntx = (g.nx + S::OX - 1) / S::OX;
  t.nty = (g.ny + S::OY - 1) / S::OY;
  const int base = t.ntx * t.nty * NCASE;
  int lz = g.nz;
  if (lz_req > 0)
    lz = lz_req < g.nz ? lz_req : g.nz;
  else
    // about 80 blocks per CU: short z-chunks cost halo planes but keep the
    // blocks of a wave of the grid close together (at 512^3, 32-plane chunks
    // and 30240 blocks ran faster than 16 or 64 planes)
    while (lz > 16 && base * ((g.nz + lz - 1) / lz) < 20480) lz = (lz + 1) / 2;
  t.lz = lz;
  t.nzc = (g.nz + lz - 1) / lz;
  t.ntiles = t.ntx * t.nty * t.nzc;
  return t;
}

// Vertex `xy` of the plane that starts at base + off.  `base + off` is the same
// for the whole workgroup, so it goes into a buffer resource (scalar registers)
// and only the 32-bit byte offset of `xy` is per thread (nx*ny*8 < 2^31 is
// checked on the host).  The range field also turns any offset past 2^31
// bytes into a dropped access instead of a stray one.
typedef unsigned int u32x2 __attribute__((__vector_size__(8)));

template <typename P>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const P* base, int64_t off) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)(base + off), (short)0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ float ld(const float* base, int64_t off, uint32_t xy) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_raw_buffer_load_b32(plane_rsrc(base, off), xy * 4u, 0, 0));
}
__device__ __forceinline__ double ld(const double* base, int64_t off, uint32_t xy) {
  return __builtin_bit_cast(double,
                            __builtin_amdgcn_raw_buffer_load_b64(plane_rsrc(base, off), xy * 8u, 0, 0));
}
__device__ __forceinline__ bf16 ld(const bf16* base, int64_t off, uint32_t xy) {
  return __builtin_bit_cast(
      bf16, (unsigned short)__builtin_amdgcn_raw_buffer_load_b16(plane_rsrc(base, off), xy * 2u, 0, 0));
}
__device__ __forceinline__ void st(bf16* base, int64_t off, uint32_t xy, bf16 v) {
  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v),
                                        plane_rsrc(base, off), xy * 2u, 0, 0);
}
__device__ __forceinline__ void st(float* base, int64_t off, uint32_t xy, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), plane_rsrc(base, off),
                                        xy * 4u, 0, 0);
}
__device__ __forceinline__ void st(double* base, int64_t off, uint32_t xy, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), plane_rsrc(base, off),
                                        xy * 8u, 0, 0);
}

// Value of lane (l - 1) of the wavefront (DPP wave_shr:1); lane 0 receives 0.
__device__ __forceinline__ float from_left(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_left(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x138, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// o[m0 + 2 m1] = sum_{b0,b1} (-1)^(m0 b0 + m1 b1) u[b0 + 2 b1]; self-inverse up to 4.
template <typename T>
__device__ __forceinline__ void bfly4(T u0, T u1, T u2, T u3, T& o0, T& o1, T& o2, T& o3) {
  const T s0 = u0 + u1, d0 = u0 - u1, s1 = u2 + u3, d1 = u2 - u3;
  o0 = s0 + s1;
  o1 = d0 + d1;
  o2 = s0 - s1;
  o3 = d0 - d1;
}

// w_hat = s * Kt * u_hat with the block pattern documented in ModeK.
template <typename T>
__device__ __forceinline__ void mode_apply(const ModeK<T>& K, T s, const T (&uh)[8][3],
                                           T (&wh)[8][3]) {
  const T sab = s * K.ab, sb = s * K.b, scs = s * K.cs, sp = s * K.p, sq = s * K.q;
  const T sfg = s * K.fg, sg = s * K.g, sz = s * K.z;
  const T sn = sb * (uh[1][0] + uh[2][1] + uh[4][2]);
  wh[1][0] = sab * uh[1][0] + sn;
  wh[2][1] = sab * uh[2][1] + sn;
  wh[4][2] = sab * uh[4][2] + sn;
  T t = scs * (uh[1][1] + uh[2][0]);
  wh[1][1] = t;
  wh[2][0] = t;
  t = scs * (uh[1][2] + uh[4][0]);
  wh[1][2] = t;
  wh[4][0] = t;
  t = scs * (uh[2][2] + uh[4][1]);
  wh[2][2] = t;
  wh[4][1] = t;
  wh[3][0] = sp * uh[3][0] + sq * uh[6][2];
  wh[6][2] = sq * uh[3][0] + sp * uh[6][2];
  wh[3][1] = sp * uh[3][1] + sq * uh[5][2];
  wh[5][2] = sq * uh[3][1] + sp * uh[5][2];
  wh[5][0] = sp * uh[5][0] + sq * uh[6][1];
  wh[6][1] = sq * uh[5][0] + sp * uh[6][1];
  const T st = sg * (uh[3][2] + uh[5][1] + uh[6][0]);
  wh[3][2] = sfg * uh[3][2] + st;
  wh[5][1] = sfg * uh[5][1] + st;
  wh[6][0] = sfg * uh[6][0] + st;
  wh[7][0] = sz * uh[7][0];
  wh[7][1] = sz * uh[7][1];
  wh[7][2] = sz * uh[7][2];
  wh[0][0] = wh[0][1] = wh[0][2] = T(0);
}

// Workgroup barrier that waits only for this wave's LDS traffic, so global loads
// issued for the next plane stay in flight across it (the plain barrier also
// drains outstanding global memory operations).
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum over the block in a fixed order; result valid in thread 0.
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

// Block index -> work item.  Workgroups are dispatched to the 8 XCDs round
// robin, so consecutive logical indices are gathered on one XCD, where they
// run in index order (one block per CU at a time).
__device__ __forceinline__ int logical_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  const int q = nb >> 3, r = nb & 7, xcd = b & 7;
  return xcd * q + (xcd < r ? xcd : r) + (b >> 3);
}

// Work item -> (load case, tile).  Consecutive items take a group of G load
// cases over a whole row of x-tiles, then the next group of the same row: the
// blocks resident on an XCD at one time then cover every x-tile of a row, so
// the 128-byte lines at the tile boundaries (a staged row of 65 values spans
// three of them) are fetched once for both neighbours, and a group's cases
// share s.  Measured at 512^3 against six cases per tile with x-tiles in turn:
// G = 2 took the FP32 matvec / residual / post-smooth from 13.8 / 9.1 / 10.8 to
// 12.1 / 8.0 / 10.3 ms (matvec reads 36.6 -> 31.9 GB); the FP64 residual (63 x 7
// tiles) is fastest with G = 3 (14.4 -> 11.4 ms).
template <typename T>
__device__ __forceinline__ void item_tile(int j, int ntx, int& c, int& tile) {
  constexpr int G = sizeof(T) == 8 ? 3 : 2;
  constexpr int NG = NCASE / G;
  static_assert(NG * G == NCASE, "case groups must tile the load cases");
  const int r = j / G;
  const int q = r / ntx;  // NG * (tile row) + group
  c = j % G + G * (q % NG);
  tile = r % ntx + ntx * (q / NG);
}

template <int V>
using Par = std::integral_constant<int, V>;

// Ops that declare DIAG = true receive, at each owned vertex, the four numbers
// that fix the vertex's diagonal block sum_e s_e K0[a_e, a_e] (Sec. 4.2): with
// the eight elements e at offsets d in {-1, 0}^3 and the sign t_i = +1 for
// d_i = -1, -1 for d_i = 0, the block is dd * S on the diagonal and
// oo * M_ij off it, where S = sum s_e and M_ij = sum s_e t_i t_j (the sign
// pattern of K0's diagonal blocks under the cube's reflections).  They arrive
// as dg = {S, M_xy, M_yz, M_xz}.
template <class Op, class = void>
struct OpDiag : std::false_type {};
template <class Op>
struct OpDiag<Op, std::void_t<decltype(Op::DIAG)>> : std::bool_constant<Op::DIAG> {};

// omega (dd S I + oo M)^-1 for the modes dg = {S, M_xy, M_yz, M_xz} (OpDiag),
// by cofactors over the determinant, as d = {xx, yy, zz, xy, yz, xz}.  In FP32
// the determinant is inverted by the hardware reciprocal (1 ulp), which a
// smoother tolerates; FP64 divides.
template <typename T>
__device__ __forceinline__ void damped_block_inverse(T dd, T oo, T omega, const T (&dg)[4],
                                                     T (&d)[6]) {
  const T d0 = dd * dg[0];
  const T d01 = oo * dg[1], d12 = oo * dg[2], d02 = oo * dg[3];
  const T c00 = d0 * d0 - d12 * d12, c11 = d0 * d0 - d02 * d02, c22 = d0 * d0 - d01 * d01;
  const T c01 = d02 * d12 - d01 * d0, c12 = d01 * d02 - d0 * d12, c02 = d01 * d12 - d02 * d0;
  const T det = d0 * c00 + d01 * c01 + d02 * c02;
  T f;
  if constexpr (sizeof(T) == 4)
    f = omega * __builtin_amdgcn_rcpf(det);
  else
    f = omega / det;
  d[0] = f * c00;
  d[1] = f * c11;
  d[2] = f * c22;
  d[3] = f * c01;
  d[4] = f * c12;
  d[5] = f * c02;
}

// 2x2 modes {sum, x, y, xy} of one element plane at a vertex, from the x-pair
// sum a and difference b of element row y - 1 (au, bu; t_y = +1) and row y
// (t_y = -1); each pair is s(x - 1) +- s(x), t_x = +1 for x - 1.
template <typename T>
__device__ __forceinline__ void plane_modes2(T au, T bu, T a, T b, T (&dm)[4]) {
  dm[0] = au + a;
  dm[1] = bu + b;
  dm[2] = au - a;
  dm[3] = bu - b;
}

// Vertex modes from the plane modes of element planes z - 1 (t_z = +1) and z.
template <typename T>
__device__ __forceinline__ void vertex_modes(const T (&lo)[4], const T (&hi)[4], T (&dg)[4]) {
  dg[0] = lo[0] + hi[0];
  dg[1] = lo[3] + hi[3];
  dg[2] = lo[2] - hi[2];
  dg[3] = lo[1] - hi[1];
}

// Occupancy target of the level-0 kernels (waves per SIMD), which bounds their
// register budget: 512 / waves VGPRs.
#ifndef HMG_OP0_WAVES
#define HMG_OP0_WAVES 4
#endif
template <typename T>
struct Op0Waves {
  static constexpr int value = sizeof(T) == 4 ? HMG_OP0_WAVES : 2;
};

// One work item of a level-0 pass: one load case of one tile of one cell
// (item_tile).
template <typename T, class Op>
__device__ __forceinline__ void op0_body(const Op& op_in, const Grid& g, const TileGeom& tg,
                                         const ModeK<T>& mk, const T* __restrict__ s, int j) {
  using S = TileShape<T>;
  __shared__ T plane[2][3][S::PY][S::PX];
  __shared__ T rowc[2][3][S::TYE][S::TXE];
  __shared__ double red[S::NTHR / 64];
  // Diagonal modes (OpDiag): the x-pair sum and difference of s in each element
  // row, handed to the row above.
  constexpr bool DIAG = OpDiag<Op>::value;
  __shared__ T sab[2][2][DIAG ? S::TYE : 1][DIAG ? S::TXE : 1];

  int c, tile;
  item_tile<T>(j, tg.ntx, c, tile);
  if (!op_in.active(c)) return;
  // Per-case scalars are read once, before any store of the kernel could be
  // taken to alias them.
  Op op = op_in;
  op.prep(c);
  const int tx = tile % tg.ntx;
  const int rem = tile / tg.ntx;
  const int ty = rem % tg.nty;
  const int zc = rem / tg.nty;
  const int x0 = tx * S::OX, y0 = ty * S::OY;
  const int z0 = zc * tg.lz;
  const int z1 = min(z0 + tg.lz, g.nz);
  const int tid = threadIdx.x, lx = tid & (S::TXE - 1), ly = tid / S::TXE;
  const int64_t nxy = (int64_t)g.nx * g.ny;

  // Plane-load slots of this thread (same vertices of every plane); each slot
  // produces the three components of one vertex.
  uint32_t ld_xy[S::NSLOT];
  int ld_pos[S::NSLOT], ld_gx[S::NSLOT], ld_gy[S::NSLOT];
  bool ld_own[S::NSLOT], ld_ok[S::NSLOT];
#pragma unroll
  for (int sl = 0; sl < S::NSLOT; ++sl) {
    const int i = tid + sl * S::NTHR;
    const int ii = i < S::NVTX ? i : 0;
    const int py = ii / S::PX, px = ii - py * S::PX;
    const int ux = x0 - 1 + px, uy = y0 - 1 + py;
    // A tile at the high x or y end of the grid needs its staged plane only up
    // to the one-vertex halo (which wraps to 0); beyond it the plane would hold
    // copies of the grid's first columns or rows, which no owned vertex uses.
    ld_ok[sl] = i < S::NVTX && ux <= g.nx && uy <= g.ny;
    ld_gx[sl] = modp(ux, g.nx);
    ld_gy[sl] = modp(uy, g.ny);
    ld_xy[sl] = (uint32_t)ld_gx[sl] + (uint32_t)g.nx * (uint32_t)ld_gy[sl];
    ld_pos[sl] = ii;
    ld_own[sl] = px >= 1 && px <= S::OX && py >= 1 && py <= S::OY && ux < g.nx && uy < g.ny;
  }
  const int ex = modp(x0 - 1 + lx, g.nx), ey = modp(y0 - 1 + ly, g.ny);
  const uint32_t exy = (uint32_t)ex + (uint32_t)g.nx * (uint32_t)ey;
  const bool outv = lx >= 1 && ly >= 1 && (x0 - 1 + lx) < g.nx && (y0 - 1 + ly) < g.ny;

  // Global loads of a plane are issued two planes ahead into one of two raw
  // register sets (fetch); the op's arithmetic and its owned-vertex side writes
  // run when the plane is staged into LDS (stage), so the loads of two planes
  // are in flight behind the compute of one.
  typename Op::Raw raw0[S::NSLOT], raw1[S::NSLOT];
  auto fetch_plane = [&](int zu, typename Op::Raw(&raw)[S::NSLOT]) {
    const int64_t zoff = nxy * modp(zu, g.nz);
    const bool ownz = zu >= z0 && zu < z1;
#pragma unroll
    for (int sl = 0; sl < S::NSLOT; ++sl)
      if (ld_ok[sl]) op.fetch(c, zoff, ld_xy[sl], ld_own[sl] && ownz, raw[sl]);
  };
  auto stage_plane = [&](int buf, int zu, const typename Op::Raw(&raw)[S::NSLOT]) {
    const int gz = modp(zu, g.nz);
    const bool ownz = zu >= z0 && zu < z1;
    const int64_t zoff = nxy * gz;
    T* base = &plane[buf][0][0][0];
#pragma unroll
    for (int sl = 0; sl < S::NSLOT; ++sl)
      if (ld_ok[sl]) {
        T v[3];
        op.finish(c, zoff, ld_xy[sl], ld_gx[sl], ld_gy[sl], gz, ld_own[sl] && ownz, raw[sl], v);
#pragma unroll
        for (int k = 0; k < 3; ++k) base[k * S::NVTX + ld_pos[sl]] = v[k];
      }
  };
  auto plane_modes = [&](int buf, T (&tm)[4][3], T (&own)[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T u0 = plane[buf][k][ly][lx], u1 = plane[buf][k][ly][lx + 1];
      const T u2 = plane[buf][k][ly + 1][lx], u3 = plane[buf][k][ly + 1][lx + 1];
      own[k] = u0;
      bfly4(u0, u1, u2, u3, tm[0][k], tm[1][k], tm[2][k], tm[3][k]);
    }
  };

  // One barrier per plane.  Step ez: (A) stage vertex plane ez+1 (fetched two
  // steps earlier); issue the loads of this step; barrier; (B) finish the
  // gather of vertex plane ez-1 and run its epilogue, then compute element
  // plane ez.  Element plane ez's output for vertex plane ez is reduced along x
  // across lanes; the half owed to the vertex row above goes to LDS (read after
  // the next barrier), the rest stays in registers.  LDS buffers alternate
  // between steps, and the loop is unrolled twice so that the register sets of
  // the previous and the new plane alternate instead of being copied.
  //
  // Loads retire in issue order as far as the wait counters go, so the loads
  // of a step are issued by distance to their use: the epilogue operands of
  // vertex plane ez and the scale of element plane ez+1 (used next step)
  // first, then vertex plane ez+3 (staged two steps later).  Every load is
  // unconditional (a loaded register merged across a branch would make the
  // compiler wait for all outstanding loads), so the steps at the ends of the
  // chunk, whose loads go unused, re-read the nearest plane of the chunk
  // instead of the next chunk's: those re-reads hit in L2 and add no memory
  // traffic.
  double acc0 = 0.0, acc1 = 0.0;
  T ta[4][3], tb[4][3], ga[4][3], rq[3], ucur[3], uprev[3];
  // OpDiag: x-pair sum / difference of s in this thread's element row, latest
  // element plane; the 2x2 modes {sum, x, y, xy} of the element plane before.
  T ab[2] = {T(0), T(0)}, dm_prev[4] = {T(0), T(0), T(0), T(0)};
  typename Op::ERaw ea, eb;
  T sa, sb;
  // Vertex plane zu lives in raw set (zu - z0 + 1) & 1.  The issue order of
  // the prologue is pinned so that the loop is entered with the loads in
  // flight in the order a full step leaves them.
  fetch_plane(z0 - 1, raw0);
  __builtin_amdgcn_sched_barrier(0);
  fetch_plane(z0, raw1);
  __builtin_amdgcn_sched_barrier(0);
  stage_plane(0, z0 - 1, raw0);
  __builtin_amdgcn_sched_barrier(0);
  sb = ld(s, nxy * modp(z0 - 1, g.nz), exy);
  __builtin_amdgcn_sched_barrier(0);
  fetch_plane(z0 + 1, raw0);
  __builtin_amdgcn_sched_barrier(0);
  lds_barrier();
  plane_modes(0, ta, ucur);
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int k = 0; k < 3; ++k) ga[q][k] = T(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) rq[k] = uprev[k] = T(0);

  auto step = [&](int ez, auto par, T (&tp)[4][3], T (&tn)[4][3],
                  typename Op::Raw(&rawn)[S::NSLOT], typename Op::ERaw& e_new,
                  const typename Op::ERaw& e_old, T& s_new, const T& s_old) {
    constexpr int cb = decltype(par)::value;  // row buffer read in this step
    constexpr int pb = 1 - cb;                // plane buffer receiving vertex plane ez + 1
    if (ez < z1) stage_plane(pb, ez + 1, rawn);
    // epilogue of vertex plane ez (used for z0 <= ez < z1)
    op.efetch(c, nxy * modp(min(max(ez, z0), z1 - 1), g.nz), exy, e_new);
    // scale of element plane ez+1 (used for ez+1 < z1)
    s_new = ld(s, nxy * modp(min(ez + 1, z1 - 1), g.nz), exy);
    __builtin_amdgcn_sched_barrier(0);
    fetch_plane(min(ez + 3, z1), rawn);  // staged for ez+3 <= z1
    __builtin_amdgcn_sched_barrier(0);
    lds_barrier();
    T dg[4] = {T(0), T(0), T(0), T(0)};
    if constexpr (DIAG) {
      if (ez >= z0) {
        // 2x2 modes of element plane ez - 1 at vertex (ex, ey): element row
        // ey - 1 (t_y = +1, from the row below in LDS) and row ey (t_y = -1).
        const int lyu = ly > 0 ? ly - 1 : 0;
        T dm[4];
        plane_modes2(sab[cb][0][lyu][lx], sab[cb][1][lyu][lx], ab[0], ab[1], dm);
        // vertex plane ez - 1 lies between element planes ez - 2 and ez - 1
        vertex_modes(dm_prev, dm, dg);
#pragma unroll
        for (int k = 0; k < 4; ++k) dm_prev[k] = dm[k];
      }
    }
    if (ez > z0 && ez <= z1 && outv) {
      T ku[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) ku[k] = rq[k] + rowc[cb][k][ly - 1][lx];
      if constexpr (DIAG)
        op.store_diag(c, nxy * (ez - 1), exy, ku, uprev, e_old, dg, acc0, acc1);
      else
        op.store(c, nxy * (ez - 1), exy, ex, ey, ez - 1, ku, uprev, e_old, acc0, acc1);
    }
    const T se = s_old;
    if (ez < z1) {
      T unext[3];
      plane_modes(pb, tn, unext);
      T uh[8][3], wh[8][3];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          uh[q][k] = tp[q][k] + tn[q][k];      // m2 = 0
          uh[q + 4][k] = tp[q][k] - tn[q][k];  // m2 = 1
        }
      mode_apply(mk, se, uh, wh);
      if (ez >= z0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T g0 = ga[0][k] + (wh[0][k] + wh[4][k]), g1 = ga[1][k] + (wh[1][k] + wh[5][k]);
          const T g2 = ga[2][k] + (wh[2][k] + wh[6][k]), g3 = ga[3][k] + (wh[3][k] + wh[7][k]);
          T y0, y1, y2, y3;
          bfly4(g0, g1, g2, g3, y0, y1, y2, y3);
          // corners: 0 -> vertex (lx, ly), 1 -> (lx+1, ly), 2 -> (lx, ly+1), 3 -> (lx+1, ly+1)
          rq[k] = y0 + from_left(y1);
          rowc[pb][k][ly][lx] = y2 + from_left(y3);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 3; ++k) ga[q][k] = wh[q][k] - wh[q + 4][k];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        uprev[k] = ucur[k];
        ucur[k] = unext[k];
      }
      if constexpr (DIAG) {
        // element (ex - 1, ey) has t_x = +1, element (ex, ey) t_x = -1
        const T sl = from_left(se);
        ab[0] = sl + se;
        ab[1] = sl - se;
        sab[pb][0][ly][lx] = ab[0];
        sab[pb][1][ly][lx] = ab[1];
      }
    }
  };
  for (int ez = z0 - 1; ez <= z1; ez += 2) {
    // Steps come in pairs; a step past z1 only issues unused loads and waits
    // at the barrier.  (An early exit between the two would give the compiler
    // a path into the loop head with the newest loads still in flight.)
    step(ez, Par<0>{}, ta, tb, raw1, ea, eb, sa, sb);
    step(ez + 1, Par<1>{}, tb, ta, raw0, eb, ea, sb, sa);
  }
  if (Op::NACC > 0) {
    const double t0 = block_sum<S::NTHR / 64>(acc0, red);
    if (tid == 0) op.part.buf[(op.slot0 * 8 + c) * op.part.stride + tile] = t0;
  }
  if (Op::NACC > 1) {
    const double t1 = block_sum<S::NTHR / 64>(acc1, red);
    if (tid == 0) op.part.buf[(op.slot1 * 8 + c) * op.part.stride + tile] = t1;
  }
}

template <typename T, class Op>
__global__ void __launch_bounds__(TileShape<T>::NTHR) __attribute__((amdgpu_waves_per_eu(Op0Waves<T>::value)))
op0_kernel(Op op, Grid g, TileGeom tg, ModeK<T> mk, const T* __restrict__ s) {
  op0_body<T, Op>(op, g, tg, mk, s, logical_block());
}

// Batched form: one persistent grid works through the items of many cells.
// Items are ordered cell by cell (largest cells first) and split into eight
// contiguous ranges, one per XCD, so that the items that item_tile puts next
// to each other still meet in one L2; the blocks of an XCD take the items of
// its range round robin.
template <typename T, class Op>
struct Op0Cell {
  Op op;
  Grid g;
  TileGeom tg;
  const T* s;
};

template <typename T, class Op>
__global__ void __launch_bounds__(TileShape<T>::NTHR) __attribute__((amdgpu_waves_per_eu(Op0Waves<T>::value)))
op0_batched_kernel(const Op0Cell<T, Op>* __restrict__ cells, const int2* __restrict__ items,
                   int nitems, ModeK<T> mk) {
  const int G = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, per_xcd_blocks = (G + 7 - xcd) >> 3;  // blocks of this XCD
  const int lo = (int)((int64_t)nitems * xcd / 8), hi = (int)((int64_t)nitems * (xcd + 1) / 8);
  for (int it = lo + (b >> 3); it < hi; it += per_xcd_blocks) {
    const int2 w = items[it];
    const Op0Cell<T, Op>& ce = cells[w.x];
    op0_body<T, Op>(ce.op, ce.g, ce.tg, mk, ce.s, w.y);
    __syncthreads();  // the next item reuses the LDS buffers
  }
}

template <typename T>
__device__ __forceinline__ bool scal_active(const double* scal, int c) {
  return scal == nullptr || scal[S_ACTIVE * 8 + c] != 0.0;
}

// ------------------------------------------------------------------ ops
// Interface: fetch/finish see vertex `xy` of the plane at offset `zoff`
// (uniform), efetch/store the thread's own vertex; `c` is the load case.
template <typename T>
struct OpApply {
  static constexpr int NACC = 0;
  __device__ void prep(int) {}
  const T* in;
  T* out;
  int64_t n;
  const double* scal;
  Partials part;
  int slot0, slot1;
  __device__ bool active(int c) const { return scal_active<T>(scal, c); }
  struct Raw {
    T u[3];
  };
  struct ERaw {};
  __device__ void fetch(int c, int64_t zoff, uint32_t xy, bool, Raw& w) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) w.u[k] = ld(in, (c * 3 + k) * n + zoff, xy);
  }
  __device__ void finish(int, int64_t, uint32_t, int, int, int, bool, const Raw& w,
                         T (&v)[3]) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = w.u[k];
  }
  __device__ void efetch(int, int64_t, uint32_t, ERaw&) const {}
  __device__ void store(int c, int64_t zoff, uint32_t xy, int, int, int, const T* ku, const T*,
                        const ERaw&, double&, double&) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) st(out, (c * 3 + k) * n + zoff, xy, ku[k]);
  }
};

// p_new = z + beta p_old (written at owned vertices), q = K p_new, acc p.q.
// With p stored in a narrower type V, p_new is rounded to V before K is
// applied, so q = K p holds for the stored direction; q itself stays in T
// (r -= alpha q must track f - K x to the working precision).
template <typename T, typename V>
struct OpMatvecP {
  static constexpr int NACC = 1;
  const V* z;
  const V* pold;
  V* pnew;
  T* q;
  int64_t n;
  const double* scal;
  Partials part;
  int slot0, slot1;
  T beta;  // set by prep
  __device__ void prep(int c) { beta = (T)scal[S_BETA * 8 + c]; }
  __device__ bool active(int c) const { return scal_active<T>(scal, c); }
  struct Raw {
    V z[3], p[3];
  };
  struct ERaw {};
  __device__ void fetch(int c, int64_t zoff, uint32_t xy, bool, Raw& w) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int64_t o = (c * 3 + k) * n + zoff;
      w.z[k] = ld(z, o, xy);
      w.p[k] = ld(pold, o, xy);
    }
  }
  __device__ void finish(int c, int64_t zoff, uint32_t xy, int, int, int, bool own, const Raw& w,
                         T (&v)[3]) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const V pv = (V)((T)w.z[k] + beta * (T)w.p[k]);
      v[k] = (T)pv;
      if (own) st(pnew, (c * 3 + k) * n + zoff, xy, pv);
    }
  }
  __device__ void efetch(int, int64_t, uint32_t, ERaw&) const {}
  __device__ void store(int c, int64_t zoff, uint32_t xy, int, int, int, const T* ku,
                        const T* uin, const ERaw&, double& a0, double&) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      st(q, (c * 3 + k) * n + zoff, xy, ku[k]);
      a0 += (double)uin[k] * (double)ku[k];
    }
  }
};

// Residual after the pre-smoothing from zero: t = (r - m) - K z0, where
// z0 = Dinv (r - m) was formed pointwise beforehand.  m is the per-component
// mean of r (FP64), removed so that rounding-level translation components of r
// are not amplified in soft regions.
template <typename T, typename V>
struct OpResidual {
  static constexpr int NACC = 0;
  const T* r;
  const T* z0;
  V* t;
  int64_t n;
  const double* scal;
  Partials part;
  int slot0, slot1;
  double m[3];  // per-case means of r (set by prep)
  __device__ void prep(int c) {
#pragma unroll
    for (int k = 0; k < 3; ++k) m[k] = scal[(S_MEAN0 + k) * 8 + c];
  }
  __device__ bool active(int c) const { return scal_active<T>(scal, c); }
  struct Raw {
    T u[3];
  };
  struct ERaw {
    T r[3];
  };
  __device__ void efetch(int c, int64_t zoff, uint32_t xy, ERaw& e) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) e.r[k] = ld(r, (c * 3 + k) * n + zoff, xy);
  }
  __device__ void fetch(int c, int64_t zoff, uint32_t xy, bool, Raw& w) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) w.u[k] = ld(z0, (c * 3 + k) * n + zoff, xy);
  }
  __device__ void finish(int, int64_t, uint32_t, int, int, int, bool, const Raw& w,
                         T (&v)[3]) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = (T)w.u[k];
  }
  __device__ void store(int c, int64_t zoff, uint32_t xy, int, int, int, const T* ku, const T*,
                        const ERaw& e, double&, double&) const {
#pragma unroll
    for (int k = 0; k < 3; ++k)
      st(t, (c * 3 + k) * n + zoff, xy, (V)((T)((double)e.r[k] - m[k]) - ku[k]));
  }
};

// Post-smoothing: zout = z1 + omega D^-1 ((r - m) - K z1), acc (r - m).zout,
// with D the vertex's diagonal block of K (formed from the diagonal modes, see
// OpDiag).  z1 is the pre-smoothed correction plus the prolongated coarse
// correction; both it and zout are multiplied by K, so they keep the
// arithmetic type.
template <typename T, typename V>
struct OpPostSmooth {
  static constexpr int NACC = 2;
  static constexpr bool DIAG = true;
  const T* z1;
  const T* r;
  T* zout;
  const T* q;  // optional: q of the last matvec, for q.zout
  int64_t n;
  const double* scal;
  Partials part;
  int slot0, slot1;
  T dd, oo, omega;  // diagonal / off-diagonal entry of K0's diagonal blocks; damping
  double m[3];      // per-case means of r (set by prep)
  __device__ void prep(int c) {
#pragma unroll
    for (int k = 0; k < 3; ++k) m[k] = scal[(S_MEAN0 + k) * 8 + c];
  }
  __device__ bool active(int c) const { return scal_active<T>(scal, c); }
  struct Raw {
    T u[3];
  };
  struct ERaw {
    T r[3], q[3];
  };
  __device__ void efetch(int c, int64_t zoff, uint32_t xy, ERaw& e) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) e.r[k] = ld(r, (c * 3 + k) * n + zoff, xy);
#pragma unroll
    for (int k = 0; k < 3; ++k) e.q[k] = q ? ld(q, (c * 3 + k) * n + zoff, xy) : T(0);
  }
  __device__ void fetch(int c, int64_t zoff, uint32_t xy, bool, Raw& w) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) w.u[k] = ld(z1, (c * 3 + k) * n + zoff, xy);
  }
  __device__ void finish(int, int64_t, uint32_t, int, int, int, bool, const Raw& w,
                         T (&v)[3]) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = (T)w.u[k];
  }
  // The damped block inverse omega D^-1 is formed here from the diagonal modes
  // dg (cofactors over the determinant), so the pass streams no stored inverse.
  __device__ void store_diag(int c, int64_t zoff, uint32_t xy, const T* ku, const T* uin,
                             const ERaw& e, const T (&dg)[4], double& a0, double& a1) const {
    T d[6];
    damped_block_inverse(dd, oo, omega, dg, d);
    const T dxx = d[0], dyy = d[1], dzz = d[2], dxy = d[3], dyz = d[4], dxz = d[5];
    T res[3], rv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      rv[k] = (T)((double)e.r[k] - m[k]);
      res[k] = rv[k] - ku[k];
    }
    T zn[3];
    zn[0] = uin[0] + (dxx * res[0] + dxy * res[1] + dxz * res[2]);
    zn[1] = uin[1] + (dxy * res[0] + dyy * res[1] + dyz * res[2]);
    zn[2] = uin[2] + (dxz * res[0] + dyz * res[1] + dzz * res[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      st(zout, (c * 3 + k) * n + zoff, xy, zn[k]);
      a0 += (double)rv[k] * (double)zn[k];
      a1 += (double)e.q[k] * (double)zn[k];
    }
  }
};

template <typename T>
__device__ __forceinline__ void forcing_at(const Grid& g, const T* __restrict__ s,
                                           const LoadTpl<T>& tpl, int c, int gx, int gy, int gz,
                                           T (&f)[3]) {
  const int xm = gx == 0 ? g.nx - 1 : gx - 1;
  const int ym = gy == 0 ? g.ny - 1 : gy - 1;
  const int zm = gz == 0 ? g.nz - 1 : gz - 1;
  const int64_t nx = g.nx, nxy = (int64_t)g.nx * g.ny;
  f[0] = f[1] = f[2] = T(0);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int64_t e = ((a & 1) ? xm : gx) + nx * ((a & 2) ? ym : gy) + nxy * ((a & 4) ? zm : gz);
    const T se = s[e];
#pragma unroll
    for (int k = 0; k < 3; ++k) f[k] += se * tpl.g[c][a][k];
  }
}

// The same with the case's 24 template values in device memory, w[3 a + k]:
// for a case index known only at run time (a by-value template indexed by it
// would be copied to scratch memory).
template <typename T>
__device__ __forceinline__ void forcing_at(const Grid& g, const T* __restrict__ s,
                                           const T* __restrict__ w, int gx, int gy, int gz,
                                           T (&f)[3]) {
  const int xm = gx == 0 ? g.nx - 1 : gx - 1;
  const int ym = gy == 0 ? g.ny - 1 : gy - 1;
  const int zm = gz == 0 ? g.nz - 1 : gz - 1;
  const int64_t nx = g.nx, nxy = (int64_t)g.nx * g.ny;
  f[0] = f[1] = f[2] = T(0);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int64_t e = ((a & 1) ? xm : gx) + nx * ((a & 2) ? ym : gy) + nxy * ((a & 4) ? zm : gz);
    const T se = s[e];
#pragma unroll
    for (int k = 0; k < 3; ++k) f[k] += se * w[3 * a + k];
  }
}

// r = f - K x (computed in T, stored as R);  acc0 f.f, acc1 r.r.  tplg: the
// load template g[c][a][k] in device memory.
template <typename T, typename R>
struct OpForceResidual {
  static constexpr int NACC = 2;
  __device__ void prep(int) {}
  const T* x;
  R* r;
  const T* s;
  const T* tplg;
  Grid g;
  int64_t n;
  const double* scal;
  Partials part;
  int slot0, slot1;
  __device__ bool active(int c) const { return scal_active<T>(scal, c); }
  struct Raw {
    T u[3];
  };
  struct ERaw {};
  __device__ void efetch(int, int64_t, uint32_t, ERaw&) const {}
  __device__ void fetch(int c, int64_t zoff, uint32_t xy, bool, Raw& w) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) w.u[k] = ld(x, (c * 3 + k) * n + zoff, xy);
  }
  __device__ void finish(int, int64_t, uint32_t, int, int, int, bool, const Raw& w,
                         T (&v)[3]) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = w.u[k];
  }
  __device__ void store(int c, int64_t zoff, uint32_t xy, int gx, int gy, int gz, const T* ku,
                        const T*, const ERaw&, double& a0, double& a1) const {
    T f[3];
    forcing_at(g, s, tplg + 24 * c, gx, gy, gz, f);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T rv = f[k] - ku[k];
      st(r, (c * 3 + k) * n + zoff, xy, (R)rv);
      a0 += (double)f[k] * (double)f[k];
      a1 += (double)rv * (double)rv;
    }
  }
};

template <typename T, class Op>
void launch_op0(const Op0Launch<T>& L, const Op& op) {
  const TileGeom tg = tile_geom<T>(L.g);
  const int nblk = tg.ntiles * NCASE;
  hipLaunchKernelGGL((op0_kernel<T, Op>), dim3(nblk), dim3(TileShape<T>::NTHR), 0, L.stream, op,
                     L.g, tg, L.mk, L.s);
}

// ------------------------------------------------------------------ pointwise kernels
template <typename R>
__global__ void forcing_kernel(Grid g, LoadTpl<double> tpl, const double* __restrict__ s,
                               R* __restrict__ f, Partials part) {
  __shared__ double red[4];
  double acc[NCASE];
#pragma unroll
  for (int c = 0; c < NCASE; ++c) acc[c] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int gx = (int)(i % g.nx);
    const int gy = (int)((i / g.nx) % g.ny);
    const int gz = (int)(i / ((int64_t)g.nx * g.ny));
#pragma unroll
    for (int c = 0; c < NCASE; ++c) {
      double fv[3];
      forcing_at(g, s, tpl, c, gx, gy, gz, fv);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        f[(int64_t)(c * 3 + k) * g.n + i] = (R)fv[k];
        acc[c] += fv[k] * fv[k];
      }
    }
  }
  if (part.buf) {
#pragma unroll
    for (int c = 0; c < NCASE; ++c) {
      const double t = block_sum<4>(acc[c], red);
      if (threadIdx.x == 0) part.buf[(S_FF * 8 + c) * part.stride + blockIdx.x] = t;
    }
  }
}

template <typename T>
__global__ void simp_kernel(int64_t n, const float* __restrict__ rho, T* __restrict__ s,
                            T* __restrict__ keep, double* __restrict__ s64,
                            double* __restrict__ keep64, double E0, double Emin, double penal,
                            int* bad) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double r = rho[i];
    if (!(r >= 0.0 && r <= 1.0)) {
      atomicOr(bad, 1);  // any thread; the flag is only tested for nonzero
      s[i] = T(E0);
      keep[i] = T(0);
      if (s64) {
        s64[i] = E0;
        keep64[i] = 0.0;
      }
      continue;
    }
    double rp;
    if (penal == 3.0)
      rp = r * r * r;
    else
      rp = (r > 0.0) ? pow(r, penal) : 0.0;
    const double sv = Emin + rp * (E0 - Emin);
    s[i] = (T)sv;
    keep[i] = (T)r;
    if (s64) {
      s64[i] = sv;
      keep64[i] = r;
    }
  }
}

// Jacobi from a zero start at level 0: z0 = omega D^-1 (r - m) for every active
// case, with the vertex's diagonal block D formed from the eight element scales
// around it (OpDiag) instead of read from a stored inverse.  Block b of nb takes
// grid rows (y, z) b, b + nb, ...; threads run along x.
template <typename T>
__device__ __forceinline__ void jacobi0s_rows(const Grid& g, const T* __restrict__ s,
                                              const BlockDiag0& bd, const T* __restrict__ r,
                                              T* __restrict__ z, const double* scal,
                                              const double* mean, int b, int nb) {
  bool on[NCASE];
  double m[NCASE][3];
#pragma unroll
  for (int c = 0; c < NCASE; ++c) {
    on[c] = scal_active<T>(scal, c);
#pragma unroll
    for (int k = 0; k < 3; ++k) m[c][k] = mean ? mean[(S_MEAN0 + k) * 8 + c] : 0.0;
  }
  const T dd = (T)bd.dd, oo = (T)bd.oo, omega = (T)bd.omega;
  const int64_t n = g.n, nx = g.nx, nxy = (int64_t)g.nx * g.ny;
  const int rows = g.ny * g.nz;
  for (int row = b; row < rows; row += nb) {
    const int y = row % g.ny, zz = row / g.ny;
    const int ym = y == 0 ? g.ny - 1 : y - 1, zm = zz == 0 ? g.nz - 1 : zz - 1;
    const T* s_lo_u = s + nxy * zm + nx * ym;  // element rows (y - 1, y) of planes z - 1, z
    const T* s_lo = s + nxy * zm + nx * y;
    const T* s_hi_u = s + nxy * zz + nx * ym;
    const T* s_hi = s + nxy * zz + nx * y;
    for (int x = threadIdx.x; x < g.nx; x += blockDim.x) {
      const int xm = x == 0 ? g.nx - 1 : x - 1;
      T lo[4], hi[4], dg[4], d[6];
      plane_modes2(s_lo_u[xm] + s_lo_u[x], s_lo_u[xm] - s_lo_u[x], s_lo[xm] + s_lo[x],
                   s_lo[xm] - s_lo[x], lo);
      plane_modes2(s_hi_u[xm] + s_hi_u[x], s_hi_u[xm] - s_hi_u[x], s_hi[xm] + s_hi[x],
                   s_hi[xm] - s_hi[x], hi);
      vertex_modes(lo, hi, dg);
      damped_block_inverse(dd, oo, omega, dg, d);
      const int64_t i = nxy * zz + nx * y + x;
#pragma unroll
      for (int c = 0; c < NCASE; ++c) {
        if (!on[c]) continue;
        const T r0 = (T)((double)r[(c * 3 + 0) * n + i] - m[c][0]);
        const T r1 = (T)((double)r[(c * 3 + 1) * n + i] - m[c][1]);
        const T r2 = (T)((double)r[(c * 3 + 2) * n + i] - m[c][2]);
        z[(c * 3 + 0) * n + i] = d[0] * r0 + d[3] * r1 + d[5] * r2;
        z[(c * 3 + 1) * n + i] = d[3] * r0 + d[1] * r1 + d[4] * r2;
        z[(c * 3 + 2) * n + i] = d[5] * r0 + d[4] * r1 + d[2] * r2;
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
jacobi0s_kernel(Grid g, const T* __restrict__ s, BlockDiag0 bd, const T* __restrict__ r,
                T* __restrict__ z, const double* scal, const double* mean) {
  jacobi0s_rows<T>(g, s, bd, r, z, scal, mean, blockIdx.x, gridDim.x);
}

// Batched form: blockIdx.y is the cell.
__global__ void __launch_bounds__(256) jacobi0s_batched_kernel(const PwBatchCell* __restrict__ cells) {
  const PwBatchCell& ce = cells[blockIdx.y];
  jacobi0s_rows<float>(ce.g, ce.s, ce.bd, ce.r, ce.z, ce.scal, ce.scal, blockIdx.x, gridDim.x);
}

// 27-point stencil of the level-0 operator: thread per (vertex, offset d).
template <typename T>
__global__ void stencil0_kernel(Grid g, const T* __restrict__ s, const double* __restrict__ K0,
                                T* __restrict__ st) {
  const int d = blockIdx.y;
  const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int gx = (int)(i % g.nx);
    const int gy = (int)((i / g.nx) % g.ny);
    const int gz = (int)(i / ((int64_t)g.nx * g.ny));
    double blk[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < 8; ++a) {
      const int a0 = a & 1, a1 = (a >> 1) & 1, a2 = a >> 2;
      const int b0 = a0 + dx, b1 = a1 + dy, b2 = a2 + dz;
      if (b0 < 0 || b0 > 1 || b1 < 0 || b1 > 1 || b2 < 0 || b2 > 1) continue;
      const int b = b0 + 2 * b1 + 4 * b2;
      const int64_t e = modp(gx - a0, g.nx) + (int64_t)g.nx * (modp(gy - a1, g.ny) +
                        (int64_t)g.ny * modp(gz - a2, g.nz));
      const double se = (double)s[e];
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) blk[p * 3 + q] += se * K0[(3 * a + p) * 24 + 3 * b + q];
    }
    for (int t = 0; t < 9; ++t) st[(int64_t)(d * 9 + t) * g.n + i] = (T)blk[t];
  }
}

inline int pw_blocks(int64_t n, int tpb, int cap) {
  int64_t b = (n + tpb - 1) / tpb;
  if (b > cap) b = cap;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

int op0_blocks_per_case(const Grid& g) {
  return std::max(tile_geom<float>(g).ntiles, tile_geom<double>(g).ntiles);
}
int op0_tiles_per_case(const Grid& g, int lz) { return tile_geom<float>(g, lz).ntiles; }

struct Op0BatchPlan {
  int kind = 0;
  void* cells = nullptr;
  int2* items = nullptr;
  int nitems = 0;
  int grid = 0;
};

namespace {
template <class Op>
Op0BatchPlan* build_plan(int kind, const std::vector<Op0Cell<float, Op>>& hc, int grid,
                         hipStream_t st) {
  std::vector<int2> items;
  for (int c = 0; c < (int)hc.size(); ++c)
    for (int j = 0; j < hc[c].tg.ntiles * NCASE; ++j) items.push_back(make_int2(c, j));
  Op0BatchPlan* p = new Op0BatchPlan;
  p->kind = kind;
  p->nitems = (int)items.size();
  p->grid = grid > 0 ? std::min(grid, p->nitems) : p->nitems;
  if (hipMalloc(&p->cells, sizeof(Op0Cell<float, Op>) * hc.size()) != hipSuccess ||
      hipMalloc((void**)&p->items, sizeof(int2) * items.size()) != hipSuccess) {
    op0_batch_free(p);
    return nullptr;
  }
  (void)hipMemcpyAsync(p->cells, hc.data(), sizeof(Op0Cell<float, Op>) * hc.size(),
                       hipMemcpyHostToDevice, st);
  (void)hipMemcpyAsync(p->items, items.data(), sizeof(int2) * items.size(),
                       hipMemcpyHostToDevice, st);
  (void)hipStreamSynchronize(st);
  return p;
}
}  // namespace

Op0BatchPlan* op0_batch_plan(int kind, const Op0BatchCell* cells, int ncells, int grid,
                             hipStream_t st) {
  if (kind == OP0B_MATVEC) {
    std::vector<Op0Cell<float, OpMatvecP<float, float>>> hc;
    for (int c = 0; c < ncells; ++c) {
      const Op0BatchCell& a = cells[c];
      OpMatvecP<float, float> op{a.in0, a.in1, a.out0, a.out1, a.g.n, a.scal, a.part, S_PQ, 0,
                                 0.f};
      hc.push_back({op, a.g, tile_geom<float>(a.g, a.lz), a.s});
    }
    return build_plan(kind, hc, grid, st);
  }
  if (kind == OP0B_RESIDUAL) {
    std::vector<Op0Cell<float, OpResidual<float, float>>> hc;
    for (int c = 0; c < ncells; ++c) {
      const Op0BatchCell& a = cells[c];
      OpResidual<float, float> op{a.in0, a.in1, a.out0, a.g.n, a.scal, Partials{}, 0, 0, {}};
      hc.push_back({op, a.g, tile_geom<float>(a.g, a.lz), a.s});
    }
    return build_plan(kind, hc, grid, st);
  }
  std::vector<Op0Cell<float, OpPostSmooth<float, float>>> hc;
  for (int c = 0; c < ncells; ++c) {
    const Op0BatchCell& a = cells[c];
    OpPostSmooth<float, float> op{a.in0,   a.in1,  a.out0,          a.in3,
                                  a.g.n,   a.scal, a.part,          S_RZNEW,
                                  S_QZ,    (float)a.bd.dd, (float)a.bd.oo, (float)a.bd.omega,
                                  {}};
    hc.push_back({op, a.g, tile_geom<float>(a.g, a.lz), a.s});
  }
  return build_plan(kind, hc, grid, st);
}

void op0_batch_launch(const Op0BatchPlan* p, const ModeK<float>& mk, hipStream_t st) {
  if (p->kind == OP0B_MATVEC)
    hipLaunchKernelGGL((op0_batched_kernel<float, OpMatvecP<float, float>>), dim3(p->grid),
                       dim3(TileShape<float>::NTHR), 0, st, (const Op0Cell<float, OpMatvecP<float, float>>*)p->cells,
                       p->items, p->nitems, mk);
  else if (p->kind == OP0B_RESIDUAL)
    hipLaunchKernelGGL((op0_batched_kernel<float, OpResidual<float, float>>), dim3(p->grid),
                       dim3(TileShape<float>::NTHR), 0, st,
                       (const Op0Cell<float, OpResidual<float, float>>*)p->cells, p->items,
                       p->nitems, mk);
  else
    hipLaunchKernelGGL((op0_batched_kernel<float, OpPostSmooth<float, float>>), dim3(p->grid),
                       dim3(TileShape<float>::NTHR), 0, st,
                       (const Op0Cell<float, OpPostSmooth<float, float>>*)p->cells, p->items,
                       p->nitems, mk);
}

void op0_batch_free(Op0BatchPlan* p) {
  if (!p) return;
  if (p->cells) (void)hipFree(p->cells);
  if (p->items) (void)hipFree(p->items);
  delete p;
}

int op0_batch_items(const Op0BatchPlan* p) { return p->nitems; }

template <typename T>
void op0_apply(const Op0Launch<T>& L, const T* in, T* out, const double* scal) {
  OpApply<T> op{in, out, L.g.n, scal, Partials{}, 0, 0};
  launch_op0(L, op);
}

template <typename T, typename V>
void op0_matvec_p(const Op0Launch<T>& L, const V* z, const V* pold, V* pnew, T* q,
                  const double* scal, Partials part, int* nblk_out) {
  // The new direction goes to a separate buffer: the kernel reads halo values of
  // pold that neighbouring blocks must not have overwritten yet.
  OpMatvecP<T, V> op{z, pold, pnew, q, L.g.n, scal, part, S_PQ, 0, T(0)};
  launch_op0(L, op);
  *nblk_out = tile_geom<T>(L.g).ntiles;
}

template <typename T, typename V>
void op0_residual(const Op0Launch<T>& L, const T* r, const T* z0, V* t, const double* scal) {
  OpResidual<T, V> op{r, z0, t, L.g.n, scal, Partials{}, 0, 0, {}};
  launch_op0(L, op);
}

template <typename T, typename V>
void op0_post_smooth(const Op0Launch<T>& L, const T* z1, const T* r, const BlockDiag0& bd,
                     T* zout, const T* q, const double* scal, Partials part, int* nblk_out) {
  OpPostSmooth<T, V> op{z1,      r,      zout,   q,          L.g.n,       scal,
                        part,    S_RZNEW, S_QZ,  (T)bd.dd,   (T)bd.oo,    (T)bd.omega, {}};
  launch_op0(L, op);
  *nblk_out = tile_geom<T>(L.g).ntiles;
}

template <typename R>
void op0_force_residual(const Op0Launch<double>& L, const double* tplg, const double* x,
                        R* r, const double* scal, Partials part, int* nblk_out) {
  OpForceResidual<double, R> op{x, r, L.s, tplg, L.g, L.g.n, scal, part, S_FF, S_TRUE};
  launch_op0(L, op);
  *nblk_out = tile_geom<double>(L.g).ntiles;
}

template <typename R>
void forcing(const Grid& g, const LoadTpl<double>& tpl, const double* s, R* f, Partials part,
             int* nblk_out, hipStream_t st) {
  const int nb = pw_blocks(g.n, 256, part.buf ? part.stride : 4096);
  hipLaunchKernelGGL(forcing_kernel<R>, dim3(nb), dim3(256), 0, st, g, tpl, s, f, part);
  if (nblk_out) *nblk_out = nb;
}

template <typename T>
void simp_scale(const Grid& g, const float* rho, T* s, T* keep, double* s64, double* keep64,
                double E0, double Emin, double penal, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(simp_kernel<T>, dim3(pw_blocks(g.n, 256, 8192)), dim3(256), 0, st, g.n, rho,
                     s, keep, s64, keep64, E0, Emin, penal, bad);
}

template <typename T>
void jacobi0_level0(const Grid& g, const T* s, const BlockDiag0& bd, const T* r, T* z,
                    const double* scal, const double* mean, hipStream_t st) {
  hipLaunchKernelGGL(jacobi0s_kernel<T>, dim3(pw_blocks((int64_t)g.ny * g.nz, 1, 8192)), dim3(256),
                     0, st, g, s, bd, r, z, scal, mean);
}

void jacobi0_batched(const PwBatchCell* cells_dev, int ncells, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(jacobi0s_batched_kernel, dim3(nblk, ncells), dim3(256), 0, st, cells_dev);
}

template <typename T>
void stencil_level0(const Grid& g, const T* s, const double* K0_dev, T* st, hipStream_t stm) {
  hipLaunchKernelGGL(stencil0_kernel<T>, dim3(pw_blocks(g.n, 256, 4096), 27), dim3(256), 0, stm, g,
                     s, K0_dev, st);
}

#define HMG_INST2(T, V)                                                                          \
  template void op0_matvec_p<T, V>(const Op0Launch<T>&, const V*, const V*, V*, T*,             \
                                   const double*, Partials, int*);                               \
  template void op0_residual<T, V>(const Op0Launch<T>&, const T*, const T*, V*, const double*); \
  template void op0_post_smooth<T, V>(const Op0Launch<T>&, const T*, const T*,                  \
                                      const BlockDiag0&, T*, const T*, const double*, Partials,   \
                                      int*);
#define HMG_INST1(T)                                                                             \
  template void op0_apply<T>(const Op0Launch<T>&, const T*, T*, const double*);                  \
  template void op0_force_residual<T>(const Op0Launch<double>&, const double*,                  \
                                      const double*, T*, const double*, Partials, int*);         \
  template void forcing<T>(const Grid&, const LoadTpl<double>&, const double*, T*, Partials,    \
                           int*, hipStream_t);                                                    \
  template void simp_scale<T>(const Grid&, const float*, T*, T*, double*, double*, double,       \
                              double, double, int*, hipStream_t);                                 \
  template void jacobi0_level0<T>(const Grid&, const T*, const BlockDiag0&, const T*, T*,         \
                                  const double*, const double*, hipStream_t);                   \
  template void stencil_level0<T>(const Grid&, const T*, const double*, T*, hipStream_t);
HMG_INST1(float)
HMG_INST1(double)
HMG_INST2(float, float)
HMG_INST2(double, double)
HMG_INST2(float, bf16)
#undef HMG_INST1
#undef HMG_INST2

}  // namespace hmg

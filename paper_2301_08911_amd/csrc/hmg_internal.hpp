// Internal declarations of the gfx950 homogenization solver: element constants,
// kernel launchers and the scalar slots shared by the PCG kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace hmg {

constexpr int NCASE = 6;  // six unit macro strains (Voigt 11,22,33,12,23,13)

// Storage of the multigrid preconditioner's streamed data (smoother
// corrections, coarse residuals and corrections, coarse stencils and block
// inverses): V is the type in memory, Acc<V> the type the kernels compute in.
// The reduced-precision form stores V = bf16 and computes in FP32; the plain
// forms store what they compute in.  The outer PCG vectors keep the
// arithmetic type.
using bf16 = __bf16;
using f16 = _Float16;
template <typename V>
struct Acc {
  using type = float;
};
template <>
struct Acc<double> {
  using type = double;
};

// Periodic grid of one multigrid level: n vertices == n elements.
struct Grid {
  int nx = 0, ny = 0, nz = 0;
  int64_t n = 0;
};

// The 24x24 element stiffness K0 (E = 1) written in the basis of 8-point
// Walsh-Hadamard modes of the nodal values: Kt = H K0 H / 64 with
// H[a][m] = (-1)^popcount(a & m).  In this basis Kt has 45 nonzeros arranged in
// a few small blocks (indices are (mode m, component k)):
//   normal strains  (1,0),(2,1),(4,2):  diag ab + b, off-diagonal b
//   shear pairs     (1,1)&(2,0), (1,2)&(4,0), (2,2)&(4,1): all four entries cs
//   bilinear pairs  (3,0)&(6,2), (3,1)&(5,2), (5,0)&(6,1): [[p q][q p]]
//   bilinear triple (3,2),(5,1),(6,0): diag fg + g, off-diagonal g
//   trilinear       (7,k): diag z
// Mode 0 (rigid translation) has an all-zero row and column.
template <typename T>
struct ModeK {
  T ab, b, cs, p, q, fg, g, z;
};

// K0 chi^i for the six unit strains: 3-vector per local node.
template <typename T>
struct LoadTpl {
  T g[NCASE][8][3];
};

// Every entry of K0 (unit brick, E = 1, isotropic) is plus or minus one of ten
// values, selected by the bits of the two nodes and the two components:
//   same component i:  v[3 e_i + c], e_i = [a_i == b_i], c = number of the
//                      other two axes on which a and b agree;
//   components i != j: (lambda +- mu) M_m / 4 with m the third axis,
//                      M_m = 1/3 if a_m == b_m else 1/6: v[6 + 2 e_m + g],
//                      g = 1 for lambda + mu (the two sign products agree),
//                      sign s(a_i) s(b_j) with s(0) = -1, s(1) = +1.
// k0_sel returns (index << 1) | negative.  build_element_consts checks that the
// ten values rebuild K0 exactly.
__host__ __device__ constexpr int k0_sel(int a, int i, int b, int j) {
  if (i == j) {
    int c = 0;
    for (int k = 0; k < 3; ++k)
      if (k != i && ((a >> k) & 1) == ((b >> k) & 1)) ++c;
    const int ei = ((a >> i) & 1) == ((b >> i) & 1) ? 1 : 0;
    return (3 * ei + c) << 1;
  }
  const int m = 3 - i - j;
  const int em = ((a >> m) & 1) == ((b >> m) & 1) ? 1 : 0;
  const int sai = ((a >> i) & 1) ? 1 : -1, sbj = ((b >> j) & 1) ? 1 : -1;
  const int saj = ((a >> j) & 1) ? 1 : -1, sbi = ((b >> i) & 1) ? 1 : -1;
  const int g = sai * sbj == saj * sbi ? 1 : 0;
  return ((6 + 2 * em + g) << 1) | (sai * sbj < 0 ? 1 : 0);
}

// Everything the library derives from (E = 1, nu) on the host, in double.
struct ElementConsts {
  double K0[24][24];          // element stiffness, dof 3a+k
  ModeK<double> mk;           // K0 in the Walsh-Hadamard mode basis
  double load[NCASE][8][3];   // K0 chi^i per local node
  double chihat[NCASE][8][3]; // H chi^i (mode basis)
  double dd, oo;              // K0[a,a] = dd I + oo * sg_p sg_q (p != q), sg = +-1 by node bit
  double msig[8][24][24];     // W_sigma^T K0 W_sigma for the 8 sub-element positions
  double lam0;                // max eigenvalue of blockdiag(K0)^-1 K0: bounds the level-0
                              // block-Jacobi spectrum for any densities
  double kv[10];              // the ten distinct magnitudes of K0 (k0_sel)
};

// Returns 0 on success; fills `err` otherwise.
int build_element_consts(double nu, ElementConsts* out, char* err, size_t errlen);
// The F^3 sub-element Galerkin matrices W_sigma^T K0 W_sigma of a coarse
// element F fine cells long (F = 2: ElementConsts::msig; F = 4: the
// non-dyadic first step), F^3 x 576 doubles.
void subelement_matrices(const double K0[24][24], int F, double* out);

// Scalar slots of the PCG state, stored as double scal[slot * 8 + case].
enum Slot {
  S_FF = 0,     // ||f||^2
  S_RR,         // ||r||^2
  S_RZ,         // r.z of the current iteration
  S_RZNEW,      // r.z just computed
  S_PQ,         // p.q
  S_ALPHA,
  S_BETA,
  S_THRESH,     // convergence threshold on ||r||
  S_ACTIVE,     // 1 while the case iterates
  S_TRIVIAL,    // 1 if ||f|| <= eps_abs
  S_MEAN0,      // per-component means (3 slots)
  S_MEAN1,
  S_MEAN2,
  S_TRUE,       // recomputed ||f - K x||^2
  S_RESTART,    // 1: the residual was just recomputed; restart the direction (beta = 0)
  S_QZ,         // q.z_new (Polak-Ribiere form of beta)
  S_REPLACED,   // 1: r was replaced by f - K x this iteration (beta falls back to r.z ratios)
  S_XALPHA,     // alphas of the directions whose x += alpha p is still pending:
  S_XALPHA2,    // S_XALPHA + j for the (j+1)-th newest (consecutive slots)
  S_XALPHA3,
  S_NSLOT
};

// Deterministic per-block partial sums: buf[(slot * 8 + c) * stride + block].
struct Partials {
  double* buf = nullptr;
  int stride = 0;
};

// ---------------------------------------------------------------- level 0
template <typename T> struct Op0Launch {
  Grid g;
  ModeK<T> mk;
  const T* s;   // element stiffness scale [n]
  hipStream_t stream;
};

template <typename T>
void op0_apply(const Op0Launch<T>& L, const T* in, T* out, const double* scal);
// p_new = z + beta p_old, q = K p_new, partial p.q (arithmetic in T; z and p
// stored as V, q as T).
template <typename T, typename V>
void op0_matvec_p(const Op0Launch<T>& L, const V* z, const V* pold, V* pnew, T* q,
                  const double* scal, Partials part, int* nblk_out);
// t = (r - m) - K z0; m from scal S_MEAN* (z0 = Dinv (r - m) from vec_jacobi0,
// or a Gauss-Seidel sweep); t is stored as V (it is only restricted, never
// multiplied by K).
template <typename T, typename V>
void op0_residual(const Op0Launch<T>& L, const T* r, const T* z0, V* t, const double* scal);
// Damped block Jacobi at level 0: the diagonal (dd) and off-diagonal (oo) entry
// of K0's diagonal blocks, and the damping factor.
struct BlockDiag0 {
  double dd, oo, omega;
};
// zout = z1 + omega D^-1 ((r - m) - K z1), D the vertex's diagonal block of K
// formed in the kernel from s; partial (r - m).zout in S_RZNEW and, if q is
// given, q.zout in S_QZ.
template <typename T, typename V>
void op0_post_smooth(const Op0Launch<T>& L, const T* z1, const T* r, const BlockDiag0& bd,
                     T* zout, const T* q, const double* scal, Partials part, int* nblk_out);
// r = f - K x evaluated in FP64 (x, s and the constants in double), stored as R.
// tplg: the FP64 load template g[c][a][k] (LoadTpl layout) in device memory.
template <typename R>
void op0_force_residual(const Op0Launch<double>& L, const double* tplg, const double* x,
                        R* r, const double* scal, Partials part, int* nblk_out);
// Upper bound of the blocks per case of any level-0 pass (FP32 or FP64 tiles).
int op0_blocks_per_case(const Grid& g);

// Batched level-0 passes (FP32) over many cells in one persistent launch.
// Vectors per kind:  matvec: in0 z, in1 p_old, out0 p_new, out1 q;
// residual: in0 r, in1 z0, out0 t;  post-smooth: in0 z1, in1 r, in3 q
// (optional), out0 z, and bd.
enum Op0BatchKind { OP0B_MATVEC = 0, OP0B_RESIDUAL = 1, OP0B_POST_SMOOTH = 2 };
struct Op0BatchCell {
  Grid g;
  int lz;  // z-chunk of a tile (<= 0: default)
  const float* s;
  const float *in0, *in1, *in2, *in3;
  float *out0, *out1;
  const double* scal;
  Partials part;
  BlockDiag0 bd;  // post-smooth only
};
struct Op0BatchPlan;
// Uploads the per-cell descriptors and the item list; `grid` blocks (<= 0: one
// per item).  Returns nullptr if a device allocation fails.
Op0BatchPlan* op0_batch_plan(int kind, const Op0BatchCell* cells, int ncells, int grid,
                             hipStream_t st);
void op0_batch_launch(const Op0BatchPlan* plan, const ModeK<float>& mk, hipStream_t st);
void op0_batch_free(Op0BatchPlan* plan);
int op0_batch_items(const Op0BatchPlan* plan);
// Tiles per case of an FP32 level-0 pass with z-chunk lz (0 = default).
int op0_tiles_per_case(const Grid& g, int lz);

// Macro-strain loads evaluated in FP64, stored as R; partial ||f||^2 in S_FF.
template <typename R>
void forcing(const Grid& g, const LoadTpl<double>& tpl, const double* s, R* f, Partials part,
             int* nblk_out, hipStream_t st);
// s = Emin + rho^p (E0 - Emin) as T (and optionally in double), rho kept as T / double.
template <typename T>
void simp_scale(const Grid& g, const float* rho, T* s, T* rho_keep, double* s64, double* rho64,
                double E0, double Emin, double penal, int* bad, hipStream_t st);
// z0 = omega D^-1 (r - m) at level 0 for the active cases, D the vertex's
// diagonal block of K formed from s (m from `mean` slots S_MEAN*, NULL: none).
template <typename T>
void jacobi0_level0(const Grid& g, const T* s, const BlockDiag0& bd, const T* r, T* z,
                    const double* scal, const double* mean, hipStream_t st);
template <typename T>
void stencil_level0(const Grid& g, const T* s, const double* K0_dev, T* st, hipStream_t stm);

// ---------------------------------------------------------------- vectors
// x += alpha p (FP64 iterate), r -= alpha q; partials ||r||^2 (S_RR) and
// sum r (S_MEAN*).
// r -= alpha q (S_ALPHA) with the FP64 iterate advanced every fourth iteration:
// npend = 0 leaves x alone (alpha p becomes pending; the caller shifts the
// pending alphas up one slot and moves S_ALPHA to S_XALPHA), otherwise
// x += sum_{j < npend} S_XALPHA+j pend[j] + S_ALPHA p, pend[j] the (j+1)-th
// newest pending direction (npend <= 3).  Partials per block of ||r||^2 (slot
// S_RR) and of sum r per component (S_MEAN*).
template <typename T>
void vec_update_r4(const Grid& g, double* x, const T* const* pend, int npend, const T* p, T* r,
                   const T* q, const double* scal, Partials part, int* nblk_out, hipStream_t st);
// x += sum_{j < npend} S_XALPHA+j pend[j] for the cases active in scal (the
// pending directions, 1 <= npend <= 3; npend = 0 does nothing).
template <typename T>
void vec_flush_x(const Grid& g, double* x, const T* const* pend, int npend, const double* scal,
                 hipStream_t st);
template <typename S, typename D>
void vec_convert(D* dst, const S* src, int64_t count, hipStream_t st);
// Batched FP32 pointwise passes over many cells (update grid: nblk x cells*6,
// one load case per block row; Jacobi grid: nblk x cells):
// update: x += alpha p, r -= alpha q (+ partials);  jacobi (level 0, grid rows
// per block): z = omega D^-1 (r - m), D formed from s, m from the cell's scal.
struct PwBatchCell {
  Grid g;
  double* x;
  const float* p;
  float* r;
  const float* q;
  const float* s;  // element scales (level-0 Jacobi)
  float* z;
  const double* scal;
  Partials part;
  BlockDiag0 bd;  // level-0 Jacobi
};
void update_batched(const PwBatchCell* cells_dev, int ncells, int nblk, hipStream_t st);
void jacobi0_batched(const PwBatchCell* cells_dev, int ncells, int nblk, hipStream_t st);
int vec_blocks_for(int64_t n);
// z = Dinv (r - m) with m from `mean` slots S_MEAN* (NULL: no shift).
template <typename R, typename D, typename Z>
void vec_jacobi0(const Grid& g, const R* r, const D* dinv, Z* z, const double* scal,
                 const double* mean, hipStream_t st);
template <typename T>
void vec_fill(T* a, int64_t count, T v, hipStream_t st);
template <typename T>
void vec_scale(T* a, int64_t count, double factor, hipStream_t st);
// x (FP64) += z
template <typename T>
void vec_add_to(double* x, const T* z, int64_t count, hipStream_t st);
// out[V] = mean of in over the f^3 fine cells of coarse cell V (gf.nx/f cells per axis).
template <typename T>
void vec_box_mean(const Grid& gf, const T* in, int f, float* out, hipStream_t st);
// Deterministic pseudo-random values in [-1, 1) (power-iteration start vectors).
template <typename T>
void vec_pattern(T* a, int64_t count, hipStream_t st);
template <typename T>
void vec_copy(T* dst, const T* src, int64_t count, hipStream_t st);
template <typename A, typename B>
void vec_dot_cases(const Grid& g, const A* a, const B* b, const double* scal, Partials part,
                   int slot, int* nblk_out, hipStream_t st);
template <typename T>
void vec_mean_partial(const Grid& g, const T* a, Partials part, int* nblk_out, hipStream_t st);
template <typename T>
void vec_mean_subtract(const Grid& g, T* a, const double* scal, hipStream_t st);
int vec_blocks(const Grid& g);
// out_dev[0] = sum_i a[i] (deterministic, two launches).
template <typename T>
void vec_sum_scalar(const T* a, int64_t n, double* out_dev, Partials part, hipStream_t st);

// Finalizers (one small launch each; read partials, update scal).
void fin_sum(const Partials& part, int slot, int nblk, double* scal, bool all_cases,
             hipStream_t st);
void fin_init(double* scal, double eps_abs, double tol, hipStream_t st);
void fin_alpha(double* scal, hipStream_t st);
// beta = r.z_new / r.z (Fletcher-Reeves), or with polak_ribiere the form
// -alpha q.z_new / r.z, which tolerates a preconditioner that varies from one
// application to the next (rounded storage); 0 after a restart.
void fin_beta(double* scal, bool polak_ribiere, hipStream_t st);
void fin_mean(const Partials& part, int nblk, int64_t n, double* scal, hipStream_t st);
void scal_set_all_active(double* scal, hipStream_t st);

// ---------------------------------------------------------------- coarse levels
// T is the storage type of the vectors, W that of the stencils and block
// inverses; arithmetic runs in Acc<T>.
template <typename T, typename W>
void kc_apply(const Grid& g, const W* st, const T* u, T* y, hipStream_t s);
template <typename T, typename W>
void kc_residual(const Grid& g, const W* st, const T* z, const T* r, T* t, const double* scal,
                 const double* mean, hipStream_t s);
template <typename T, typename W>
void kc_smooth(const Grid& g, const W* st, const T* z, const T* r, const W* dinv, T* zout,
               const double* scal, const double* mean, hipStream_t s);
template <typename T>
void restrict_to(const Grid& gf, const Grid& gc, const T* tf, T* rc, const double* scal,
                 hipStream_t s);
// zf (fine, type F) (+)= P ec (coarse, type C).
template <typename F, typename C>
void prolong_add(const Grid& gf, const Grid& gc, F* zf, const C* ec, const double* scal,
                 bool overwrite, hipStream_t s);
template <typename S, typename T>
void galerkin_first(const Grid& gf, const Grid& gc, const S* s, const double* msig_dev, T* st,
                    hipStream_t stm);
template <typename T>
void galerkin_next(const Grid& gf, const Grid& gc, const T* stf, T* stc, hipStream_t stm);
template <typename T>
void dinv_from_stencil(const Grid& g, const T* st, double omega, T* dinv, hipStream_t stm);
template <typename T>
void dense_from_stencil(const Grid& g, const T* st, double* A, hipStream_t stm);
// In-place inverse of the N x N SPD matrix A; A must be followed by
// coarse_scratch_doubles(N) doubles of scratch, which coarse_solve also uses.
void gauss_jordan_inverse(int N, double* A, hipStream_t stm);
int64_t coarse_scratch_doubles(int N);
template <typename R, typename T>
void coarse_solve(const Grid& g, const double* Ainv, const R* r, T* z, const double* scal,
                  hipStream_t stm);

// ---------------------------------------------------------------- Gauss-Seidel
// Eight-colour symmetric block Gauss-Seidel sweeps (gs.hip).  A forward sweep
// relaxes colours 0..7, a backward sweep 7..0; "fresh" marks a forward sweep
// whose z starts at zero (z need not be cleared).  The right-hand side is
// r - m with m from the S_MEAN* slots of `mean` (NULL: no shift).
// True if the grid's rows fit the level-0 kernels (even extents, nx <= 1024).
bool gs_supported(const Grid& g);
// Level 0, matrix free (k0v: the ten magnitudes of K0, ElementConsts::kv, on
// the host).  With nblk_out set (backward sweeps), partials of (r - m).z go to
// slot S_RZNEW and, if q is given, of q.z to S_QZ; *nblk_out receives their
// count.
template <typename T>
void gs0_sweep(const Grid& g, const double* k0v, const T* s, const T* r, const double* mean, T* z,
               const T* q, const double* scal, Partials part, bool forward, bool fresh,
               int* nblk_out, hipStream_t st);
int gs0_blocks_per_case(const Grid& g);
// Coarse levels from stored stencils; dinv holds the undamped block inverses.
template <typename V, typename W>
void gsc_sweep(const Grid& g, const W* st, const W* dinv, const V* r, const double* mean, V* z,
               const double* scal, bool forward, bool fresh, hipStream_t stm);

// ---------------------------------------------------------------- design space
// Symmetry group as signed axis permutations (design.hip): code[t] =
// perm0 | perm1 << 2 | perm2 << 4 | flips << 6; output axis a takes input
// axis perm_a, mirrored (c -> N - 1 - c) when bit a of flips is set.
struct SymOps {
  int count = 0;
  int code[48] = {};
};
void symmetrize(const Grid& g, const float* in, float* out, const SymOps& ops, hipStream_t st);
constexpr int TRIG_MAX_FREQ = 4;
constexpr int TRIG_MAX_WEIGHTS = 6 * TRIG_MAX_FREQ + 3 * TRIG_MAX_FREQ * (6 * TRIG_MAX_FREQ + 1);
struct TrigBasis {
  double R[9];  // rotation of the centred element coordinates
  int nfreq;    // 1..TRIG_MAX_FREQ
};
// y = sum_m w_m Q_m(x_e) (w: 6 nfreq + 6 nfreq (6 nfreq + 1) / 2 doubles on the device)
void trig_field(const Grid& g, const TrigBasis& tb, const double* w_dev, float* y,
                hipStream_t st);
// y <- rho_min + Vh / (1 + exp(-k (y - mu))) with mu by `steps` bisection steps
// on the mean; state (4 doubles) ends with mu in state[3].  part needs a stride
// of at least 4096 and two rows.
void sigmoid_project(const Grid& g, float* y, double volfrac, double rho_min, double k,
                     double* state, Partials part, int steps, hipStream_t st);
// out = H(x g) / max(1e-3, x) with the normalized cone weights w_dev
void sensitivity_filter(const Grid& g, const float* x, const float* gin, float* out,
                        const float* w_dev, int h, hipStream_t st);

// ---------------------------------------------------------------- post-processing
// u is stored as U: the arithmetic type, or FP16 (the cast of Sec. 4.3, with T = float)
template <typename T, typename U>
void elastic_partials(const Grid& g, const ModeK<T>& mk, const LoadTpl<T>& chihat, const T* s,
                      const U* u, Partials part, int* nblk_out, hipStream_t st);
void elastic_finalize(const Partials& part, int nblk, int64_t n, double* out36, hipStream_t st);
template <typename T, typename U>
void sensitivity(const Grid& g, const ModeK<T>& mk, const LoadTpl<T>& chihat, const T* rho,
                 const U* u, const double* w21_dev, double coef, double penal, float* out,
                 hipStream_t st);
void density_filter(const Grid& g, const float* in, float* out, const float* w_dev, int h,
                    hipStream_t st);
void oc_partial(const Grid& g, const float* x, const float* dfdx, double move, double damp,
                double xmin, const double* state, Partials part, int* nblk_out, hipStream_t st);
void oc_step(const Partials& part, int nblk, int64_t n, double volfrac, double* state,
             hipStream_t st);
void oc_apply(const Grid& g, float* x, const float* dfdx, double move, double damp, double xmin,
              const double* state, hipStream_t st);
void oc_init(double* state, hipStream_t st);

}  // namespace hmg

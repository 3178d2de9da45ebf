// Internal declarations of the gfx950 homogenization solver: element constants,
// kernel launchers and the scalar slots shared by the PCG kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace hmg {

constexpr int NCASE = 6;  // six unit macro strains (Voigt 11,22,33,12,23,13)

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
};

// Returns 0 on success; fills `err` otherwise.
int build_element_consts(double nu, ElementConsts* out, char* err, size_t errlen);

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
  S_XALPHA,     // step not yet applied to x: x += S_XALPHA * p (done by the next matvec)
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
// p_new = z + beta p_old, q = K p_new, partial p.q; also x += alpha_x p_old
// (the pending iterate update) at owned vertices.
template <typename T>
void op0_matvec_p(const Op0Launch<T>& L, const T* z, const T* pold, T* pnew, T* q, double* x,
                  const double* scal, Partials part, int* nblk_out);
// z0 = Dinv (r - m) (also written out) and t = (r - m) - K z0; m from scal S_MEAN*.
template <typename T>
void op0_residual(const Op0Launch<T>& L, const T* r, const T* dinv, T* z0, T* t,
                  const double* scal);
// zout = z1 + Dinv ((r - m) - K z1); partial (r - m).zout in S_RZNEW.
template <typename T>
void op0_post_smooth(const Op0Launch<T>& L, const T* z1, const T* r, const T* dinv, T* zout,
                     const double* scal, Partials part, int* nblk_out);
// r = f - K x evaluated in FP64 (x, s and the constants in double), stored as R.
template <typename R>
void op0_force_residual(const Op0Launch<double>& L, const LoadTpl<double>& tpl, const double* x,
                        R* r, const double* scal, Partials part, int* nblk_out);
int op0_blocks_per_case(const Grid& g);

// Macro-strain loads evaluated in FP64, stored as R; partial ||f||^2 in S_FF.
template <typename R>
void forcing(const Grid& g, const LoadTpl<double>& tpl, const double* s, R* f, Partials part,
             int* nblk_out, hipStream_t st);
// s = Emin + rho^p (E0 - Emin) as T (and optionally in double), rho kept as T / double.
template <typename T>
void simp_scale(const Grid& g, const float* rho, T* s, T* rho_keep, double* s64, double* rho64,
                double E0, double Emin, double penal, int* bad, hipStream_t st);
template <typename T>
void dinv_level0(const Grid& g, const T* s, double dd, double oo, double omega, T* dinv,
                 hipStream_t st);
template <typename T>
void stencil_level0(const Grid& g, const T* s, const double* K0_dev, T* st, hipStream_t stm);

// ---------------------------------------------------------------- vectors
// r -= alpha q; partials ||r||^2 (S_RR) and sum r (S_MEAN*).  The iterate
// update is deferred (slot S_XALPHA); vec_flush_x applies it: x += alpha_x p.
template <typename T>
void vec_update_r(const Grid& g, T* r, const T* q, const double* scal, Partials part,
                  int* nblk_out, hipStream_t st);
template <typename T>
void vec_flush_x(const Grid& g, double* x, const T* p, double* scal, hipStream_t st);
template <typename S, typename D>
void vec_convert(D* dst, const S* src, int64_t count, hipStream_t st);
// z = Dinv (r - m) with m from `mean` slots S_MEAN* (NULL: no shift).
template <typename T>
void vec_jacobi0(const Grid& g, const T* r, const T* dinv, T* z, const double* scal,
                 const double* mean, hipStream_t st);
template <typename T>
void vec_fill(T* a, int64_t count, T v, hipStream_t st);
// Deterministic pseudo-random values in [-1, 1) (power-iteration start vectors).
template <typename T>
void vec_pattern(T* a, int64_t count, hipStream_t st);
template <typename T>
void vec_copy(T* dst, const T* src, int64_t count, hipStream_t st);
template <typename T>
void vec_dot_cases(const Grid& g, const T* a, const T* b, const double* scal, Partials part,
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
void fin_beta(double* scal, hipStream_t st);
void fin_mean(const Partials& part, int nblk, int64_t n, double* scal, hipStream_t st);
void scal_set_all_active(double* scal, hipStream_t st);

// ---------------------------------------------------------------- coarse levels
template <typename T>
void kc_apply(const Grid& g, const T* st, const T* u, T* y, hipStream_t s);
template <typename T>
void kc_residual(const Grid& g, const T* st, const T* z, const T* r, T* t, const double* scal,
                 const double* mean, hipStream_t s);
template <typename T>
void kc_smooth(const Grid& g, const T* st, const T* z, const T* r, const T* dinv, T* zout,
               const double* scal, const double* mean, hipStream_t s);
template <typename T>
void restrict_to(const Grid& gf, const Grid& gc, const T* tf, T* rc, const double* scal,
                 hipStream_t s);
template <typename T>
void prolong_add(const Grid& gf, const Grid& gc, T* zf, const T* ec, const double* scal,
                 bool overwrite, hipStream_t s);
template <typename T>
void galerkin_first(const Grid& gf, const Grid& gc, const T* s, const double* msig_dev, T* st,
                    hipStream_t stm);
template <typename T>
void galerkin_next(const Grid& gf, const Grid& gc, const T* stf, T* stc, hipStream_t stm);
template <typename T>
void dinv_from_stencil(const Grid& g, const T* st, double omega, T* dinv, hipStream_t stm);
template <typename T>
void dense_from_stencil(const Grid& g, const T* st, double* A, hipStream_t stm);
void gauss_jordan_inverse(int N, double* A, hipStream_t stm);
template <typename T>
void coarse_solve(const Grid& g, const double* Ainv, const T* r, T* z, const double* scal,
                  hipStream_t stm);

// ---------------------------------------------------------------- post-processing
template <typename T>
void elastic_partials(const Grid& g, const ModeK<T>& mk, const LoadTpl<T>& chihat, const T* s,
                      const T* u, Partials part, int* nblk_out, hipStream_t st);
void elastic_finalize(const Partials& part, int nblk, int64_t n, double* out36, hipStream_t st);
template <typename T>
void sensitivity(const Grid& g, const ModeK<T>& mk, const LoadTpl<T>& chihat, const T* rho,
                 const T* u, const double* w21_dev, double coef, double penal, float* out,
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

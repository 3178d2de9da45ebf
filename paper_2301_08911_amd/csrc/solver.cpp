// Host runtime of the solver and the extern "C" entry points of include/hmg.h.
//
// One context = one periodic cell on one device.  It owns the multigrid
// hierarchy (Sec. 3.3) and the PCG work fields, drives the kernels on the
// caller's HIP stream, and keeps every scalar of the six CG recurrences in
// FP64 on the device; the host only reads them back once per iteration to
// decide convergence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/hmg.h"
#include "../../include/hmg_nn.h"
#include "hmg_internal.hpp"
#include "nn_internal.hpp"

using namespace hmg;

namespace {

constexpr int MAX_COARSE_DOF = 12288;  // dense inverse of the coarsest grid (16^3 vertices)

struct Status {
  hmg_status code = HMG_OK;
  std::string msg;
};

class DeviceArena {
 public:
  ~DeviceArena() { release(); }
  void* alloc(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 256;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    ptrs_.push_back(p);
    return p;
  }
  void release() {
    for (void* p : ptrs_) (void)hipFree(p);
    ptrs_.clear();
  }

 private:
  std::vector<void*> ptrs_;
};

// Optional per-kernel timing with HIP events recorded on the context stream
// around the tracked launches; elapsed times are harvested when read.
class KernelClock {
 public:
  static constexpr int NK = 9;
  ~KernelClock() {
    for (auto& p : pending_) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : pool_) (void)hipEventDestroy(e);
  }
  void enable(bool on) {
    on_ = on;
    if (on) {
      harvest();
      for (int k = 0; k < NK; ++k) {
        ms_[k] = 0.0;
        bytes_[k] = 0.0;
        count_[k] = 0;
      }
    }
  }
  template <class F>
  void timed(int k, double bytes, hipStream_t st, F&& launch) {
    if (!on_) {
      launch();
      return;
    }
    Rec r{k, bytes, get(), get()};
    (void)hipEventRecord(r.a, st);
    launch();
    (void)hipEventRecord(r.b, st);
    pending_.push_back(r);
    if (pending_.size() > 4096) harvest();
  }
  void read(int k, int64_t* count, double* ms, double* bytes) {
    harvest();
    *count = count_[k];
    *ms = ms_[k];
    *bytes = bytes_[k];
  }

 private:
  struct Rec {
    int k;
    double bytes;
    hipEvent_t a, b;
  };
  hipEvent_t get() {
    if (!pool_.empty()) {
      hipEvent_t e = pool_.back();
      pool_.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  void harvest() {
    for (auto& p : pending_) {
      (void)hipEventSynchronize(p.b);
      float t = 0.0f;
      (void)hipEventElapsedTime(&t, p.a, p.b);
      ms_[p.k] += t;
      bytes_[p.k] += p.bytes;
      count_[p.k] += 1;
      pool_.push_back(p.a);
      pool_.push_back(p.b);
    }
    pending_.clear();
  }
  bool on_ = false;
  std::vector<Rec> pending_;
  std::vector<hipEvent_t> pool_;
  double ms_[NK] = {}, bytes_[NK] = {};
  int64_t count_[NK] = {};
};

// Precision-independent interface of a typed solver.
class SolverIface {
 public:
  virtual ~SolverIface() = default;
  virtual Status init() = 0;
  virtual Status set_density(const float* rho) = 0;
  virtual Status solve(double tol, int max_iter, int init, const void* u0, int iters[6],
                       double relres[6]) = 0;
  virtual Status elastic(double C[36]) = 0;
  virtual Status sens(const double W[36], float* out) = 0;
  virtual Status get_disp(void* u) = 0;
  virtual Status apply_op(int level, const void* u, void* y) = 0;
  virtual Status get_stencil(int level, void* out) = 0;
  virtual Status loads(void* f) = 0;
  virtual Status vcycle(const void* r, void* z) = 0;
  virtual Status transfer(int level, int dir, const void* in, void* out) = 0;
  virtual Status warm_start(Net& net, double accept, double* relres, int* used) = 0;
  virtual int levels() const = 0;
  virtual Grid level_grid(int l) const = 0;
  virtual double level_omega(int l) const = 0;
  KernelClock clock;
};

Status fail(hmg_status code, const char* fmt, ...) {
  Status s;
  s.code = code;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  s.msg = buf;
  return s;
}

Status check_hip(const char* where) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HMG_E_DEVICE, "%s: %s", where, hipGetErrorString(e));
  return Status{};
}

#define HMG_TRY(expr)                        \
  do {                                       \
    Status _s = (expr);                      \
    if (_s.code != HMG_OK) return _s;        \
  } while (0)

class BatchSolver;

// T: arithmetic type of the solver vectors; V: their storage type (and that of
// the coarse stencils).  The FP64 iterate, the FP64 scalars and the level-0
// residual r (type T) are the same in every form.
template <typename T, typename V, typename W>
class Solver final : public SolverIface {
  // Rounded storage makes the preconditioner vary slightly between
  // applications; beta then takes the Polak-Ribiere form.
  static constexpr bool kPR = !std::is_same<T, V>::value;
  friend class BatchSolver;

 public:
  Solver(const hmg_config& cfg, hipStream_t st, const ElementConsts& ec, std::vector<Grid> grids)
      : cfg_(cfg), st_(st), ec_(ec), grids_(std::move(grids)) {}

  int levels() const override { return (int)grids_.size(); }
  int stride_tiles(int lz) const { return op0_tiles_per_case(grids_[0], lz); }
  Grid level_grid(int l) const override { return grids_[l]; }
  double level_omega(int l) const override {
    return l < (int)omega_.size() ? omega_[l] : 0.0;
  }

  Status init() override {
    const Grid& g0 = grids_[0];
    const int64_t F = (int64_t)NCASE * 3 * g0.n;
    mk_ = cast_mode(ec_.mk);
    mk64_ = ec_.mk;
    for (int c = 0; c < NCASE; ++c)
      for (int a = 0; a < 8; ++a)
        for (int k = 0; k < 3; ++k) {
          tpl_.g[c][a][k] = (T)ec_.load[c][a][k];
          tpl64_.g[c][a][k] = ec_.load[c][a][k];
          chh64_.g[c][a][k] = ec_.chihat[c][a][k];
          chh32_.g[c][a][k] = (float)ec_.chihat[c][a][k];
        }
    auto A = [&](size_t bytes) { return arena_.alloc(bytes); };
    s_ = (T*)A(sizeof(T) * g0.n);
    rho_ = (T*)A(sizeof(T) * g0.n);
    x_ = (double*)A(sizeof(double) * F);
    if (sizeof(T) == sizeof(double)) {
      s64_ = (double*)s_;
      rho64_ = (double*)rho_;
    } else {
      s64_ = (double*)A(sizeof(double) * g0.n);
      rho64_ = (double*)A(sizeof(double) * g0.n);
    }
    r_ = (T*)A(sizeof(T) * F);
    z_ = (T*)A(sizeof(T) * F);
    t_ = (V*)A(sizeof(V) * F);
    pa_ = (T*)A(sizeof(T) * F);
    pb_ = (T*)A(sizeof(T) * F);
    pc_ = (T*)A(sizeof(T) * F);
    pd_ = (T*)A(sizeof(T) * F);
    q_ = (T*)A(sizeof(T) * F);
    // The plain forms reuse q (dead while the V-cycle runs); the reduced-
    // precision form keeps q for the Polak-Ribiere beta.
    w0_ = kPR ? (T*)A(sizeof(T) * F) : q_;
    const int L = levels();
    lev_.resize(L);
    for (int l = 1; l < L; ++l) {
      const Grid& g = grids_[l];
      const int64_t Fl = (int64_t)NCASE * 3 * g.n;
      lev_[l].st = (W*)A(sizeof(W) * 243 * g.n);
      lev_[l].dinv = (W*)A(sizeof(W) * 6 * g.n);
      lev_[l].r = (V*)A(sizeof(V) * Fl);
      lev_[l].z = (V*)A(sizeof(V) * Fl);
      lev_[l].t = (V*)A(sizeof(V) * Fl);
      lev_[l].ms = (double*)A(sizeof(double) * S_NSLOT * 8);
    }
    const Grid& gL = grids_[L - 1];
    ncdof_ = (int)(3 * gL.n);
    // the coarsest correction is the largest, smoothest field of the cycle and
    // is multiplied by K after prolongation: it keeps the arithmetic type
    if (L > 1) zc_ = (T*)A(sizeof(T) * NCASE * 3 * gL.n);
    Ainv_ = (double*)A(sizeof(double) *
                       ((size_t)ncdof_ * ncdof_ + (size_t)coarse_scratch_doubles(ncdof_)));
    if (L == 1) st0_ = (T*)A(sizeof(T) * 243 * g0.n);
    stride_ = std::max(op0_blocks_per_case(g0), 4096);
    if (gs_) stride_ = std::max(stride_, 4 * gs0_blocks_per_case(g0));
    part_.buf = (double*)A(sizeof(double) * (size_t)S_NSLOT * 8 * stride_);
    part_.stride = stride_;
    scal_ = (double*)A(sizeof(double) * S_NSLOT * 8);
    aux_ = (double*)A(sizeof(double) * S_NSLOT * 8);
    misc_ = (double*)A(sizeof(double) * 64);
    K0dev_ = (double*)A(sizeof(double) * 576);
    tplg_ = (double*)A(sizeof(LoadTpl<double>));
    msig_ = (double*)A(sizeof(double) * 8 * 576);
    bad_ = (int*)A(sizeof(int) * 4);
    for (void* p : {(void*)s_, (void*)rho_, (void*)x_, (void*)r_, (void*)z_,
                    (void*)t_, (void*)pa_, (void*)pb_, (void*)pc_, (void*)pd_, (void*)q_, (void*)Ainv_, (void*)part_.buf,
                    (void*)scal_, (void*)aux_, (void*)misc_, (void*)K0dev_, (void*)tplg_,
                    (void*)msig_,
                    (void*)bad_, (void*)s64_, (void*)rho64_})
      if (!p) return fail(HMG_E_OOM, "device allocation failed for a %dx%dx%d cell", g0.nx, g0.ny,
                          g0.nz);
    if (L == 1 && !st0_) return fail(HMG_E_OOM, "device allocation failed (level-0 stencil)");
    for (int l = 1; l < L; ++l)
      if (!lev_[l].st || !lev_[l].dinv || !lev_[l].r || !lev_[l].z || !lev_[l].t || !lev_[l].ms)
        return fail(HMG_E_OOM, "device allocation failed at level %d", l);
    if (hipHostMalloc((void**)&hscal_, sizeof(double) * S_NSLOT * 8 * 3) != hipSuccess)
      return fail(HMG_E_OOM, "pinned host allocation failed");
    hstage_ = hscal_ + 2 * S_NSLOT * 8;
    (void)hipMemcpyAsync(K0dev_, &ec_.K0[0][0], sizeof(double) * 576, hipMemcpyHostToDevice, st_);
    (void)hipMemcpyAsync(tplg_, &tpl64_.g[0][0][0], sizeof(LoadTpl<double>), hipMemcpyHostToDevice,
                         st_);
    (void)hipMemcpyAsync(msig_, &ec_.msig[0][0][0], sizeof(double) * 8 * 576, hipMemcpyHostToDevice,
                   st_);
    if (L > 1 && grids_[0].nx == 4 * grids_[1].nx) {
      // non-dyadic first step: 64 sub-element matrices
      msig4_host_.assign(64 * 576, 0.0);
      subelement_matrices(ec_.K0, 4, msig4_host_.data());
      msig4_ = (double*)A(sizeof(double) * 64 * 576);
      if (!msig4_) return fail(HMG_E_OOM, "device allocation failed (sub-element matrices)");
      (void)hipMemcpyAsync(msig4_, msig4_host_.data(), sizeof(double) * 64 * 576,
                           hipMemcpyHostToDevice, st_);
    }

    vec_fill<double>(x_, F, 0.0, st_);
    HMG_TRY(check_hip("init"));
    if (hipStreamSynchronize(st_) != hipSuccess) return check_hip("init sync");
    return Status{};
  }

  ~Solver() override {
    if (hscal_) (void)hipHostFree(hscal_);
    if (nnbuf_) (void)hipFree(nnbuf_);
  }

  // Learned initial guess (see hmg_warm_start): density box mean on level lt,
  // network prediction of u/N there, times N, zero mean per component,
  // trilinear prolongation to the fine grid, FP64 residual test.
  Status warm_start(Net& net, double accept, double* relres, int* used) override {
    fp16_ready_ = false;
    if (!have_density_) return fail(HMG_E_STATE, "hmg_set_density has not been called");
    const Grid& g0 = grids_[0];
    if (g0.nx != g0.ny || g0.nx != g0.nz) return fail(HMG_E_INVALID, "warm start needs a cubic cell");
    if (net.in_channels() != 1 || net.out_channels() != 3 * NCASE)
      return fail(HMG_E_INVALID, "the network must map 1 channel to %d", 3 * NCASE);
    int lt = -1;
    for (int l = 0; l < levels(); ++l) {
      const int d = grids_[l].nx;
      if (d <= 64 && d % net.dim_multiple() == 0 && d >= net.min_dim()) {
        lt = l;
        break;
      }
    }
    if (lt < 0) return fail(HMG_E_INVALID, "no multigrid level of this cell fits the network");
    const Grid& gt = grids_[lt];
    const int64_t Ft = (int64_t)NCASE * 3 * gt.n, F = (int64_t)NCASE * 3 * g0.n;
    if (!nnbuf_ && hipMalloc((void**)&nnbuf_, sizeof(float) * 19 * 64 * 64 * 64) != hipSuccess)
      return fail(HMG_E_OOM, "warm-start buffer allocation failed");
    float* xin = nnbuf_;
    float* yout = nnbuf_ + gt.n;
    vec_box_mean<T>(g0, rho_, g0.nx / gt.nx, xin, st_);
    const std::string e = net.forward(xin, 1, gt.nx, yout);
    if (!e.empty()) return fail(HMG_E_DEVICE, "%s", e.c_str());
    vec_scale<float>(yout, Ft, (double)g0.nx, st_);  // u = N * (u / N)
    int nb = 0;
    vec_mean_partial<float>(gt, yout, part_, &nb, st_);
    fin_mean(part_, nb, gt.n, aux_, st_);
    vec_mean_subtract<float>(gt, yout, aux_, st_);
    if (lt == 0) {
      vec_convert<float, double>(x_, yout, F, st_);
    } else {
      vec_convert<float, V>(lev_[lt].z, yout, Ft, st_);
      for (int l = lt - 1; l >= 1; --l)
        prolong_add<V, V>(grids_[l], grids_[l + 1], lev_[l].z, lev_[l + 1].z, nullptr, true, st_);
      prolong_add<T, V>(g0, grids_[1], w0_, lev_[1].z, nullptr, true, st_);
      vec_convert<T, double>(x_, w0_, F, st_);
    }
    // relative residual of the guess, then of the guess after one V-cycle
    // correction x += M (f - K x): a guess right at low frequencies can carry a
    // large high-frequency residual, which a single cycle removes
    Op0Launch<double> L64{g0, mk64_, s64_, st_};
    const double lam1 = cfg_.nu / ((1 + cfg_.nu) * (1 - 2 * cfg_.nu));
    const double mu1 = 1.0 / (2 * (1 + cfg_.nu));
    const double eps_abs = 1e-12 * std::sqrt((double)g0.n) * (lam1 + 2 * mu1) * mean_s_;
    auto worst_relres = [&](double* out) -> Status {
      scal_set_all_active(aux_, st_);
      op0_force_residual<T>(L64, tplg_, x_, r_, nullptr, part_, &nb);
      fin_sum(part_, S_FF, nb, aux_, true, st_);
      fin_sum(part_, S_TRUE, nb, aux_, true, st_);
      HMG_TRY(read_scal(aux_, hscal_ + S_NSLOT * 8));
      const double* ha = hscal_ + S_NSLOT * 8;
      double w = 0.0;
      for (int c = 0; c < NCASE; ++c) {
        const double ff = std::sqrt(ha[S_FF * 8 + c]), tr = std::sqrt(ha[S_TRUE * 8 + c]);
        if (ff > eps_abs) w = std::max(w, tr / ff);
      }
      *out = w;
      return Status{};
    };
    // Energy-optimal scale of every case's guess: alpha = u.f / u.K u minimizes
    // the energy error ||u* - alpha u||_K over alpha, so the scaled guess is
    // never further from the solution in that norm than the zero start.
    {
      T* fbuf = q_;  // free until the solve
      int nbd = 0;
      scal_set_all_active(aux_, st_);
      forcing<T>(g0, tpl64_, s64_, fbuf, part_, &nbd, st_);
      vec_dot_cases<double, T>(g0, x_, fbuf, aux_, part_, S_PQ, &nbd, st_);
      fin_sum(part_, S_PQ, nbd, aux_, true, st_);  // u.f
      op0_force_residual<T>(L64, tplg_, x_, r_, nullptr, part_, &nbd);
      vec_dot_cases<double, T>(g0, x_, r_, aux_, part_, S_RZ, &nbd, st_);
      fin_sum(part_, S_RZ, nbd, aux_, true, st_);  // u.(f - K u)
      HMG_TRY(read_scal(aux_, hscal_ + S_NSLOT * 8));
      const double* ha = hscal_ + S_NSLOT * 8;
      const int64_t cs = 3 * g0.n;
      for (int c = 0; c < NCASE; ++c) {
        const double uf = ha[S_PQ * 8 + c], uku = uf - ha[S_RZ * 8 + c];
        guess_scale_[c] = uku > 0.0 ? uf / uku : 0.0;
        vec_scale<double>(x_ + c * cs, cs, guess_scale_[c], st_);
      }
    }
    double raw = 0.0, worst = 0.0;
    HMG_TRY(worst_relres(&raw));
    vec_mean_partial<T>(g0, r_, part_, &nb, st_);
    fin_mean(part_, nb, g0.n, aux_, st_);
    HMG_TRY(vcycle_apply(r_, z_, nullptr, aux_, &nb));
    vec_add_to<T>(x_, z_, F, st_);
    HMG_TRY(worst_relres(&worst));
    raw_relres_ = raw;
    *relres = worst;
    *used = worst <= accept ? 1 : 0;
    if (*used) {
      have_iterate_ = true;
    } else {
      vec_fill<double>(x_, F, 0.0, st_);
      have_iterate_ = false;
    }
    have_solution_ = false;
    return check_hip("warm_start");
  }

  Status set_density(const float* rho) override {
    const Grid& g0 = grids_[0];
    (void)hipMemsetAsync(bad_, 0, sizeof(int), st_);
    const bool sep = sizeof(T) != sizeof(double);
    simp_scale<T>(g0, rho, s_, rho_, sep ? s64_ : nullptr, sep ? rho64_ : nullptr, cfg_.E0,
                  cfg_.Emin, cfg_.penal, bad_, st_);
    int bad = 0;
    (void)hipMemcpyAsync(&bad, bad_, sizeof(int), hipMemcpyDeviceToHost, st_);
    if (hipStreamSynchronize(st_) != hipSuccess) return check_hip("set_density");
    if (bad) return fail(HMG_E_INVALID, "density contains NaN or a value outside [0, 1]");
    vec_sum_scalar<T>(s_, g0.n, misc_, part_, st_);
    const int L = levels();
    omega_.assign(L, 0.0);
    lambda_.assign(L, 0.0);
    lambda_[0] = ec_.lam0;
    // Gauss-Seidel needs no damping: level 0 forms its blocks from s on the
    // fly, coarse levels keep the undamped inverses.
    omega_[0] = gs_ ? 1.0 : omega_for(ec_.lam0);
    for (int l = 1; l < L; ++l) {
      if (l == 1)
        galerkin_first<T, W>(g0, grids_[1], s_, msig4_ ? msig4_ : msig_, lev_[1].st, st_);
      else
        galerkin_next<W>(grids_[l - 1], grids_[l], lev_[l - 1].st, lev_[l].st, st_);
      if (l == L - 1) continue;  // the coarsest level is solved directly
      dinv_from_stencil<W>(grids_[l], lev_[l].st, 1.0, lev_[l].dinv, st_);
      if (gs_) {
        omega_[l] = 1.0;
        continue;
      }
      double lam = 0.0;
      HMG_TRY(estimate_lambda(l, &lam));
      lambda_[l] = lam;
      omega_[l] = omega_for(lam);
      dinv_from_stencil<W>(grids_[l], lev_[l].st, omega_[l], lev_[l].dinv, st_);
    }
    if (L == 1) {
      stencil_level0<T>(g0, s_, K0dev_, st0_, st_);
      dense_from_stencil<T>(g0, st0_, Ainv_, st_);
    } else {
      dense_from_stencil<W>(grids_[L - 1], lev_[L - 1].st, Ainv_, st_);
    }
    gauss_jordan_inverse(ncdof_, Ainv_, st_);
    double ssum = 0.0;
    (void)hipMemcpyAsync(&ssum, misc_, sizeof(double), hipMemcpyDeviceToHost, st_);
    if (hipStreamSynchronize(st_) != hipSuccess) return check_hip("set_density assembly");
    HMG_TRY(check_hip("set_density"));
    mean_s_ = ssum / (double)g0.n;
    have_density_ = true;
    have_solution_ = false;  // x_ stays as the start of an init = 1 solve
    return Status{};
  }

  Status solve(double tol, int max_iter, int init, const void* u0, int iters[6],
               double relres[6]) override {
    fp16_ready_ = false;
    if (!have_density_) return fail(HMG_E_STATE, "hmg_set_density has not been called");
    if (!(tol > 0.0) || max_iter <= 0 || init < 0 || init > 2 || (init == 2 && !u0))
      return fail(HMG_E_INVALID, "bad solve arguments (tol %g, max_iter %d, init %d)", tol,
                  max_iter, init);
    if (init == 1 && !have_iterate_) init = 0;
    const Grid& g0 = grids_[0];
    const int64_t F = (int64_t)NCASE * 3 * g0.n;
    const int64_t cs = 3 * g0.n;
    Op0Launch<T> L0{g0, mk_, s_, st_};
    Op0Launch<double> L64{g0, mk64_, s64_, st_};
    const double lam1 = cfg_.nu / ((1 + cfg_.nu) * (1 - 2 * cfg_.nu));
    const double mu1 = 1.0 / (2 * (1 + cfg_.nu));
    const double eps_abs = 1e-12 * std::sqrt((double)g0.n) * (lam1 + 2 * mu1) * mean_s_;

    if (init == 0) vec_fill<double>(x_, F, 0.0, st_);
    if (init == 2) vec_convert<T, double>(x_, (const T*)u0, F, st_);
    vec_fill<T>(pa_, F, T(0), st_);
    scal_set_all_active(scal_, st_);
    int nb = 0;
    // r = f - K x with f and K x in FP64 (f alone for a zero start).
    if (init == 0) {
      forcing<T>(g0, tpl64_, s64_, r_, part_, &nb, st_);
      fin_sum(part_, S_FF, nb, scal_, true, st_);
      (void)hipMemcpyAsync(scal_ + S_RR * 8, scal_ + S_FF * 8, sizeof(double) * 8,
                           hipMemcpyDeviceToDevice, st_);
    } else {
      op0_force_residual<T>(L64, tplg_, x_, r_, nullptr, part_, &nb);
      fin_sum(part_, S_FF, nb, scal_, true, st_);
      fin_sum(part_, S_TRUE, nb, scal_, true, st_);
      (void)hipMemcpyAsync(scal_ + S_RR * 8, scal_ + S_TRUE * 8, sizeof(double) * 8,
                           hipMemcpyDeviceToDevice, st_);
    }
    residual_mean(scal_);
    fin_init(scal_, eps_abs, tol, st_);
    HMG_TRY(read_scal(scal_, hscal_));
    bool active[NCASE];
    int it_count[NCASE];
    for (int c = 0; c < NCASE; ++c) {
      active[c] = hscal_[S_ACTIVE * 8 + c] != 0.0;
      last_true_[c] = std::sqrt(hscal_[S_RR * 8 + c]);
      it_count[c] = 0;
      if (hscal_[S_TRIVIAL * 8 + c] != 0.0) vec_fill<double>(x_ + c * cs, cs, 0.0, st_);
    }
    // Directions rotate through NB buffers: buf[ib] holds the newest one (the
    // matvec's p_old), buf[ib - j] the (j+1)-th newest.
    constexpr int NB = 4;
    T* buf[NB] = {pa_, pb_, pc_, pd_};
    int ib = 0;
    active_count_ = count(active);
    if (any(active)) {
      HMG_TRY(vcycle_apply(r_, z_, nullptr, scal_, &nb));
      fin_sum(part_, S_RZNEW, nb, scal_, false, st_);
      (void)hipMemcpyAsync(scal_ + S_RZ * 8, scal_ + S_RZNEW * 8, sizeof(double) * 8,
                           hipMemcpyDeviceToDevice, st_);
    }
    int it = 0;
    // Directions whose x += alpha p is still owed: the npend newest ones,
    // buf[ib - j] with its alpha in slot S_XALPHA + j (npend <= NB - 1).
    int npend = 0;
    auto pending_dirs = [&](const T** pend) {
      for (int j = 0; j < npend; ++j) pend[j] = buf[(ib - j + NB) % NB];
    };
    auto flush = [&]() {
      if (npend > 0) {
        const T* pend[NB - 1];
        pending_dirs(pend);
        vec_flush_x<T>(g0, x_, pend, npend, scal_, st_);
      }
      npend = 0;
    };
    while (any(active) && it < max_iter) {
      ++it;
      const double nact = (double)count(active), vn = (double)g0.n, TB = sizeof(T), VB = sizeof(V);
      T* pold = buf[ib];
      T* pnew = buf[(ib + 1) % NB];  // held p_{k-NB}, whose x term is no longer owed
      clock.timed(HMG_K_MATVEC, vn * (nact * 12 * TB + TB), st_, [&] {
        op0_matvec_p<T, T>(L0, z_, pold, pnew, q_, scal_, part_, &nb);
      });
      fin_sum(part_, S_PQ, nb, scal_, false, st_);
      fin_alpha(scal_, st_);
      // x advances every NB-th iteration, by alpha_{k-NB+1} p_{k-NB+1} + .. +
      // alpha_k p_k (all NB directions are still in the p buffers): the update
      // pass moves 60 B per vertex and case on average instead of 96 for
      // advancing x every iteration.  A recomputation of f - K x and the end of
      // the solve first flush the pending terms.
      const bool defer = npend < NB - 1;
      clock.timed(HMG_K_UPDATE, vn * nact * (defer ? 9 * TB : 48 + 3 * (NB + 3) * TB), st_, [&] {
        const T* pend[NB - 1];
        pending_dirs(pend);
        vec_update_r4<T>(g0, x_, pend, defer ? 0 : npend, pnew, r_, q_, scal_, part_, &nb, st_);
      });
      if (defer) {
        // shift the pending alphas one slot older, then the new one into S_XALPHA
        for (int j = npend; j > 0; --j)
          (void)hipMemcpyAsync(scal_ + (S_XALPHA + j) * 8, scal_ + (S_XALPHA + j - 1) * 8,
                               sizeof(double) * 8, hipMemcpyDeviceToDevice, st_);
        (void)hipMemcpyAsync(scal_ + S_XALPHA * 8, scal_ + S_ALPHA * 8, sizeof(double) * 8,
                             hipMemcpyDeviceToDevice, st_);
        ++npend;
      } else {
        npend = 0;
      }
      fin_sum(part_, S_RR, nb, scal_, false, st_);
      fin_mean(part_, nb, g0.n, scal_, st_);
      ib = (ib + 1) % NB;
      for (int c = 0; c < NCASE; ++c) it_count[c] += active[c] ? 1 : 0;
      HMG_TRY(read_scal(scal_, hscal_));
      bool check[NCASE], event[NCASE];
      bool anycheck = false;
      const bool replace = cfg_.replace_every > 0 && it % cfg_.replace_every == 0;
      for (int c = 0; c < NCASE; ++c) {
        const double rn = std::sqrt(hscal_[S_RR * 8 + c]);
        // recompute when the recursive residual claims convergence or has
        // dropped 100x below the last recomputed one, and every
        // replace_every iterations.  The recomputed residual replaces the
        // recursive one and the search direction is kept (reliable update);
        // only the bf16 forms, whose rounded preconditioner makes the
        // recursion drift further, restart the direction after an event.
        // A restart would discard the Krylov space built so far: in FP32 it
        // cost up to 20 % more iterations on the 512^3 benchmark cell.
        event[c] = active[c] && (rn <= hscal_[S_THRESH * 8 + c] || rn <= 1e-2 * last_true_[c]);
        check[c] = event[c] || (active[c] && replace);
        anycheck |= check[c];
      }
      if (anycheck) {
        // Confirm on the residual f - K x recomputed in FP64 before a case
        // stops; the recomputed residual also replaces the recursive one (it
        // is written over r of the checked cases: a case that stops no longer
        // needs r).
        flush();
        set_mask(aux_, check);
        clock.timed(HMG_K_TRUE_RESIDUAL, (double)g0.n * (count(check) * (24 + 3 * sizeof(T)) + 8),
                    st_, [&] { op0_force_residual<T>(L64, tplg_, x_, r_, aux_, part_, &nb); });
        fin_sum(part_, S_TRUE, nb, aux_, false, st_);
        HMG_TRY(read_scal(aux_, hscal_ + S_NSLOT * 8));
        const double* ha = hscal_ + S_NSLOT * 8;
        bool restart[NCASE];
        for (int c = 0; c < NCASE; ++c) {
          restart[c] = false;
          if (!check[c]) continue;
          const double tr = std::sqrt(ha[S_TRUE * 8 + c]);
          last_true_[c] = tr;
          if (tr <= hscal_[S_THRESH * 8 + c])
            active[c] = false;
          else
            restart[c] = event[c] && kPR;
        }
        set_mask(scal_, active);
        set_slot(scal_, S_RESTART, restart);
        set_slot(scal_, S_REPLACED, check);
        residual_mean(scal_);
      }
      if (!any(active)) break;
      active_count_ = count(active);
      HMG_TRY(vcycle_apply(r_, z_, kPR ? q_ : nullptr, scal_, &nb));
      fin_sum(part_, S_RZNEW, nb, scal_, false, st_);
      if (kPR) fin_sum(part_, S_QZ, nb, scal_, false, st_);
      fin_beta(scal_, kPR, st_);
    }
    flush();
    // Zero-mean solution, recomputed final residuals.
    vec_mean_partial<double>(g0, x_, part_, &nb, st_);
    fin_mean(part_, nb, g0.n, aux_, st_);
    vec_mean_subtract<double>(g0, x_, aux_, st_);
    scal_set_all_active(aux_, st_);
    op0_force_residual<T>(L64, tplg_, x_, r_, aux_, part_, &nb);
    fin_sum(part_, S_FF, nb, aux_, true, st_);
    fin_sum(part_, S_TRUE, nb, aux_, true, st_);
    HMG_TRY(read_scal(aux_, hscal_ + S_NSLOT * 8));
    const double* ha = hscal_ + S_NSLOT * 8;
    for (int c = 0; c < NCASE; ++c) {
      iters[c] = it_count[c];
      const bool trivial = hscal_[S_TRIVIAL * 8 + c] != 0.0;
      const double ff = ha[S_FF * 8 + c];
      relres[c] = trivial || ff <= 0.0 ? 0.0 : std::sqrt(ha[S_TRUE * 8 + c] / ff);
    }
    have_solution_ = true;
    have_iterate_ = true;
    fp16_ready_ = false;
    if (any(active))
      return fail(HMG_E_NOT_CONVERGED, "max_iter %d reached before rel_tol %g", max_iter, tol);
    return Status{};
  }

  // FP16 copy of the solution for C^H and the sensitivities (Sec. 4.3), kept in
  // the residual buffer, which the solve no longer needs; FP32-storage forms only.
  const f16* fp16_solution() {
    if (!fp16_ready_) {
      vec_convert<double, f16>(reinterpret_cast<f16*>(r_), x_, (int64_t)NCASE * 3 * grids_[0].n,
                               st_);
      fp16_ready_ = true;
    }
    return reinterpret_cast<const f16*>(r_);
  }
  bool use_fp16() const { return cfg_.post_fp16 != 0 && sizeof(T) == sizeof(float); }

  Status elastic(double C[36]) override {
    if (!have_solution_) return fail(HMG_E_STATE, "hmg_solve_cases has not been called");
    int nb = 0;
    if (use_fp16())
      elastic_partials<float, f16>(grids_[0], cast_mode_f(mk64_), chh32_, (const float*)s_,
                                   fp16_solution(), part_, &nb, st_);
    else
      elastic_partials<double, double>(grids_[0], mk64_, chh64_, s64_, x_, part_, &nb, st_);
    elastic_finalize(part_, nb, grids_[0].n, misc_, st_);
    (void)hipMemcpyAsync(C, misc_, sizeof(double) * 36, hipMemcpyDeviceToHost, st_);
    if (hipStreamSynchronize(st_) != hipSuccess) return check_hip("elastic_tensor");
    return check_hip("elastic_tensor");
  }

  Status sens(const double Wt[36], float* out) override {
    if (!have_solution_) return fail(HMG_E_STATE, "hmg_solve_cases has not been called");
    double w21[21];
    int t = 0;
    for (int j = 0; j < NCASE; ++j)
      for (int i = 0; i <= j; ++i)
        w21[t++] = (i == j) ? Wt[i * 6 + i] : Wt[i * 6 + j] + Wt[j * 6 + i];
    (void)hipMemcpyAsync(misc_ + 36, w21, sizeof(double) * 21, hipMemcpyHostToDevice, st_);
    const double coef = cfg_.penal * (cfg_.E0 - cfg_.Emin) / (double)grids_[0].n;
    if (use_fp16())
      sensitivity<float, f16>(grids_[0], cast_mode_f(mk64_), chh32_, (const float*)rho_,
                              fp16_solution(), misc_ + 36, coef, cfg_.penal, out, st_);
    else
      sensitivity<double, double>(grids_[0], mk64_, chh64_, rho64_, x_, misc_ + 36, coef,
                                  cfg_.penal, out, st_);
    // the host array w21 must outlive the copy
    if (hipStreamSynchronize(st_) != hipSuccess) return check_hip("sensitivity");
    return check_hip("sensitivity");
  }

  Status get_disp(void* u) override {
    if (!have_solution_ && !have_iterate_)
      return fail(HMG_E_STATE, "neither hmg_solve_cases nor an accepted warm start has run");
    vec_convert<double, T>((T*)u, x_, (int64_t)NCASE * 3 * grids_[0].n, st_);
    return check_hip("get_displacement");
  }

  // The inspection entry points below take and return fields of type T; with
  // a narrower storage type the coarse-level data pass through conversions.
  Status apply_op(int level, const void* u, void* y) override {
    if (!have_density_) return fail(HMG_E_STATE, "hmg_set_density has not been called");
    if (level == 0) {
      Op0Launch<T> L0{grids_[0], mk_, s_, st_};
      op0_apply<T>(L0, (const T*)u, (T*)y, nullptr);
    } else {
      const int64_t Fl = (int64_t)NCASE * 3 * grids_[level].n;
      vec_convert<T, V>(lev_[level].z, (const T*)u, Fl, st_);
      kc_apply<V, W>(grids_[level], lev_[level].st, lev_[level].z, lev_[level].t, st_);
      vec_convert<V, T>((T*)y, lev_[level].t, Fl, st_);
    }
    return check_hip("apply_operator");
  }

  Status get_stencil(int level, void* out) override {
    if (!have_density_) return fail(HMG_E_STATE, "hmg_set_density has not been called");
    if (level == 0)
      stencil_level0<T>(grids_[0], s_, K0dev_, (T*)out, st_);
    else
      vec_convert<W, T>((T*)out, lev_[level].st, 243 * grids_[level].n, st_);
    return check_hip("get_stencil");
  }

  Status loads(void* f) override {
    if (!have_density_) return fail(HMG_E_STATE, "hmg_set_density has not been called");
    forcing<T>(grids_[0], tpl64_, s64_, (T*)f, Partials{}, nullptr, st_);
    return check_hip("load_vectors");
  }

  Status vcycle(const void* r, void* z) override {
    if (!have_density_) return fail(HMG_E_STATE, "hmg_set_density has not been called");
    scal_set_all_active(aux_, st_);
    active_count_ = NCASE;
    int nb = 0;
    vec_mean_partial<T>(grids_[0], (const T*)r, part_, &nb, st_);
    fin_mean(part_, nb, grids_[0].n, aux_, st_);
    HMG_TRY(vcycle_apply((const T*)r, (T*)z, nullptr, aux_, &nb));
    return check_hip("vcycle");
  }

  Status transfer(int level, int dir, const void* in, void* out) override {
    const Grid& gf = grids_[level];
    const Grid& gc = grids_[level + 1];
    const int64_t Ff = (int64_t)NCASE * 3 * gf.n, Fc = (int64_t)NCASE * 3 * gc.n;
    if (dir == 0) {
      vec_convert<T, V>(t_, (const T*)in, Ff, st_);
      restrict_to<V>(gf, gc, t_, lev_[level + 1].r, nullptr, st_);
      vec_convert<V, T>((T*)out, lev_[level + 1].r, Fc, st_);
    } else {
      if (reinterpret_cast<uintptr_t>(out) % (2 * sizeof(T)) != 0)
        return fail(HMG_E_INVALID, "transfer output must be aligned to %d bytes",
                    (int)(2 * sizeof(T)));
      vec_convert<T, V>(lev_[level + 1].z, (const T*)in, Fc, st_);
      prolong_add<T, V>(gf, gc, (T*)out, lev_[level + 1].z, nullptr, true, st_);
    }
    return check_hip("transfer");
  }

 private:
  struct Lev {
    W* st = nullptr;
    W* dinv = nullptr;
    V* r = nullptr;
    V* z = nullptr;
    V* t = nullptr;
    double* ms = nullptr;  // FP64 per-component means of r at this level (slots S_MEAN*)
  };

  static ModeK<T> cast_mode(const ModeK<double>& m) {
    return ModeK<T>{(T)m.ab, (T)m.b, (T)m.cs, (T)m.p, (T)m.q, (T)m.fg, (T)m.g, (T)m.z};
  }
  static ModeK<float> cast_mode_f(const ModeK<double>& m) {
    return ModeK<float>{(float)m.ab, (float)m.b, (float)m.cs, (float)m.p,
                        (float)m.q,  (float)m.fg, (float)m.g, (float)m.z};
  }
  // Damping of block Jacobi on a level whose spectrum bound is lam: 1.6/lam
  // (near the smoothing optimum 2/(lam + lam/4)); a configured omega is used
  // when given but capped at 1.9/lam so the smoother stays convergent.
  double omega_for(double lam) const {
    return cfg_.omega > 0.0 ? std::min(cfg_.omega, 1.9 / lam) : 1.6 / lam;
  }

  // Largest eigenvalue of D^-1 K_l by power iteration (six start vectors; the
  // largest Rayleigh estimate, increased by 5 % because power iteration
  // approaches it from below).  Expects lev_[l].dinv to hold D^-1 (omega 1).
  Status estimate_lambda(int l, double* out) {
    Lev& lv = lev_[l];
    const Grid& g = grids_[l];
    const int64_t F = (int64_t)NCASE * 3 * g.n;
    vec_pattern<V>(lv.z, F, st_);
    for (int k = 0; k < 15; ++k) {
      kc_apply<V, W>(g, lv.st, lv.z, lv.t, st_);                        // y = K x
      vec_jacobi0<V, W, V>(g, lv.t, lv.dinv, lv.z, nullptr, nullptr, st_);  // x = D^-1 y
    }
    kc_apply<V, W>(g, lv.st, lv.z, lv.r, st_);
    scal_set_all_active(aux_, st_);
    int nb = 0;
    vec_dot_cases<V, V>(g, lv.z, lv.r, aux_, part_, S_PQ, &nb, st_);   // x^T K x
    fin_sum(part_, S_PQ, nb, aux_, true, st_);
    vec_dot_cases<V, V>(g, lv.z, lv.t, aux_, part_, S_RZ, &nb, st_);   // x^T D x
    fin_sum(part_, S_RZ, nb, aux_, true, st_);
    HMG_TRY(read_scal(aux_, hscal_ + S_NSLOT * 8));
    const double* ha = hscal_ + S_NSLOT * 8;
    double lam = 0.0;
    for (int c = 0; c < NCASE; ++c)
      if (ha[S_RZ * 8 + c] > 0.0) lam = std::max(lam, ha[S_PQ * 8 + c] / ha[S_RZ * 8 + c]);
    if (!(lam > 0.0) || !std::isfinite(lam))
      return fail(HMG_E_DEVICE, "spectral estimate failed on level %d", l);
    *out = 1.05 * lam;
    return Status{};
  }
  static int count(const bool* a) {
    int k = 0;
    for (int c = 0; c < NCASE; ++c) k += a[c] ? 1 : 0;
    return k;
  }
  static bool any(const bool* a) {
    for (int c = 0; c < NCASE; ++c)
      if (a[c]) return true;
    return false;
  }

  Status read_scal(const double* dev, double* host) {
    (void)hipMemcpyAsync(host, dev, sizeof(double) * S_NSLOT * 8, hipMemcpyDeviceToHost, st_);
    if (hipStreamSynchronize(st_) != hipSuccess) return check_hip("scalar readback");
    return check_hip("scalar readback");
  }

  // Writes a per-case 0/1 mask into one slot of a device scalar array.
  void set_slot(double* scal, int slot, const bool* on) {
    double* h = hstage_;
    for (int c = 0; c < 8; ++c) h[c] = (c < NCASE && on[c]) ? 1.0 : 0.0;
    (void)hipMemcpyAsync(scal + slot * 8, h, sizeof(double) * 8, hipMemcpyHostToDevice, st_);
    (void)hipStreamSynchronize(st_);
  }
  void set_mask(double* scal, const bool* on) { set_slot(scal, S_ACTIVE, on); }

  // Means of r per case and component (FP64) into slots S_MEAN* of scal.
  void residual_mean(double* scal) {
    int nb = 0;
    vec_mean_partial<T>(grids_[0], r_, part_, &nb, st_);
    fin_mean(part_, nb, grids_[0].n, scal, st_);
  }

  // zout = M r0: one symmetric V(1,1) cycle (Alg. 1) started from zero, with
  // the translation component of every residual removed in FP64 before the
  // block-Jacobi smoother and the coarsest solve.  scal supplies the active
  // cases and the means of r0; per-block partials of (r0 - m).zout are left in
  // slot S_RZNEW.  Work buffers: w0_ (pre-smoothed z0, aliases q_) and t_.
  Status vcycle_apply(const T* r0, T* zout, const T* qpr, const double* scal, int* nb) {
    const int L = levels();
    const Grid& g0 = grids_[0];
    if (L == 1) {
      coarse_solve<T, T>(g0, Ainv_, r0, zout, scal, st_);
      if (qpr) vec_dot_cases<T, T>(g0, qpr, zout, scal, part_, S_QZ, nb, st_);
      vec_dot_cases<T, T>(g0, r0, zout, scal, part_, S_RZNEW, nb, st_);
      return check_hip("vcycle");
    }
    Op0Launch<T> L0{g0, mk_, s_, st_};
    const double vn = (double)g0.n, TB = sizeof(T), VB = sizeof(V), nact = active_count_;
    if (gs_) {
      // forward sweep from zero, residual + restriction, coarse correction,
      // backward sweep with the partial dot products of the result
      // Algorithmic bytes of a sweep per vertex and active case: r read, z
      // written, and (backward) z read once; plus s per vertex.
      clock.timed(HMG_K_GS_FORWARD, vn * (nact * 6 * TB + TB), st_, [&] {
        gs0_sweep<T>(g0, ec_.kv, s_, r0, scal, zout, nullptr, scal, part_, true, true, nullptr,
                     st_);
      });
      clock.timed(HMG_K_RESIDUAL, vn * (nact * 3 * (2 * TB + VB) + TB), st_,
                  [&] { op0_residual<T, V>(L0, r0, zout, t_, scal); });
      restrict_to<V>(g0, grids_[1], t_, lev_[1].r, scal, st_);
      descend(1, scal);
      if (L == 2)
        prolong_add<T, T>(g0, grids_[1], zout, zc_, scal, false, st_);
      else
        prolong_add<T, V>(g0, grids_[1], zout, lev_[1].z, scal, false, st_);
      clock.timed(HMG_K_GS_BACKWARD, vn * (nact * 3 * (3 * TB + (qpr ? TB : 0)) + TB), st_, [&] {
        gs0_sweep<T>(g0, ec_.kv, s_, r0, scal, zout, qpr, scal, part_, false, false, nb, st_);
      });
      return check_hip("vcycle");
    }
    clock.timed(HMG_K_JACOBI, vn * (nact * 6 * TB + TB), st_, [&] {
      jacobi0_level0<T>(g0, s_, BlockDiag0{ec_.dd, ec_.oo, omega_[0]}, r0, w0_, scal, scal, st_);
    });
    clock.timed(HMG_K_RESIDUAL, vn * (nact * 3 * (2 * TB + VB) + TB), st_,
                [&] { op0_residual<T, V>(L0, r0, w0_, t_, scal); });
    restrict_to<V>(g0, grids_[1], t_, lev_[1].r, scal, st_);
    descend(1, scal);
    const double cb = (double)grids_[1].n * nact * 3 * (L == 2 ? TB : VB);
    clock.timed(HMG_K_PROLONG, vn * nact * 6 * TB + cb, st_, [&] {
      if (L == 2)
        prolong_add<T, T>(g0, grids_[1], w0_, zc_, scal, false, st_);
      else
        prolong_add<T, V>(g0, grids_[1], w0_, lev_[1].z, scal, false, st_);
    });
    clock.timed(HMG_K_POST_SMOOTH, vn * (nact * 3 * (3 * TB + (qpr ? TB : 0)) + TB), st_, [&] {
      op0_post_smooth<T, V>(L0, w0_, r0, BlockDiag0{ec_.dd, ec_.oo, omega_[0]}, zout, qpr, scal,
                            part_, nb);
    });
    return check_hip("vcycle");
  }

  void descend(int l, const double* scal) {
    const int L = levels();
    Lev& lv = lev_[l];
    const Grid& g = grids_[l];
    if (l == L - 1) {
      coarse_solve<V, T>(g, Ainv_, lv.r, zc_, scal, st_);
      return;
    }
    int nb = 0;
    vec_mean_partial<V>(g, lv.r, part_, &nb, st_);
    fin_mean(part_, nb, g.n, lv.ms, st_);
    if (gs_) {
      gsc_sweep<V, W>(g, lv.st, lv.dinv, lv.r, lv.ms, lv.z, scal, true, true, st_);
      kc_residual<V, W>(g, lv.st, lv.z, lv.r, lv.t, scal, lv.ms, st_);
      restrict_to<V>(g, grids_[l + 1], lv.t, lev_[l + 1].r, scal, st_);
      descend(l + 1, scal);
      if (l + 1 == L - 1)
        prolong_add<V, T>(g, grids_[l + 1], lv.z, zc_, scal, false, st_);
      else
        prolong_add<V, V>(g, grids_[l + 1], lv.z, lev_[l + 1].z, scal, false, st_);
      gsc_sweep<V, W>(g, lv.st, lv.dinv, lv.r, lv.ms, lv.z, scal, false, false, st_);
      return;
    }
    vec_jacobi0<V, W, V>(g, lv.r, lv.dinv, lv.z, scal, lv.ms, st_);
    kc_residual<V, W>(g, lv.st, lv.z, lv.r, lv.t, scal, lv.ms, st_);
    restrict_to<V>(g, grids_[l + 1], lv.t, lev_[l + 1].r, scal, st_);
    descend(l + 1, scal);
    if (l + 1 == L - 1)
      prolong_add<V, T>(g, grids_[l + 1], lv.z, zc_, scal, false, st_);
    else
      prolong_add<V, V>(g, grids_[l + 1], lv.z, lev_[l + 1].z, scal, false, st_);
    kc_smooth<V, W>(g, lv.st, lv.z, lv.r, lv.dinv, lv.t, scal, lv.ms, st_);
    std::swap(lv.z, lv.t);
  }

  hmg_config cfg_;
  hipStream_t st_;
  ElementConsts ec_;
  std::vector<Grid> grids_;
  DeviceArena arena_;
  ModeK<T> mk_{};
  ModeK<double> mk64_{};
  LoadTpl<T> tpl_{};
  LoadTpl<double> tpl64_{};
  double* tplg_ = nullptr;  // tpl64_ in device memory (FP64 residual)
  LoadTpl<double> chh64_{};
  LoadTpl<float> chh32_{};
  bool fp16_ready_ = false;  // r_ holds the FP16 cast of the current solution
  T *s_ = nullptr, *rho_ = nullptr;
  double* s64_ = nullptr;    // FP64 copies used by the residual recomputation and C^H
  double* rho64_ = nullptr;
  double* x_ = nullptr;      // iterate kept in FP64
  T* r_ = nullptr;  // level-0 residual (arithmetic type)
  T* z_ = nullptr;  // preconditioned residual
  V* t_ = nullptr;  // V-cycle work: level-0 residual after pre-smoothing
  T *pa_ = nullptr, *pb_ = nullptr, *pc_ = nullptr, *pd_ = nullptr;
  T* q_ = nullptr;   // q = K p
  T* w0_ = nullptr;  // V-cycle level-0 correction (the plain forms alias q_)
  T* zc_ = nullptr;  // coarsest-level correction
  T* st0_ = nullptr;
  std::vector<Lev> lev_;
  double* Ainv_ = nullptr;
  int ncdof_ = 0;
  Partials part_{};
  int stride_ = 0;
  double *scal_ = nullptr, *aux_ = nullptr, *misc_ = nullptr;
  double *K0dev_ = nullptr, *msig_ = nullptr;
  double* msig4_ = nullptr;          // non-dyadic first step: 64 sub-element matrices
  std::vector<double> msig4_host_;   // their host copy (outlives the upload)
  bool gs_ = cfg_.smoother == 1;  // eight-colour symmetric Gauss-Seidel instead of damped Jacobi
  int* bad_ = nullptr;
  double* hscal_ = nullptr;  // pinned: device scalars read back (main, aux)
  double* hstage_ = nullptr; // pinned: staging for host-to-device masks
  double mean_s_ = 1.0;
  int active_count_ = NCASE;
  std::vector<double> omega_;   // block-Jacobi damping per level
  std::vector<double> lambda_;  // spectral bound of D^-1 K per level
  double last_true_[NCASE] = {};  // last recomputed residual norm per case
  bool have_density_ = false;
  bool have_solution_ = false;  // x_ solves the current density (C^H, sensitivities)
  bool have_iterate_ = false;   // x_ holds a solution or an accepted guess (init = 1)
  float* nnbuf_ = nullptr;      // warm start: network input and output (<= 64^3)
  double raw_relres_ = 0.0;     // warm start: relative residual before the correction cycle
  double guess_scale_[NCASE] = {};  // warm start: energy-optimal scale of each case's guess
};


// ---------------------------------------------------------------- batched cells
// Many independent cells (each with its own hierarchy) solved in lockstep: one
// PCG iteration is two captured graphs.  The level-0 passes (matvec, update,
// Jacobi, residual, post-smoothing) are single launches over all cells (a
// persistent grid over the cells' tiles, largest cells first); the coarse
// levels and the scalar finalizers are per-cell launches inside the graphs.
// The host reads the scalars of every cell once per iteration to decide
// convergence and residual recomputations, exactly as in a single solve.
class BatchSolver {
 public:
  using S = Solver<float, float, float>;
  BatchSolver(hipStream_t st) : st_(st) {}
  ~BatchSolver() {
    free_plans();
    for (auto* d : pw_) if (d) (void)hipFree(d);
    if (hsc_) (void)hipHostFree(hsc_);
  }

  std::vector<std::unique_ptr<S>> cells;
  std::vector<hmg_config> cfgs;
  std::vector<int> lz;  // tuned z-chunk per cell (0 = default)
  int grid = 0;         // persistent grid of the level-0 passes (0 = one block per item)

  Status init() {
    if (hipHostMalloc((void**)&hsc_, sizeof(double) * S_NSLOT * 8 * cells.size()) != hipSuccess)
      return fail(HMG_E_OOM, "pinned host allocation failed");
    lz.assign(cells.size(), 0);
    // largest cells first: their tiles head the item list of every pass
    order_.resize(cells.size());
    for (size_t i = 0; i < cells.size(); ++i) order_[i] = (int)i;
    std::stable_sort(order_.begin(), order_.end(), [&](int a, int b) {
      return cells[a]->grids_[0].n > cells[b]->grids_[0].n;
    });
    return Status{};
  }

  // Plans cover the live cells (those with an unconverged case), largest
  // first; a solve rebuilds them whenever a cell finishes, so that finished
  // cells cost no launches or items.
  Status build_plans() {
    free_plans();
    if (live_.empty()) live_ = order_;
    const int B = (int)live_.size();
    std::vector<Op0BatchCell> mv[2], rs, ps;
    std::vector<PwBatchCell> up[2], jc;
    nblk_ = 1;
    for (int c : live_) nblk_ = std::max(nblk_, vec_blocks_for(cells[c]->grids_[0].n));
    for (int c : live_) {
      S& X = *cells[c];
      const Grid& g = X.grids_[0];
      if (op0_tiles_per_case(g, lz[c]) > X.stride_)
        return fail(HMG_E_INVALID, "z-chunk %d gives more tiles than the partial buffers hold", lz[c]);
      for (int par = 0; par < 2; ++par) {
        float* pold = par ? X.pb_ : X.pa_;
        float* pnew = par ? X.pa_ : X.pb_;
        mv[par].push_back({g, lz[c], X.s_, X.z_, pold, nullptr, nullptr, pnew, X.q_, X.scal_,
                           X.part_});
        up[par].push_back({g, X.x_, pnew, X.r_, X.q_, nullptr, nullptr, X.scal_, X.part_});
      }
      rs.push_back({g, lz[c], X.s_, X.r_, X.w0_, nullptr, nullptr, X.t_, nullptr, X.scal_,
                    Partials{}});
      ps.push_back({g, lz[c], X.s_, X.w0_, X.r_, nullptr, nullptr, X.z_, nullptr, X.scal_,
                    X.part_, {X.ec_.dd, X.ec_.oo, X.omega_[0]}});
      jc.push_back({g, nullptr, nullptr, X.r_, nullptr, X.s_, X.w0_, X.scal_, Partials{},
                    {X.ec_.dd, X.ec_.oo, X.omega_[0]}});
    }
    for (int par = 0; par < 2; ++par) {
      mvp_[par] = op0_batch_plan(OP0B_MATVEC, mv[par].data(), B, grid, st_);
      if (!mvp_[par]) return fail(HMG_E_OOM, "batch plan allocation failed");
    }
    rsp_ = op0_batch_plan(OP0B_RESIDUAL, rs.data(), B, grid, st_);
    psp_ = op0_batch_plan(OP0B_POST_SMOOTH, ps.data(), B, grid, st_);
    if (!rsp_ || !psp_) return fail(HMG_E_OOM, "batch plan allocation failed");
    auto upload = [&](const std::vector<PwBatchCell>& v, PwBatchCell** d) -> bool {
      if (!*d && hipMalloc((void**)d, sizeof(PwBatchCell) * v.size()) != hipSuccess) return false;
      (void)hipMemcpyAsync(*d, v.data(), sizeof(PwBatchCell) * v.size(), hipMemcpyHostToDevice,
                           st_);
      return true;
    };
    if (!upload(up[0], &pw_[0]) || !upload(up[1], &pw_[1]) || !upload(jc, &pw_[2]))
      return fail(HMG_E_OOM, "batch descriptor allocation failed");
    (void)hipStreamSynchronize(st_);
    return check_hip("batch plans");
  }

  // Times the batched matvec for candidate z-chunks (per cell size) and
  // persistent grid sizes; keeps the fastest.
  Status tune(int* grid_out, int* lz_out) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    auto time_mv = [&]() -> double {
      for (int w = 0; w < 2; ++w) launch_matvec(0);
      (void)hipEventRecord(a, st_);
      for (int k = 0; k < 5; ++k) launch_matvec(0);
      (void)hipEventRecord(b, st_);
      (void)hipEventSynchronize(b);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, a, b);
      return ms / 5.0;
    };
    for (auto& X : cells) scal_set_all_active(X->scal_, st_);
    live_ = order_;
    // z-chunk, one size class at a time (the others keep their current value)
    std::vector<int> sizes;
    for (auto& X : cells) sizes.push_back(X->grids_[0].nz);
    std::sort(sizes.begin(), sizes.end());
    sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
    for (int nz : sizes) {
      double best = 1e30;
      int bestlz = 0;
      for (int cand : {0, 4, 8, 16, 32, 64}) {
        if (cand > nz) continue;
        for (size_t c = 0; c < cells.size(); ++c)
          if (cells[c]->grids_[0].nz == nz) lz[c] = cand;
        Status st = build_plans();
        if (st.code != HMG_OK) continue;
        const double t = time_mv();
        if (t < best) {
          best = t;
          bestlz = cand;
        }
      }
      for (size_t c = 0; c < cells.size(); ++c)
        if (cells[c]->grids_[0].nz == nz) lz[c] = bestlz;
    }
    double best = 1e30;
    int bestg = 0;
    for (int cand : {0, 512, 1024, 2048, 4096}) {
      grid = cand;
      HMG_TRY(build_plans());
      const double t = time_mv();
      if (t < best) {
        best = t;
        bestg = cand;
      }
    }
    grid = bestg;
    HMG_TRY(build_plans());
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *grid_out = grid;
    for (size_t c = 0; c < cells.size(); ++c) lz_out[c] = lz[c];
    tuned_ms_ = best;
    return check_hip("batch tune");
  }

  Status solve(double tol, int max_iter, int* iters, double* relres) {
    const int B = (int)cells.size();
    for (auto& X : cells)
      if (!X->have_density_) return fail(HMG_E_STATE, "a cell has no density");
    if (!mvp_[0] || live_.size() != cells.size()) {
      live_ = order_;
      HMG_TRY(build_plans());
    }
    destroy_graphs();
    std::vector<std::array<bool, NCASE>> active(B);
    std::vector<std::array<int, NCASE>> count(B);
    // per-cell start: x = 0, r = f, thresholds (as in a single solve)
    for (int c = 0; c < B; ++c) {
      S& X = *cells[c];
      const Grid& g0 = X.grids_[0];
      const int64_t F = (int64_t)NCASE * 3 * g0.n;
      const double lam1 = X.cfg_.nu / ((1 + X.cfg_.nu) * (1 - 2 * X.cfg_.nu));
      const double mu1 = 1.0 / (2 * (1 + X.cfg_.nu));
      const double eps_abs = 1e-12 * std::sqrt((double)g0.n) * (lam1 + 2 * mu1) * X.mean_s_;
      vec_fill<double>(X.x_, F, 0.0, st_);
      vec_fill<float>(X.pa_, F, 0.f, st_);
      scal_set_all_active(X.scal_, st_);
      int nb = 0;
      forcing<float>(g0, X.tpl64_, X.s64_, X.r_, X.part_, &nb, st_);
      fin_sum(X.part_, S_FF, nb, X.scal_, true, st_);
      (void)hipMemcpyAsync(X.scal_ + S_RR * 8, X.scal_ + S_FF * 8, sizeof(double) * 8,
                           hipMemcpyDeviceToDevice, st_);
      X.residual_mean(X.scal_);
      fin_init(X.scal_, eps_abs, tol, st_);
    }
    HMG_TRY(read_all());
    for (int c = 0; c < B; ++c) {
      const double* h = hsc_ + (size_t)c * S_NSLOT * 8;
      for (int k = 0; k < NCASE; ++k) {
        active[c][k] = h[S_ACTIVE * 8 + k] != 0.0;
        count[c][k] = 0;
        cells[c]->last_true_[k] = std::sqrt(h[S_RR * 8 + k]);
      }
    }
    auto cell_live = [&](int c) {
      for (int k = 0; k < NCASE; ++k)
        if (active[c][k]) return true;
      return false;
    };
    // drops finished cells from the plans (and the captured graphs)
    auto refresh_live = [&]() -> Status {
      std::vector<int> nl;
      for (int c : live_)
        if (cell_live(c)) nl.push_back(c);
      if (nl.size() == live_.size() || nl.empty()) return Status{};
      live_ = nl;
      HMG_TRY(build_plans());
      return Status{};
    };
    HMG_TRY(refresh_live());
    vcycle();
    for (int c : live_) {
      S& X = *cells[c];
      fin_sum(X.part_, S_RZNEW, X.stride_tiles(lz[c]), X.scal_, false, st_);
      (void)hipMemcpyAsync(X.scal_ + S_RZ * 8, X.scal_ + S_RZNEW * 8, sizeof(double) * 8,
                           hipMemcpyDeviceToDevice, st_);
    }
    auto any_active = [&]() {
      for (int c = 0; c < B; ++c)
        for (int k = 0; k < NCASE; ++k)
          if (active[c][k]) return true;
      return false;
    };
    int it = 0;
    while (any_active() && it < max_iter) {
      ++it;
      HMG_TRY(run_graph(g1_[(it - 1) & 1], [&] { phase1((it - 1) & 1); }));
      HMG_TRY(read_all());
      for (int c = 0; c < B; ++c)
        for (int k = 0; k < NCASE; ++k) count[c][k] += active[c][k] ? 1 : 0;
      const bool replace = cfgs[0].replace_every > 0 && it % cfgs[0].replace_every == 0;
      for (int c : live_) HMG_TRY(check_cell(c, replace, active[c]));
      if (!any_active()) break;
      HMG_TRY(refresh_live());
      HMG_TRY(run_graph(g2_, [&] { phase2(); }));
    }
    for (int c = 0; c < B; ++c) {
      S& X = *cells[c];
      const Grid& g0 = X.grids_[0];
      int nb = 0;
      Op0Launch<double> L64{g0, X.mk64_, X.s64_, st_};
      vec_mean_partial<double>(g0, X.x_, X.part_, &nb, st_);
      fin_mean(X.part_, nb, g0.n, X.aux_, st_);
      vec_mean_subtract<double>(g0, X.x_, X.aux_, st_);
      scal_set_all_active(X.aux_, st_);
      op0_force_residual<float>(L64, X.tplg_, X.x_, X.r_, X.aux_, X.part_, &nb);
      fin_sum(X.part_, S_FF, nb, X.aux_, true, st_);
      fin_sum(X.part_, S_TRUE, nb, X.aux_, true, st_);
      HMG_TRY(X.read_scal(X.aux_, X.hscal_ + S_NSLOT * 8));
      HMG_TRY(X.read_scal(X.scal_, X.hscal_));
      const double* ha = X.hscal_ + S_NSLOT * 8;
      for (int k = 0; k < NCASE; ++k) {
        iters[c * NCASE + k] = count[c][k];
        const bool trivial = X.hscal_[S_TRIVIAL * 8 + k] != 0.0;
        const double ff = ha[S_FF * 8 + k];
        relres[c * NCASE + k] = trivial || ff <= 0.0 ? 0.0 : std::sqrt(ha[S_TRUE * 8 + k] / ff);
      }
      X.have_solution_ = true;
      X.have_iterate_ = true;
    }
    iters_run_ = it;
    if (any_active())
      return fail(HMG_E_NOT_CONVERGED, "max_iter %d reached before rel_tol %g", max_iter, tol);
    return Status{};
  }

  double tuned_ms() const { return tuned_ms_; }

 private:
  void launch_matvec(int par) { op0_batch_launch(mvp_[par], cells[0]->mk_, st_); }

  // matvec, alpha, update, residual norms and means (per parity of p)
  void phase1(int par) {
    launch_matvec(par);
    for (int c : live_) {
      S& X = *cells[c];
      fin_sum(X.part_, S_PQ, X.stride_tiles(lz[c]), X.scal_, false, st_);
      fin_alpha(X.scal_, st_);
    }
    update_batched(pw_[par], (int)live_.size(), nblk_, st_);
    for (int c : live_) {
      S& X = *cells[c];
      fin_sum(X.part_, S_RR, nblk_, X.scal_, false, st_);
      fin_mean(X.part_, nblk_, X.grids_[0].n, X.scal_, st_);
    }
  }
  // preconditioner and beta
  void phase2() {
    vcycle();
    for (int c : live_) {
      S& X = *cells[c];
      fin_sum(X.part_, S_RZNEW, X.stride_tiles(lz[c]), X.scal_, false, st_);
      fin_beta(X.scal_, false, st_);
    }
  }
  void vcycle() {
    jacobi0_batched(pw_[2], (int)live_.size(), nblk_, st_);
    op0_batch_launch(rsp_, cells[0]->mk_, st_);
    for (int c : live_) {
      S& X = *cells[c];
      const Grid& g0 = X.grids_[0];
      const int L = X.levels();
      if (L == 1) continue;  // one-level cells are not batched (rejected at creation)
      restrict_to<float>(g0, X.grids_[1], X.t_, X.lev_[1].r, X.scal_, st_);
      X.descend(1, X.scal_);
      if (L == 2)
        prolong_add<float, float>(g0, X.grids_[1], X.w0_, X.zc_, X.scal_, false, st_);
      else
        prolong_add<float, float>(g0, X.grids_[1], X.w0_, X.lev_[1].z, X.scal_, false, st_);
    }
    op0_batch_launch(psp_, cells[0]->mk_, st_);
  }

  Status check_cell(int c, bool replace, std::array<bool, NCASE>& active) {
    S& X = *cells[c];
    const double* h = hsc_ + (size_t)c * S_NSLOT * 8;
    bool check[NCASE], event[NCASE];
    bool anycheck = false;
    for (int k = 0; k < NCASE; ++k) {
      const double rn = std::sqrt(h[S_RR * 8 + k]);
      event[k] = active[k] && (rn <= h[S_THRESH * 8 + k] || rn <= 1e-2 * X.last_true_[k]);
      check[k] = event[k] || (active[k] && replace);
      anycheck |= check[k];
    }
    if (!anycheck) return Status{};
    const Grid& g0 = X.grids_[0];
    Op0Launch<double> L64{g0, X.mk64_, X.s64_, st_};
    X.set_mask(X.aux_, check);
    int nb = 0;
    op0_force_residual<float>(L64, X.tplg_, X.x_, X.r_, X.aux_, X.part_, &nb);
    fin_sum(X.part_, S_TRUE, nb, X.aux_, false, st_);
    HMG_TRY(X.read_scal(X.aux_, X.hscal_ + S_NSLOT * 8));
    const double* ha = X.hscal_ + S_NSLOT * 8;
    // FP32 cells keep the search direction after a replacement (Solver::solve)
    bool restart[NCASE], act[NCASE];
    for (int k = 0; k < NCASE; ++k) {
      restart[k] = false;
      if (check[k]) {
        const double tr = std::sqrt(ha[S_TRUE * 8 + k]);
        X.last_true_[k] = tr;
        if (tr <= h[S_THRESH * 8 + k]) active[k] = false;
      }
      act[k] = active[k];
    }
    X.set_mask(X.scal_, act);
    X.set_slot(X.scal_, S_RESTART, restart);
    X.set_slot(X.scal_, S_REPLACED, check);
    X.residual_mean(X.scal_);
    return Status{};
  }

  template <class F>
  Status run_graph(hipGraphExec_t& ex, F&& record) {
    if (!ex) {
      hipGraph_t gr = nullptr;
      if (hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return check_hip("graph capture");
      record();
      if (hipStreamEndCapture(st_, &gr) != hipSuccess) return check_hip("graph capture end");
      if (hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(gr);
        return check_hip("graph instantiate");
      }
      (void)hipGraphDestroy(gr);
    }
    if (hipGraphLaunch(ex, st_) != hipSuccess) return check_hip("graph launch");
    return Status{};
  }
  void destroy_graphs() {
    for (auto* e : {&g1_[0], &g1_[1], &g2_})
      if (*e) {
        (void)hipGraphExecDestroy(*e);
        *e = nullptr;
      }
  }
  void free_plans() {
    destroy_graphs();
    for (auto*& p : mvp_) {
      op0_batch_free(p);
      p = nullptr;
    }
    op0_batch_free(rsp_);
    op0_batch_free(psp_);
    rsp_ = psp_ = nullptr;
  }
  // scalars of the live cells (those of finished cells no longer change)
  Status read_all() {
    for (int c : live_)
      (void)hipMemcpyAsync(hsc_ + (size_t)c * S_NSLOT * 8, cells[c]->scal_,
                           sizeof(double) * S_NSLOT * 8, hipMemcpyDeviceToHost, st_);
    if (hipStreamSynchronize(st_) != hipSuccess) return check_hip("batch scalar readback");
    return check_hip("batch scalar readback");
  }

  hipStream_t st_;
  std::vector<int> order_;
  std::vector<int> live_;  // cells in the current plans (largest first)
  Op0BatchPlan* mvp_[2] = {nullptr, nullptr};
  Op0BatchPlan *rsp_ = nullptr, *psp_ = nullptr;
  PwBatchCell* pw_[3] = {nullptr, nullptr, nullptr};  // update (2 parities), Jacobi
  hipGraphExec_t g1_[2] = {nullptr, nullptr};
  hipGraphExec_t g2_ = nullptr;
  double* hsc_ = nullptr;
  int nblk_ = 1;
  int iters_run_ = 0;
  double tuned_ms_ = 0.0;
};

}  // namespace

struct hmg_batch_s {
  std::unique_ptr<BatchSolver> bs;
  std::string err;
};

struct hmg_ctx_s {
  hmg_config cfg{};
  hipStream_t stream = nullptr;
  std::string err;
  std::unique_ptr<SolverIface> solver;
  Grid g0{};
  DeviceArena arena;
  double* ocstate = nullptr;
  Partials ocpart{};
  float* fw = nullptr;      // filter weights, (2h+1)^3
  double fw_radius = -1.0;
  double* tw = nullptr;     // trigonometric-initialization weights
};

namespace {

hmg_status report(hmg_ctx ctx, const Status& s) {
  if (ctx) ctx->err = s.msg;
  return s.code;
}

Status validate(const hmg_config& c, std::vector<Grid>* grids) {
  if (c.nx < 4 || c.ny < 4 || c.nz < 4)
    return fail(HMG_E_INVALID, "every axis needs at least 4 cells (got %dx%dx%d)", c.nx, c.ny, c.nz);
  if ((int64_t)c.nx * c.ny * c.nz > (int64_t)1 << 31)
    return fail(HMG_E_INVALID, "cell too large");
  if ((int64_t)c.nx * c.ny > (int64_t)1 << 27)
    return fail(HMG_E_INVALID, "an xy plane may hold at most 2^27 cells (got %dx%d)", c.nx, c.ny);
  if (!(c.E0 > 0.0) || !(c.nu > -1.0 && c.nu < 0.5) || !(c.penal >= 1.0) || !(c.Emin >= 0.0) ||
      !(c.Emin < c.E0))
    return fail(HMG_E_INVALID, "bad material (E0 %g, nu %g, penal %g, Emin %g)", c.E0, c.nu,
                c.penal, c.Emin);
  if (c.omega < 0.0 || c.omega >= 1.0) return fail(HMG_E_INVALID, "omega must be in [0, 1)");
  if ((c.nu_pre != 0 && c.nu_pre != 1) || (c.nu_post != 0 && c.nu_post != 1))
    return fail(HMG_E_INVALID, "only one pre- and one post-smoothing sweep are supported");
  if (c.precision != HMG_FP64 && c.precision != HMG_FP32 && c.precision != HMG_MIXED_BF16 &&
      c.precision != HMG_MIXED_BF16_STENCIL)
    return fail(HMG_E_INVALID, "precision %d is not built in this library", c.precision);
  if (c.levels < 0 || c.replace_every < 0) return fail(HMG_E_INVALID, "bad levels/replace_every");
  if (c.smoother != 0 && c.smoother != 1)
    return fail(HMG_E_INVALID, "smoother must be 0 (damped block Jacobi) or 1 (Gauss-Seidel)");
  if (c.post_fp16 != 0 && c.post_fp16 != 1) return fail(HMG_E_INVALID, "post_fp16 must be 0 or 1");
  if (c.post_fp16 == 1 && c.precision == HMG_FP64)
    return fail(HMG_E_INVALID, "the FP16 displacement cast needs an FP32-storage precision");
  if (c.smoother == 1 && c.nx > 1024)
    return fail(HMG_E_INVALID, "the Gauss-Seidel smoother takes at most 1024 cells along x");
  if (c.nondyadic != 0 && c.nondyadic != 1) return fail(HMG_E_INVALID, "nondyadic must be 0 or 1");
  grids->clear();
  Grid g{c.nx, c.ny, c.nz, (int64_t)c.nx * c.ny * c.nz};
  grids->push_back(g);
  while (true) {
    if (c.levels > 0 && (int)grids->size() == c.levels) break;
    const Grid& f = grids->back();
    // the first step divides by 4 with non-dyadic coarsening (Sec. 4.2)
    const int F = (c.nondyadic && grids->size() == 1) ? 4 : 2;
    if (f.nx % F || f.ny % F || f.nz % F || f.nx / F < 4 || f.ny / F < 4 || f.nz / F < 4) break;
    Grid h{f.nx / F, f.ny / F, f.nz / F, (int64_t)(f.nx / F) * (f.ny / F) * (f.nz / F)};
    grids->push_back(h);
  }
  if (c.nondyadic && grids->size() < 2)
    return fail(HMG_E_INVALID, "non-dyadic coarsening needs every axis divisible by 4, >= 16");
  if (c.levels > 0 && (int)grids->size() != c.levels)
    return fail(HMG_E_INVALID, "cannot build %d levels on a %dx%dx%d cell", c.levels, c.nx, c.ny,
                c.nz);
  const int64_t ndof = 3 * grids->back().n;
  if (ndof > MAX_COARSE_DOF)
    return fail(HMG_E_INVALID, "coarsest grid has %lld unknowns; the direct solver takes at most %d",
                (long long)ndof, MAX_COARSE_DOF);
  return Status{};
}

}  // namespace

extern "C" {

hmg_status hmg_create(const hmg_config* cfg, void* hip_stream, hmg_ctx* out) {
  if (!cfg || !out) return HMG_E_INVALID;
  *out = nullptr;
  std::vector<Grid> grids;
  Status s = validate(*cfg, &grids);
  if (s.code != HMG_OK) {
    std::fprintf(stderr, "hmg_create: %s\n", s.msg.c_str());
    return s.code;
  }
  ElementConsts* ec = new ElementConsts;
  char err[256] = {0};
  if (build_element_consts(cfg->nu, ec, err, sizeof(err)) != 0) {
    std::fprintf(stderr, "hmg_create: %s\n", err);
    delete ec;
    return HMG_E_INVALID;
  }
  hmg_ctx ctx = new hmg_ctx_s;
  ctx->cfg = *cfg;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->g0 = grids[0];
  if (cfg->precision == HMG_FP64)
    ctx->solver.reset(new Solver<double, double, double>(*cfg, ctx->stream, *ec, grids));
  else if (cfg->precision == HMG_FP32)
    ctx->solver.reset(new Solver<float, float, float>(*cfg, ctx->stream, *ec, grids));
  else if (cfg->precision == HMG_MIXED_BF16)
    ctx->solver.reset(new Solver<float, bf16, float>(*cfg, ctx->stream, *ec, grids));
  else
    ctx->solver.reset(new Solver<float, bf16, bf16>(*cfg, ctx->stream, *ec, grids));
  delete ec;
  s = ctx->solver->init();
  if (s.code == HMG_OK) {
    ctx->ocstate = (double*)ctx->arena.alloc(sizeof(double) * 8);
    ctx->ocpart.buf = (double*)ctx->arena.alloc(sizeof(double) * 2 * 4096);
    ctx->ocpart.stride = 4096;
    ctx->tw = (double*)ctx->arena.alloc(sizeof(double) * TRIG_MAX_WEIGHTS);
    if (!ctx->ocstate || !ctx->ocpart.buf || !ctx->tw)
      s = fail(HMG_E_OOM, "device allocation failed");
  }
  if (s.code != HMG_OK) {
    std::fprintf(stderr, "hmg_create: %s\n", s.msg.c_str());
    delete ctx;
    return s.code;
  }
  *out = ctx;
  return HMG_OK;
}

hmg_status hmg_destroy(hmg_ctx ctx) {
  if (!ctx) return HMG_OK;
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
  return HMG_OK;
}

hmg_status hmg_set_density(hmg_ctx ctx, const float* rho_dev) {
  if (!ctx) return HMG_E_INVALID;
  if (!rho_dev) return report(ctx, fail(HMG_E_INVALID, "rho_dev is NULL"));
  return report(ctx, ctx->solver->set_density(rho_dev));
}

hmg_status hmg_solve_cases(hmg_ctx ctx, double rel_tol, int32_t max_iter, int32_t init,
                           const void* u0_dev, int32_t iters_out[6], double relres_out[6]) {
  if (!ctx) return HMG_E_INVALID;
  if (!iters_out || !relres_out) return report(ctx, fail(HMG_E_INVALID, "NULL host output"));
  int it[6];
  double rr[6];
  Status s = ctx->solver->solve(rel_tol, max_iter, init, u0_dev, it, rr);
  if (s.code == HMG_OK || s.code == HMG_E_NOT_CONVERGED)
    for (int c = 0; c < 6; ++c) {
      iters_out[c] = it[c];
      relres_out[c] = rr[c];
    }
  return report(ctx, s);
}

hmg_status hmg_elastic_tensor(hmg_ctx ctx, double C_out[36]) {
  if (!ctx) return HMG_E_INVALID;
  if (!C_out) return report(ctx, fail(HMG_E_INVALID, "C_out is NULL"));
  return report(ctx, ctx->solver->elastic(C_out));
}

hmg_status hmg_sensitivity(hmg_ctx ctx, const double W[36], float* dfdrho_dev) {
  if (!ctx) return HMG_E_INVALID;
  if (!W || !dfdrho_dev) return report(ctx, fail(HMG_E_INVALID, "NULL argument"));
  return report(ctx, ctx->solver->sens(W, dfdrho_dev));
}

hmg_status hmg_oc_update(hmg_ctx ctx, float* x_dev, const float* dfdx_dev, double volfrac,
                         double move, double damp, double xmin, double* lambda_out) {
  if (!ctx) return HMG_E_INVALID;
  if (!x_dev || !dfdx_dev) return report(ctx, fail(HMG_E_INVALID, "NULL argument"));
  if (!(volfrac > 0.0 && volfrac <= 1.0) || !(move > 0.0) || !(damp > 0.0) ||
      !(xmin >= 0.0 && xmin < 1.0))
    return report(ctx, fail(HMG_E_INVALID, "bad OC parameters"));
  hipStream_t st = ctx->stream;
  oc_init(ctx->ocstate, st);
  int nb = 0;
  for (int k = 0; k < 200; ++k) {
    oc_partial(ctx->g0, x_dev, dfdx_dev, move, damp, xmin, ctx->ocstate, ctx->ocpart, &nb, st);
    oc_step(ctx->ocpart, nb, ctx->g0.n, volfrac, ctx->ocstate, st);
  }
  oc_apply(ctx->g0, x_dev, dfdx_dev, move, damp, xmin, ctx->ocstate, st);
  double state[4];
  (void)hipMemcpyAsync(state, ctx->ocstate, sizeof(double) * 4, hipMemcpyDeviceToHost, st);
  if (hipStreamSynchronize(st) != hipSuccess) return report(ctx, check_hip("oc_update"));
  if (lambda_out) *lambda_out = state[3];
  return report(ctx, check_hip("oc_update"));
}

}  // extern "C"

namespace {
// Normalized cone weights of `radius` in ctx->fw (uploaded when the radius changes).
Status filter_weights(hmg_ctx ctx, double radius) {
  const int h = (int)std::ceil(radius) - 1;
  if (radius != ctx->fw_radius) {
    const int span = 2 * h + 1;
    std::vector<float> w((size_t)span * span * span);
    double sum = 0.0;
    std::vector<double> wd(w.size());
    int t = 0;
    for (int dz = -h; dz <= h; ++dz)
      for (int dy = -h; dy <= h; ++dy)
        for (int dx = -h; dx <= h; ++dx, ++t) {
          const double v = radius - std::sqrt((double)(dx * dx + dy * dy + dz * dz));
          wd[t] = v > 0.0 ? v : 0.0;
          sum += wd[t];
        }
    for (size_t i = 0; i < w.size(); ++i) w[i] = (float)(wd[i] / sum);
    if (!ctx->fw) ctx->fw = (float*)ctx->arena.alloc(sizeof(float) * 7 * 7 * 7);
    if (!ctx->fw) return fail(HMG_E_OOM, "device allocation failed");
    // earlier filter launches on the context stream may still read the old
    // weights: the copy is ordered on that stream, and the host vector must
    // outlive it
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return check_hip("filter");
    (void)hipMemcpyAsync(ctx->fw, w.data(), sizeof(float) * w.size(), hipMemcpyHostToDevice,
                         ctx->stream);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return check_hip("filter");
    ctx->fw_radius = radius;
  }
  return Status{};
}
}  // namespace

extern "C" {

hmg_status hmg_filter(hmg_ctx ctx, const float* in_dev, float* out_dev, double radius,
                      int32_t adjoint) {
  (void)adjoint;  // the cone filter is symmetric: H^T = H
  if (!ctx) return HMG_E_INVALID;
  if (!in_dev || !out_dev || in_dev == out_dev)
    return report(ctx, fail(HMG_E_INVALID, "filter needs distinct non-NULL buffers"));
  if (!(radius > 1.0 && radius <= 4.0))
    return report(ctx, fail(HMG_E_INVALID, "radius must be in (1, 4]"));
  Status st = filter_weights(ctx, radius);
  if (st.code != HMG_OK) return report(ctx, st);
  density_filter(ctx->g0, in_dev, out_dev, ctx->fw, (int)std::ceil(radius) - 1, ctx->stream);
  return report(ctx, check_hip("filter"));
}

hmg_status hmg_filter_sensitivity(hmg_ctx ctx, const float* x_dev, const float* g_dev,
                                  float* out_dev, double radius) {
  if (!ctx) return HMG_E_INVALID;
  if (!x_dev || !g_dev || !out_dev || out_dev == x_dev || out_dev == g_dev)
    return report(ctx, fail(HMG_E_INVALID, "sensitivity filter needs distinct non-NULL buffers"));
  if (!(radius > 1.0 && radius <= 4.0))
    return report(ctx, fail(HMG_E_INVALID, "radius must be in (1, 4]"));
  Status st = filter_weights(ctx, radius);
  if (st.code != HMG_OK) return report(ctx, st);
  sensitivity_filter(ctx->g0, x_dev, g_dev, out_dev, ctx->fw, (int)std::ceil(radius) - 1,
                     ctx->stream);
  return report(ctx, check_hip("filter_sensitivity"));
}

hmg_status hmg_objective(int32_t kind, const double C[36], int32_t iteration,
                         const double* params, double* F_out, double W_out[36]) {
  if (!C || !F_out || !W_out || iteration < 0) return HMG_E_INVALID;
  // beta, eta, tau, gamma (tau = NaN: -1 / E0^gamma with E0 = 1)
  double beta = 0.8, eta = 0.6, tau = std::nan(""), gamma = 0.5;
  if (params) {
    beta = params[0];
    eta = params[1];
    tau = params[2];
    gamma = params[3];
  }
  if (std::isnan(tau)) tau = -1.0;
  double W[36] = {0.0};
  double F = 0.0;
  switch (kind) {
    case HMG_OBJ_BULK:
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) W[i * 6 + j] = -1.0 / 9.0;
      break;
    case HMG_OBJ_SHEAR:
      for (int i = 3; i < 6; ++i) W[i * 6 + i] = -1.0 / 3.0;
      break;
    case HMG_OBJ_POISSON_RELAXED: {
      if (!(beta > 0.0 && beta < 1.0)) return HMG_E_INVALID;
      const double b = std::pow(beta, (double)iteration);
      W[0 * 6 + 1] = W[0 * 6 + 2] = W[1 * 6 + 2] = 1.0;
      for (int i = 0; i < 3; ++i) W[i * 6 + i] = -b;
      break;
    }
    case HMG_OBJ_POISSON_LOG: {
      const double A = C[0 * 6 + 1] + C[1 * 6 + 2] + C[2 * 6 + 0];
      const double B = C[0] + C[7] + C[14];
      if (!(B > 0.0) || !(1.0 + eta * A / B > 0.0)) return HMG_E_INVALID;
      F = std::log(1.0 + eta * A / B) + tau * std::pow(B, gamma);
      const double dA = eta / (B + eta * A);
      const double dB = -eta * A / (B * (B + eta * A)) + tau * gamma * std::pow(B, gamma - 1.0);
      W[0 * 6 + 1] = W[1 * 6 + 2] = W[2 * 6 + 0] = dA;
      for (int i = 0; i < 3; ++i) W[i * 6 + i] = dB;
      std::memcpy(W_out, W, sizeof(W));
      *F_out = F;
      return HMG_OK;
    }
    default:
      return HMG_E_INVALID;
  }
  for (int t = 0; t < 36; ++t) F += W[t] * C[t];
  std::memcpy(W_out, W, sizeof(W));
  *F_out = F;
  return HMG_OK;
}

hmg_status hmg_should_stop(const double* history, int32_t count, double rel_change,
                           int32_t window, int32_t max_iter, int32_t* stop_out) {
  if ((!history && count > 0) || count < 0 || !stop_out || !(rel_change > 0.0) || window < 1 ||
      max_iter < 1)
    return HMG_E_INVALID;
  int stop = count >= max_iter ? 1 : 0;
  if (!stop && count >= window + 1) {
    stop = 1;
    for (int k = count - window; k < count; ++k)
      if (!(std::fabs(history[k] - history[k - 1]) < rel_change * std::fabs(history[k - 1])))
        stop = 0;
  }
  *stop_out = stop;
  return HMG_OK;
}

hmg_status hmg_symmetrize(hmg_ctx ctx, const float* in_dev, float* out_dev, int32_t kind) {
  if (!ctx) return HMG_E_INVALID;
  if (!in_dev || !out_dev || in_dev == out_dev)
    return report(ctx, fail(HMG_E_INVALID, "symmetrize needs distinct non-NULL buffers"));
  if (kind < HMG_SYM_REFLECT3 || kind > HMG_SYM_ROTATE3)
    return report(ctx, fail(HMG_E_INVALID, "unknown symmetry %d", kind));
  const Grid& g = ctx->g0;
  if (kind != HMG_SYM_REFLECT3 && !(g.nx == g.ny && g.ny == g.nz))
    return report(ctx, fail(HMG_E_INVALID, "reflect6 and rotate3 need a cubic cell"));
  // signed permutations in the order (permutation lexicographic, flips binary
  // with the x bit most significant), kept by kind
  SymOps ops;
  int perm[3] = {0, 1, 2};
  do {
    const int inv = (perm[0] > perm[1]) + (perm[0] > perm[2]) + (perm[1] > perm[2]);
    for (int f = 0; f < 8; ++f) {
      const int fx = (f >> 2) & 1, fy = (f >> 1) & 1, fz = f & 1;
      const int det = ((inv & 1) ? -1 : 1) * (((fx + fy + fz) & 1) ? -1 : 1);
      const bool identity = perm[0] == 0 && perm[1] == 1 && perm[2] == 2;
      if (kind == HMG_SYM_REFLECT3 && !identity) continue;
      if (kind == HMG_SYM_ROTATE3 && det != 1) continue;
      ops.code[ops.count++] = perm[0] | perm[1] << 2 | perm[2] << 4 | (fx | fy << 1 | fz << 2) << 6;
    }
  } while (std::next_permutation(perm, perm + 3));
  symmetrize(g, in_dev, out_dev, ops, ctx->stream);
  return report(ctx, check_hip("symmetrize"));
}

hmg_status hmg_trig_init(hmg_ctx ctx, int32_t nfreq, const double q[4], const double* weights,
                         int32_t nweights, double volfrac, double rho_min, double k_sigmoid,
                         float* x_out_dev, double* mu_out) {
  if (!ctx) return HMG_E_INVALID;
  if (!q || !weights || !x_out_dev || nfreq < 1 || nfreq > TRIG_MAX_FREQ)
    return report(ctx, fail(HMG_E_INVALID, "bad trig_init arguments (nfreq %d)", nfreq));
  const int nt = 6 * nfreq;
  if (nweights != nt + nt * (nt + 1) / 2)
    return report(ctx, fail(HMG_E_INVALID, "need %d weights, got %d", nt + nt * (nt + 1) / 2,
                            nweights));
  if (!(volfrac > 0.0 && volfrac < 1.0) || !(rho_min >= 0.0) ||
      !(rho_min + std::fmin(1.5 * volfrac, 1.0) > volfrac) || !(k_sigmoid > 0.0))
    return report(ctx, fail(HMG_E_INVALID, "bad projection parameters"));
  const double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if (!(qn > 0.0)) return report(ctx, fail(HMG_E_INVALID, "the quaternion is zero"));
  const double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
  TrigBasis tb{{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)},
               nfreq};
  hipStream_t st = ctx->stream;
  (void)hipMemcpyAsync(ctx->tw, weights, sizeof(double) * nweights, hipMemcpyHostToDevice, st);
  trig_field(ctx->g0, tb, ctx->tw, x_out_dev, st);
  sigmoid_project(ctx->g0, x_out_dev, volfrac, rho_min, k_sigmoid, ctx->ocstate, ctx->ocpart, 200,
                  st);
  double state[4];
  (void)hipMemcpyAsync(state, ctx->ocstate, sizeof(double) * 4, hipMemcpyDeviceToHost, st);
  if (hipStreamSynchronize(st) != hipSuccess) return report(ctx, check_hip("trig_init"));
  if (mu_out) *mu_out = state[3];
  return report(ctx, check_hip("trig_init"));
}

hmg_status hmg_get_displacement(hmg_ctx ctx, void* u_dev) {
  if (!ctx) return HMG_E_INVALID;
  if (!u_dev) return report(ctx, fail(HMG_E_INVALID, "u_dev is NULL"));
  return report(ctx, ctx->solver->get_disp(u_dev));
}

hmg_status hmg_warm_start(hmg_ctx ctx, hmg_nn net, double accept_relres, double* relres_out,
                          int32_t* used_out) {
  if (!ctx) return HMG_E_INVALID;
  if (!net || !relres_out || !used_out || !(accept_relres >= 0.0))
    return report(ctx, fail(HMG_E_INVALID, "bad warm-start arguments"));
  int used = 0;
  Status s = ctx->solver->warm_start(*hmg_nn_internal(net), accept_relres, relres_out, &used);
  *used_out = used;
  return report(ctx, s);
}


hmg_status hmg_batch_create(const hmg_config* base, int32_t ncells, const int32_t* dims,
                            void* hip_stream, hmg_batch* out) {
  if (!base || !dims || !out || ncells < 1 || ncells > 4096) return HMG_E_INVALID;
  *out = nullptr;
  if (!hip_stream) {
    std::fprintf(stderr, "hmg_batch_create: graphs need a created stream, not the NULL stream\n");
    return HMG_E_INVALID;
  }
  if (base->precision != HMG_FP32) {
    std::fprintf(stderr, "hmg_batch_create: batched solves are FP32\n");
    return HMG_E_INVALID;
  }
  ElementConsts* ec = new ElementConsts;
  char err[256] = {0};
  if (build_element_consts(base->nu, ec, err, sizeof(err)) != 0) {
    std::fprintf(stderr, "hmg_batch_create: %s\n", err);
    delete ec;
    return HMG_E_INVALID;
  }
  hmg_batch b = new hmg_batch_s;
  b->bs.reset(new BatchSolver((hipStream_t)hip_stream));
  Status s;
  for (int c = 0; c < ncells && s.code == HMG_OK; ++c) {
    hmg_config cfg = *base;
    if (cfg.smoother != 0 || cfg.nondyadic != 0 || cfg.post_fp16 != 0) {
      s = fail(HMG_E_INVALID, "batched solves take the plain configuration (Jacobi, dyadic)");
      break;
    }
    cfg.nx = dims[3 * c];
    cfg.ny = dims[3 * c + 1];
    cfg.nz = dims[3 * c + 2];
    std::vector<Grid> grids;
    s = validate(cfg, &grids);
    if (s.code == HMG_OK && grids.size() < 2)
      s = fail(HMG_E_INVALID, "cell %d has a single multigrid level", c);
    if (s.code != HMG_OK) break;
    auto* X = new Solver<float, float, float>(cfg, (hipStream_t)hip_stream, *ec, grids);
    b->bs->cells.emplace_back(X);
    b->bs->cfgs.push_back(cfg);
    s = X->init();
  }
  delete ec;
  if (s.code == HMG_OK) s = b->bs->init();
  if (s.code != HMG_OK) {
    std::fprintf(stderr, "hmg_batch_create: %s\n", s.msg.c_str());
    delete b;
    return s.code;
  }
  *out = b;
  return HMG_OK;
}

hmg_status hmg_batch_destroy(hmg_batch b) {
  delete b;
  return HMG_OK;
}

hmg_status hmg_batch_set_density(hmg_batch b, int32_t cell, const float* rho_dev) {
  if (!b) return HMG_E_INVALID;
  if (cell < 0 || cell >= (int)b->bs->cells.size() || !rho_dev) {
    b->err = "bad cell index or NULL density";
    return HMG_E_INVALID;
  }
  Status s = b->bs->cells[cell]->set_density(rho_dev);
  b->err = s.msg;
  return s.code;
}

hmg_status hmg_batch_tune(hmg_batch b, int32_t* grid_out, int32_t* lz_out) {
  if (!b || !grid_out || !lz_out) return HMG_E_INVALID;
  int g = 0;
  std::vector<int> lz(b->bs->cells.size());
  Status s = b->bs->tune(&g, lz.data());
  *grid_out = g;
  for (size_t c = 0; c < lz.size(); ++c) lz_out[c] = lz[c];
  b->err = s.msg;
  return s.code;
}

hmg_status hmg_batch_solve(hmg_batch b, double rel_tol, int32_t max_iter, int32_t* iters_out,
                           double* relres_out) {
  if (!b || !iters_out || !relres_out || !(rel_tol > 0.0) || max_iter <= 0) return HMG_E_INVALID;
  std::vector<int> it(b->bs->cells.size() * NCASE);
  Status s = b->bs->solve(rel_tol, max_iter, it.data(), relres_out);
  for (size_t k = 0; k < it.size(); ++k) iters_out[k] = it[k];
  b->err = s.msg;
  return s.code;
}

hmg_status hmg_batch_elastic_tensors(hmg_batch b, double* C_out) {
  if (!b || !C_out) return HMG_E_INVALID;
  for (size_t c = 0; c < b->bs->cells.size(); ++c) {
    Status s = b->bs->cells[c]->elastic(C_out + 36 * c);
    if (s.code != HMG_OK) {
      b->err = s.msg;
      return s.code;
    }
  }
  return HMG_OK;
}

const char* hmg_batch_last_error(hmg_batch b) { return b ? b->err.c_str() : "NULL batch"; }

const char* hmg_last_error(hmg_ctx ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

hmg_status hmg_num_levels(hmg_ctx ctx, int32_t* levels_out) {
  if (!ctx || !levels_out) return HMG_E_INVALID;
  *levels_out = ctx->solver->levels();
  return HMG_OK;
}

hmg_status hmg_level_dims(hmg_ctx ctx, int32_t level, int32_t dims_out[3]) {
  if (!ctx || !dims_out) return HMG_E_INVALID;
  if (level < 0 || level >= ctx->solver->levels())
    return report(ctx, fail(HMG_E_INVALID, "level %d out of range", level));
  const Grid g = ctx->solver->level_grid(level);
  dims_out[0] = g.nx;
  dims_out[1] = g.ny;
  dims_out[2] = g.nz;
  return HMG_OK;
}

hmg_status hmg_profile(hmg_ctx ctx, int32_t enable) {
  if (!ctx) return HMG_E_INVALID;
  (void)hipStreamSynchronize(ctx->stream);
  ctx->solver->clock.enable(enable != 0);
  return HMG_OK;
}

hmg_status hmg_profile_read(hmg_ctx ctx, int32_t kernel, int64_t* launches, double* total_ms,
                            double* total_bytes) {
  if (!ctx || !launches || !total_ms || !total_bytes) return HMG_E_INVALID;
  if (kernel < 0 || kernel >= KernelClock::NK)
    return report(ctx, fail(HMG_E_INVALID, "unknown kernel id %d", kernel));
  ctx->solver->clock.read(kernel, launches, total_ms, total_bytes);
  return HMG_OK;
}

hmg_status hmg_element_constants(double nu, double* K0_out, double* load_out, double* lam0_out,
                                 double* msig_out) {
  if (!K0_out || !(nu > -1.0 && nu < 0.5)) return HMG_E_INVALID;
  std::unique_ptr<ElementConsts> ec(new ElementConsts);
  char err[256] = {0};
  if (build_element_consts(nu, ec.get(), err, sizeof(err)) != 0) return HMG_E_INVALID;
  std::memcpy(K0_out, ec->K0, sizeof(ec->K0));
  if (load_out) std::memcpy(load_out, ec->load, sizeof(ec->load));
  if (lam0_out) *lam0_out = ec->lam0;
  if (msig_out) std::memcpy(msig_out, ec->msig, sizeof(ec->msig));
  return HMG_OK;
}

hmg_status hmg_level_omega(hmg_ctx ctx, int32_t level, double* omega_out) {
  if (!ctx || !omega_out) return HMG_E_INVALID;
  if (level < 0 || level >= ctx->solver->levels())
    return report(ctx, fail(HMG_E_INVALID, "level %d out of range", level));
  *omega_out = ctx->solver->level_omega(level);
  return HMG_OK;
}

hmg_status hmg_apply_operator(hmg_ctx ctx, int32_t level, const void* u_dev, void* y_dev) {
  if (!ctx) return HMG_E_INVALID;
  if (level < 0 || level >= ctx->solver->levels() || !u_dev || !y_dev || u_dev == y_dev)
    return report(ctx, fail(HMG_E_INVALID, "bad apply_operator arguments"));
  return report(ctx, ctx->solver->apply_op(level, u_dev, y_dev));
}

hmg_status hmg_get_stencil(hmg_ctx ctx, int32_t level, void* out_dev) {
  if (!ctx) return HMG_E_INVALID;
  if (level < 0 || level >= ctx->solver->levels() || !out_dev)
    return report(ctx, fail(HMG_E_INVALID, "bad get_stencil arguments"));
  return report(ctx, ctx->solver->get_stencil(level, out_dev));
}

hmg_status hmg_load_vectors(hmg_ctx ctx, void* f_dev) {
  if (!ctx) return HMG_E_INVALID;
  if (!f_dev) return report(ctx, fail(HMG_E_INVALID, "f_dev is NULL"));
  return report(ctx, ctx->solver->loads(f_dev));
}

hmg_status hmg_vcycle(hmg_ctx ctx, const void* r_dev, void* z_dev) {
  if (!ctx) return HMG_E_INVALID;
  if (!r_dev || !z_dev || r_dev == z_dev)
    return report(ctx, fail(HMG_E_INVALID, "bad vcycle arguments"));
  return report(ctx, ctx->solver->vcycle(r_dev, z_dev));
}

hmg_status hmg_transfer(hmg_ctx ctx, int32_t level, int32_t direction, const void* in_dev,
                        void* out_dev) {
  if (!ctx) return HMG_E_INVALID;
  if (level < 0 || level + 1 >= ctx->solver->levels() || (direction != 0 && direction != 1) ||
      !in_dev || !out_dev || in_dev == out_dev)
    return report(ctx, fail(HMG_E_INVALID, "bad transfer arguments"));
  return report(ctx, ctx->solver->transfer(level, direction, in_dev, out_dev));
}

}  // extern "C"

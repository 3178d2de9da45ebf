/*
 * hmg.h - C ABI of the MI355X (gfx950) periodic homogenization solver.
 *
 * The library computes, for a periodic unit cell of nx*ny*nz unit voxels
 * (8-node trilinear bricks), the six macro-strain fluctuation fields, the
 * homogenized elasticity tensor C^H and its element sensitivities, following
 * Zhang et al., arXiv 2301.08911:
 *   - problem statement: Sec. 3.1, Eq. (opt-prob);
 *   - loads, FE solve, C^H:  Sec. 3.2, Eq. (el-force), (fem), (elasttensor);
 *   - sensitivities:         Sec. 3.2, Eq. (obj-grad), (ch-sens);
 *   - multigrid hierarchy:   Sec. 3.3 (Galerkin K_{l+1} = R K_l I, Alg. 1),
 *                            Sec. 4.2 (macro strain, relaxation split,
 *                            level-2 stencil assembly, null-space removal);
 *   - filter and OC update:  Sec. 5.2 and Sec. 6 parameters.
 * The FE systems are solved by conjugate gradients preconditioned with one
 * geometric-multigrid V-cycle (damped 3x3 block-Jacobi or eight-colour block
 * Gauss-Seidel smoothing, trilinear prolongation, restriction = its
 * transpose, FP64 direct coarsest solve).
 *
 * Conventions shared by every entry point
 *   - Index of vertex / element (x, y, z): idx = x + nx*(y + ny*z); the grid is
 *     periodic, so there are n = nx*ny*nz vertices and n elements.  Element
 *     idx has local node a = a0 + 2 a1 + 4 a2 at vertex (x+a0, y+a1, z+a2).
 *   - Nodal fields of the six load cases are "case-major SoA":
 *     u[(c*3 + k)*n + idx], case c in 0..5 (Voigt 11,22,33,12,23,13), comp k.
 *     Their element type is the context's field type: double for HMG_FP64,
 *     float otherwise.
 *   - Displacements are in element units (element-relative macro strain,
 *     Sec. 4.2 Eq. (macro-strain)); they are defined up to a translation and
 *     are returned with zero mean per case and component.
 *   - C^H is in units of E0, row-major 6x6, Voigt order 11,22,33,12,23,13
 *     (Sec. 3.2), normalised by |Omega| = n.
 *   - Pointers named *_dev are device pointers on the context's device; the
 *     caller owns them and they must stay valid until the call's work has
 *     completed on the context's stream.  Host arrays are plain C arrays.
 *   - Calls enqueue on the context's HIP stream.  Calls with host outputs
 *     (iters_out, relres_out, C_out, lambda_out, status checks of
 *     hmg_set_density) synchronize that stream before returning.
 *   - The library keeps no mutable process-wide state: separate contexts may
 *     be created and used from different host threads.  Calls on one context
 *     must not overlap.
 *   - Errors are reported by status code only; nothing throws across the ABI.
 *     hmg_last_error() gives a per-context message.  Argument errors leave the
 *     context state unchanged.
 */
#ifndef HMG_H
#define HMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hmg_ctx_s* hmg_ctx;

typedef enum {
  HMG_OK = 0,
  HMG_E_INVALID = 1,       /* bad argument, shape, density value or limit      */
  HMG_E_OOM = 2,           /* device allocation failed                          */
  HMG_E_DEVICE = 3,        /* a HIP runtime call failed                         */
  HMG_E_NOT_CONVERGED = 4, /* max_iter reached; outputs hold the partial state  */
  HMG_E_STATE = 5          /* called before its prerequisite step               */
} hmg_status;

typedef enum {
  HMG_FP64 = 0,        /* all fields, stencils and reductions in double        */
  HMG_FP32 = 1,        /* float fields/stencils, FP64 dots and coarsest solve  */
  HMG_MIXED_BF16 = 2,  /* Sec. 4.1 / Sec. 6.3 (Tab. pre) mixed precision: the multigrid preconditioner
                          streams its vectors (smoother corrections, coarse
                          residuals and corrections) in bf16 and computes in
                          FP32; outer PCG vectors FP32, iterate FP64, FP64
                          dots, residual recomputation (replace_every) and
                          coarsest solve; coarse stencils FP32                */
  HMG_MIXED_FP16 = 3,  /* reserved, not built: fp16 vectors cannot hold the
                          smoother corrections of soft regions (1/Emin scale)  */
  HMG_MIXED_BF16_STENCIL = 4 /* HMG_MIXED_BF16 with the coarse stencils and
                          block inverses also in bf16 (Sec. 4.1: low-precision
                          stencils, higher-precision vectors).  The centre
                          block of a rounded stencil is never read: it is
                          minus the sum of the 26 stored blocks, applied in
                          difference form, so translations (of the cell or of
                          a stiff island in void) stay exactly in the null
                          space and high-contrast cells converge as in FP32 */
} hmg_precision;

/* Solver configuration (Sec. 6 defaults: E0 = 1, nu = 0.3, p = 3). */
typedef struct hmg_config {
  int32_t nx, ny, nz;     /* cells per axis, each >= 4; nx*ny <= 2^27,         */
                          /* nx*ny*nz <= 2^31                                  */
  double E0;              /* Young's modulus of the solid (> 0)               */
  double nu;              /* Poisson ratio, in (-1, 0.5)                      */
  double penal;           /* SIMP exponent p (>= 1)                           */
  double Emin;            /* stiffness floor: s = Emin + rho^p (E0 - Emin)    */
  int32_t levels;         /* multigrid levels; 0 = coarsen 1:2 while every
                             axis stays even and the coarse mesh is >= 4 per
                             axis (Sec. 3.3)                                   */
  double omega;           /* block-Jacobi damping; 0 = per level 1.6/lambda_l  */
  int32_t nu_pre;         /* pre-smoothing sweeps; only 1 is supported          */
  int32_t nu_post;        /* post-smoothing sweeps; only 1 is supported         */
  int32_t precision;      /* hmg_precision                                     */
  int32_t replace_every;  /* recompute r = f - K x every k PCG iterations
                             (0 = never)                                      */
  int32_t smoother;       /* 0 = damped 3x3 block Jacobi (omega above);
                             1 = eight-colour symmetric block Gauss-Seidel
                             (Sec. 4.1 vertex subsets, Sec. 4.2 Eq.
                             (st-gs-relx)): colours (x mod 2) + 2 (y mod 2) +
                             4 (z mod 2) relaxed 0..7 before the coarse
                             correction and 7..0 after it; needs nx <= 1024;
                             single cells only (the batch API rejects it)    */
  int32_t post_fp16;      /* 1 = hmg_elastic_tensor and hmg_sensitivity read an
                             FP16 cast of the displacements (Sec. 4.3, the
                             cast before C^H and the sensitivity analysis),
                             held in the residual buffer, and compute in FP32
                             with FP64 sums; FP32-storage precisions only.
                             C^H is second order in the rounding (the
                             residual vanishes), the sensitivities first
                             order (about 1e-3 relative)                      */
  int32_t nondyadic;      /* 1 = the first coarsening divides every axis by 4
                             (Sec. 4.2 non-dyadic coarsening: the stencil goes
                             from the first level straight to the third, which
                             saves the largest stored stencil); later steps
                             halve.  Needs every axis divisible by 4 and
                             >= 16.  Transfers to and from that level use the
                             weights (4 - |a|)/4 of Eq. (st-assemb-w)         */
} hmg_config;

/* Create a context for one cell on the current HIP device.  `hip_stream` is a
 * hipStream_t (NULL = default stream).  Allocates the multigrid hierarchy and
 * the PCG work fields in device memory.  Fails with HMG_E_INVALID for a bad
 * configuration (shape, material, levels, or a coarsest grid above the direct
 * solver's limit of 12288 unknowns, a 16^3 grid) and HMG_E_OOM if the device is too small. */
hmg_status hmg_create(const hmg_config* cfg, void* hip_stream, hmg_ctx* out);

/* Release every device buffer of the context.  NULL is accepted. */
hmg_status hmg_destroy(hmg_ctx ctx);

/* Set the physical (already filtered) element densities rho~ in [0, 1]:
 * rho_dev is float[n].  Computes s_e = Emin + rho^p (E0 - Emin) (SIMP,
 * Sec. 3.2), the block-Jacobi inverses, the Galerkin stencils of every coarse
 * level (level 2 from the densities as in Sec. 4.2 Eq. (st-level-2), deeper
 * levels from the finer stencil) and the FP64 factor of the coarsest level.
 * A NaN or a value outside [0, 1] gives HMG_E_INVALID (checked on the device;
 * this call synchronizes). */
hmg_status hmg_set_density(hmg_ctx ctx, const float* rho_dev);

/* Solve K u^i = f^i for the six unit macro strains (Sec. 3.2 Eq. (fem),
 * loads Eq. (el-force) with the element-relative chi of Sec. 4.2).
 *   rel_tol   a case stops when ||f - K u|| <= max(rel_tol ||f||, eps_abs)
 *             with eps_abs = 1e-12 sqrt(n) (lambda1 + 2 mu1) mean(s), where
 *             lambda1, mu1 are the Lame constants of (E = 1, nu);
 *             a case with ||f|| <= eps_abs is solved by u = 0 in 0 iterations.
 *   max_iter  PCG iteration limit per case (> 0).
 *   init      0 = zero initial guess, 1 = the previous solution of this
 *             context, 2 = u0_dev (field type, case-major SoA).
 *   iters_out PCG iterations per case (host int32[6]).
 *   relres_out ||f - K u|| / ||f|| per case, recomputed at the end
 *             (host double[6]; 0 for a trivial case).
 * Returns HMG_E_NOT_CONVERGED if a case hit max_iter (outputs still filled),
 * HMG_E_STATE before hmg_set_density. */
hmg_status hmg_solve_cases(hmg_ctx ctx, double rel_tol, int32_t max_iter, int32_t init,
                           const void* u0_dev, int32_t iters_out[6], double relres_out[6]);

/* Homogenized tensor of the last solve, Sec. 3.2 Eq. (elasttensor):
 * C_ij = (1/n) sum_e s_e (chi^i - u^i_e)^T K0 (chi^j - u^j_e), host double[36].
 * HMG_E_STATE before hmg_solve_cases. */
hmg_status hmg_elastic_tensor(hmg_ctx ctx, double C_out[36]);

/* Element sensitivities of sum_ij W_ij C_ij with respect to rho~_e,
 * Sec. 3.2 Eq. (obj-grad) and (ch-sens), read per element:
 *   dfdrho[e] = (1/n) p rho_e^(p-1) (E0 - Emin) sum_ij W_ij d_e^i.K0 d_e^j,
 * d_e^i = chi^i - u^i_e.  W is host double[36] (row-major, e.g. dF/dC^H);
 * dfdrho_dev is float[n].  HMG_E_STATE before hmg_solve_cases. */
hmg_status hmg_sensitivity(hmg_ctx ctx, const double W[36], float* dfdrho_dev);

/* Optimality-criteria update (Sec. 3.3 step 4; parameters of Sec. 6), in place
 * on the design field x_dev (float[n]) with gradient dfdx_dev (float[n]):
 *   x_new = clamp(x * (max(0, -g)/lambda)^damp, max(xmin, x - move), min(1, x + move)),
 * with lambda found by bisection of log(lambda) on [1e-40, 1e40] so that
 * mean(x_new) = volfrac.  The chosen lambda is written to *lambda_out (host;
 * may be NULL).  Needs only hmg_create. */
hmg_status hmg_oc_update(hmg_ctx ctx, float* x_dev, const float* dfdx_dev, double volfrac,
                         double move, double damp, double xmin, double* lambda_out);

/* Periodic density filter (Sec. 5.2: rho~ = conv(x); radius 2 in Sec. 6):
 * out = H in, with weights max(0, radius - |d|) over integer offsets d,
 * normalised to sum 1.  H is symmetric, so `adjoint` (apply H^T, used to take
 * dF/drho~ back to dF/dx) gives the same result.  in_dev/out_dev are float[n]
 * and must not overlap.  radius in (1, 4]. */
hmg_status hmg_filter(hmg_ctx ctx, const float* in_dev, float* out_dev, double radius,
                      int32_t adjoint);

/* Copy the current iterate (field type, case-major SoA) to u_dev: the last
 * solution (zero mean), or, after an accepted hmg_warm_start and before the
 * next solve, that guess.  HMG_E_STATE if there is neither. */
hmg_status hmg_get_displacement(hmg_ctx ctx, void* u_dev);

/* ---- design-space steps of the optimization loop --------------------------- */

/* Sensitivity filter (Sec. 5.3, the OC optimizer's filter of the sensitivity
 * when the density itself is not filtered):
 *   out_e = sum_f w_ef x_f g_f / (max(1e-3, x_e) sum_f w_ef),
 * w the periodic cone weights of hmg_filter.  x_dev, g_dev, out_dev are
 * float[n]; out must not overlap the inputs.  radius in (1, 4]. */
hmg_status hmg_filter_sensitivity(hmg_ctx ctx, const float* x_dev, const float* g_dev,
                                  float* out_dev, double radius);

/* Symmetry groups of the cube (Sec. 6.1). */
typedef enum {
  HMG_SYM_REFLECT3 = 0, /* mirror planes x, y, z = 0.5 (8 elements); any box  */
  HMG_SYM_REFLECT6 = 1, /* those and x = y, y = z, z = x (48); cubic cells    */
  HMG_SYM_ROTATE3 = 2   /* quarter turns about the axes through the centre and
                           their compositions (24); cubic cells                */
} hmg_symmetry;

/* Orbit averaging (Sec. 6.1): out_e = (1/|G|) sum_{g in G} in_{g(e)}, the
 * element of cell coordinates c mapped by a signed axis permutation
 * (c_a -> c_{perm a}, mirrored as N - 1 - c where flipped).  in_dev/out_dev
 * are float[n] and must not overlap; the sum is taken in double.
 * HMG_E_INVALID for an unknown kind or a non-cubic cell with reflect6 or
 * rotate3. */
hmg_status hmg_symmetrize(hmg_ctx ctx, const float* in_dev, float* out_dev, int32_t kind);

/* Trigonometric initialization (Sec. 6.2).  With xb = R_q (x - (0.5, 0.5, 0.5)),
 * x the element centre in [0, 1]^3 and R_q the rotation of the quaternion q
 * (w, x, y, z; normalized here), T_n = cos(2 pi k xb_i), sin(2 pi k xb_i) in
 * the order (axis i = 0..2, k = 1..nfreq, cos then sin) and Q_n = T_n
 * followed by the products T_a T_b for a <= b (row-major in (a, b)):
 *   y_e = sum_m weights[m] Q_m(x_e),
 *   x_e = rho_min + Vh / (1 + exp(-k (y_e - mu))),  Vh = min(1.5 volfrac, 1),
 * with mu by bisection (200 halvings of [min y - 40/k, max y + 40/k]) so that
 * mean(x) = volfrac.  nfreq in 1..4; nweights must be 6 nfreq + 3 nfreq
 * (6 nfreq + 1); weights and q are host arrays (the caller draws them);
 * x_out_dev is float[n]; *mu_out (host, may be NULL) receives mu.  The paper
 * uses k = 15 and rho_min = 1e-3.  Synchronizes. */
hmg_status hmg_trig_init(hmg_ctx ctx, int32_t nfreq, const double q[4], const double* weights,
                         int32_t nweights, double volfrac, double rho_min, double k_sigmoid,
                         float* x_out_dev, double* mu_out);

/* Objectives F(C^H) and W = dF/dC^H (Sec. 5.2 Eq. (bulk-obj), Sec. 5.3 Eq.
 * (shear-obj), (poisson-relx), (poisson-new)); host only, no context or GPU.
 * W is written entry by entry as the formula reads (row-major 6x6; C^H is
 * symmetric, so the contraction with dC^H/drho is the same either way).
 *   BULK            F = -(1/9) sum_{i,j<3} C_ij
 *   SHEAR           F = -(C33 + C44 + C55) / 3
 *   POISSON_RELAXED F = C01 + C02 + C12 - beta^iteration (C00 + C11 + C22)
 *   POISSON_LOG     F = log(1 + eta A / B) + tau B^gamma,
 *                   A = C01 + C12 + C20, B = C00 + C11 + C22
 * params = {beta, eta, tau, gamma} or NULL for {0.8, 0.6, -1, 0.5} (the paper's
 * eta, gamma and tau = -1/E0^gamma with E0 = 1; beta is the user's constant
 * in (0, 1)); tau = NaN also selects -1.  HMG_E_INVALID for an unknown kind,
 * beta outside (0, 1), or B <= 0 / 1 + eta A / B <= 0 for POISSON_LOG. */
typedef enum {
  HMG_OBJ_BULK = 0,
  HMG_OBJ_SHEAR = 1,
  HMG_OBJ_POISSON_RELAXED = 2,
  HMG_OBJ_POISSON_LOG = 3
} hmg_objective_kind;
hmg_status hmg_objective(int32_t kind, const double C[36], int32_t iteration,
                         const double* params, double* F_out, double W_out[36]);

/* Stopping rule (Sec. 6): *stop_out = 1 once the relative change
 * |F_k - F_{k-1}| / |F_{k-1}| of the objective history has stayed below
 * rel_change for `window` consecutive iterations, or count >= max_iter; else 0.
 * The paper's values are 5e-4, 3 and 300.  Host only. */
hmg_status hmg_should_stop(const double* history, int32_t count, double rel_change,
                           int32_t window, int32_t max_iter, int32_t* stop_out);

/* Message of the last failed call on this context ("" if none). */
const char* hmg_last_error(hmg_ctx ctx);

/* ---- kernel timing --------------------------------------------------------- */

/* Kernels whose launches inside hmg_solve_cases can be timed. */
typedef enum {
  HMG_K_MATVEC = 0,        /* p = z + beta p, q = K p, p.q          (level-0 operator) */
  HMG_K_RESIDUAL = 1,      /* t = (r - m) - K z0                    (level-0 operator) */
  HMG_K_POST_SMOOTH = 2,   /* z = z1 + D^-1 ((r - m) - K z1)       (level-0 operator) */
  HMG_K_UPDATE = 3,        /* x += alpha p (FP64), r -= alpha q                          */
  HMG_K_TRUE_RESIDUAL = 4, /* r = f - K x in FP64                                        */
  HMG_K_JACOBI = 5,        /* z0 = D^-1 (r - m), level 0, all cases per vertex           */
  HMG_K_GS_FORWARD = 6,    /* level-0 Gauss-Seidel sweep 0..7 from zero (4 launches)     */
  HMG_K_GS_BACKWARD = 7,   /* level-0 Gauss-Seidel sweep 7..0 with (r - m).z (4 launches) */
  HMG_K_PROLONG = 8        /* z1 = z0 + P e, level 0 (damped-Jacobi cycle)               */
} hmg_kernel;

/* enable != 0 clears the counters and starts recording a HIP event pair around
 * every launch of the kernels above (on the context stream); 0 stops. */
hmg_status hmg_profile(hmg_ctx ctx, int32_t enable);

/* Launch count, summed event time (ms) and summed algorithmic bytes of one
 * kernel since profiling was enabled.  Algorithmic bytes are the unique bytes
 * the launch must move for its active cases (inputs read once, outputs written
 * once; halo re-reads not counted).  Synchronizes the stream. */
hmg_status hmg_profile_read(hmg_ctx ctx, int32_t kernel, int64_t* launches, double* total_ms,
                            double* total_bytes);

/* ---- batched cells (many independent cells, one launch per level-0 pass) --
 * Not part of the paper's method: a throughput form for many small unit cells
 * of uneven resolution.  The cells (each with its own multigrid hierarchy and
 * six load cases) are solved in lockstep by FP32 MG-PCG: each level-0 pass
 * (matvec, update, block Jacobi, residual, post-smoothing) is ONE persistent
 * launch over the tiles of all cells (largest cells first), and each PCG
 * iteration replays two captured HIP graphs that also hold the coarse levels
 * and the scalar finalizers.  Convergence, residual recomputation and the
 * per-case tolerance are those of hmg_solve_cases. */
typedef struct hmg_batch_s* hmg_batch;

/* base: material and solver settings (precision must be HMG_FP32; levels 0 =
 * paper rule per cell); dims: ncells x (nx, ny, nz).  Every cell needs at
 * least two multigrid levels.  hip_stream must be a created stream (graphs
 * cannot be captured on the NULL stream); all batch calls run on it. */
hmg_status hmg_batch_create(const hmg_config* base, int32_t ncells, const int32_t* dims,
                            void* hip_stream, hmg_batch* out);
hmg_status hmg_batch_destroy(hmg_batch b);
/* rho_dev: float[nx*ny*nz] of that cell (as hmg_set_density). */
hmg_status hmg_batch_set_density(hmg_batch b, int32_t cell, const float* rho_dev);
/* Autotuner: times the batched matvec for candidate tile z-chunks (per cell
 * size) and persistent grid sizes and keeps the fastest; grid_out (0 = one
 * block per tile) and lz_out[ncells] (0 = default chunk) report the choice.
 * Needs the densities set (it runs the real kernels). */
hmg_status hmg_batch_tune(hmg_batch b, int32_t* grid_out, int32_t* lz_out);
/* iters_out[ncells*6], relres_out[ncells*6] (recomputed FP64 relative
 * residuals); HMG_E_NOT_CONVERGED if any case hit max_iter. */
hmg_status hmg_batch_solve(hmg_batch b, double rel_tol, int32_t max_iter, int32_t* iters_out,
                           double* relres_out);
/* C_out[ncells*36]: each cell's homogenized tensor (as hmg_elastic_tensor). */
hmg_status hmg_batch_elastic_tensors(hmg_batch b, double* C_out);
const char* hmg_batch_last_error(hmg_batch b);

/* ---- inspection entry points (used by the parity tests) ------------------ */

/* The library's element constants for E = 1 and Poisson ratio nu: the
 * stiffness K0 of the unit trilinear brick (Sec. 3.2, Eq. (el-force)) and the
 * unit-strain load template K0 chi^i of the six cases (Sec. 4.2,
 * Eq. (macro-strain)).  K0_out: host array of 24*24 doubles, row-major, dof
 * 3a+k of local node a = a0 + 2 a1 + 4 a2.  load_out: host array of 6*24
 * doubles, load_out[i*24 + 3a+k], or NULL.  lam0_out: the largest eigenvalue
 * of blockdiag(K0)^-1 K0 (3x3 node blocks), which bounds the spectrum of the
 * level-0 block-Jacobi operator for any densities, or NULL.  msig_out: host
 * array of 8*24*24 doubles, or NULL: for each sub-position sigma = s0 + 2 s1 +
 * 4 s2 of a fine element inside a coarse element, W_sigma^T K0 W_sigma, where
 * W_sigma interpolates the coarse element's nodes trilinearly to the fine
 * element's nodes (the first coarse level is assembled from these, Sec. 4.2
 * Eq. (st-level-2)); msig_out[(sigma*24 + 3A+p)*24 + 3B+q].  Host-only: no
 * device is touched, so the call works without a GPU.  HMG_E_INVALID for a
 * NULL K0_out or nu outside (-1, 0.5). */
hmg_status hmg_element_constants(double nu, double* K0_out, double* load_out, double* lam0_out,
                                 double* msig_out);

/* Number of multigrid levels and the cells per axis of one level. */
hmg_status hmg_num_levels(hmg_ctx ctx, int32_t* levels_out);
hmg_status hmg_level_dims(hmg_ctx ctx, int32_t level, int32_t dims_out[3]);

/* Block-Jacobi damping used on a level after the last hmg_set_density:
 * 1.6 / lambda_l, with lambda_l a bound of the spectrum of D_l^-1 K_l (level 0:
 * the element bound, valid for any densities; coarser levels: power
 * iteration + 5 %).  A configured omega replaces 1.6/lambda_l but is capped at
 * 1.9/lambda_l.  0 for the coarsest level, which is solved directly. */
hmg_status hmg_level_omega(hmg_ctx ctx, int32_t level, double* omega_out);

/* y = K_l u for the six cases on one level (field type, case-major SoA at that
 * level's size).  Level 0 is the matrix-free operator of Sec. 4.2
 * Eq. (st-assemb); deeper levels use the stored Galerkin stencils. */
hmg_status hmg_apply_operator(hmg_ctx ctx, int32_t level, const void* u_dev, void* y_dev);

/* The 27-point stencil of level l: out[((d*3 + i)*3 + j)*n_l + v] is the
 * (i, j) entry of the 3x3 block coupling vertex v to v + offset(d), with
 * d = (dx+1) + 3 (dy+1) + 9 (dz+1).  Level 0 is assembled from the densities
 * for this call; deeper levels are the stored Galerkin stencils (Sec. 4.2). */
hmg_status hmg_get_stencil(hmg_ctx ctx, int32_t level, void* out_dev);

/* The six macro-strain load vectors f^i (field type, case-major SoA),
 * Sec. 4.2 "Enforce macro strain". */
hmg_status hmg_load_vectors(hmg_ctx ctx, void* f_dev);

/* z = M r: one application of the multigrid V-cycle preconditioner on the
 * six cases (field type, case-major SoA at level 0). */
hmg_status hmg_vcycle(hmg_ctx ctx, const void* r_dev, void* z_dev);

/* Grid transfer between level l and l+1: direction 0 restricts (R = P^T) a
 * level-l field into a level-(l+1) field; direction 1 prolongates (P) a
 * level-(l+1) field into a level-l field (overwriting it).  The output of
 * direction 1 is written two values at a time: out_dev must be aligned to
 * twice the field element size (HMG_E_INVALID otherwise). */
hmg_status hmg_transfer(hmg_ctx ctx, int32_t level, int32_t direction, const void* in_dev,
                        void* out_dev);

#ifdef __cplusplus
}
#endif

#endif /* HMG_H */

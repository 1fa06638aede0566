/*
 * rlbm.h - C ABI of the MI355X (gfx950) relativistic lattice Boltzmann library.
 *
 * The library advances the second-order relativistic lattice Boltzmann method
 * for particles of finite mass of Gabbana, Mendoza, Succi and Tripiccione,
 * "Towards a unified lattice kinetic scheme for relativistic hydrodynamics"
 * (arXiv:1703.04605):
 *
 *   f_i(x + n_i, t + 1) = f_i(x, t) - (p_i^mu U_mu)/(p_i^0 tau) (f_i - f_i^eq)
 *
 * (Sec. III.B, eq. discrete-relativistic-boltzmann) on 2D (Nx x Ny) and 1D
 * (Nx x 1) lattices.  Units: T_R = 1 (the temperature unit of Sec. III.A),
 * lattice spacing 1, time step 1 = dx/v0 (eq. v0dt=dx), so the particle mass
 * is mbar = m/T_R ("zeta").
 *
 * Conventions of every entry point:
 *   - C linkage, no exceptions cross the ABI; a negative return is an error
 *     code (RLBM_E*), and rlbm_last_error() gives a message for the context.
 *   - Pointers marked "device" are HIP device pointers (e.g. torch CUDA tensor
 *     data_ptr()), pointers marked "host" are ordinary host memory.
 *   - Field arrays are row-major with x fastest: element (y, x) at y*nx + x.
 *   - "stream" is a hipStream_t passed as void* (NULL = the default stream).
 *     Device work is enqueued on it and returns without synchronising, unless
 *     stated otherwise.
 *   - Population buffers and field buffers are owned by the caller; the
 *     library keeps the raw pointers until the next rlbm_init_fields() or
 *     rlbm_destroy().  The context and its stencil tables are owned by the
 *     library.  Only rlbm_init_stencil (the constant tables),
 *     rlbm_init_fields (a small per-tile health array), the warm start and
 *     the batched and network set-up calls allocate device memory; the
 *     time-stepping entry points never do.
 */
#ifndef RLBM_H
#define RLBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------- */
#define RLBM_OK 0
#define RLBM_EINVAL (-1)      /* invalid argument or size */
#define RLBM_ENOSTENCIL (-2)  /* no quadrature with all weights positive */
#define RLBM_EHIP (-3)        /* a HIP runtime call failed */
#define RLBM_ENUMERIC (-4)    /* a fatal health flag was raised on the GPU */
#define RLBM_ESTATE (-5)      /* call out of order (e.g. step before init) */

/* ---- storage precisions ---------------------------------------------- */
#define RLBM_FP64 0      /* populations f_i stored and processed in float64 */
#define RLBM_FP32_DEV 1  /* f_i = f_i^ref + d_i, d_i stored/processed in float32,
                            Landau frame, EOS and projections in float64 */
#define RLBM_FP16_DEV 2  /* d_i = s_i h_i, h_i stored as binary16, arithmetic
                            as RLBM_FP32_DEV */

/* ---- boundary conditions (per axis) ----------------------------------- */
#define RLBM_BC_PERIODIC 0
#define RLBM_BC_OUTFLOW 1  /* zero gradient: a population pulled from outside
                              the domain takes the post-collision value of the
                              nearest in-domain site */

/* ---- relaxation time ---------------------------------------------------- */
#define RLBM_TAU_CONST 0       /* tau (lattice units) constant */
#define RLBM_TAU_ETA_OVER_S 1  /* tau per site from eta/s (Sec. IV) */

/* ---- health flags (OR-ed over all sites since the last reset) ---------- */
#define RLBM_H_NAN 1u          /* non-finite moment or field */
#define RLBM_H_LANDAU 2u       /* Landau iteration hit its cap */
#define RLBM_H_SUPERLUMINAL 4u /* |u| >= 1 */
#define RLBM_H_RANGE 8u        /* n <= 0, eps <= 0 or eps/n below the rest mass */
#define RLBM_H_EOS 16u         /* EOS Newton iteration hit its cap */
#define RLBM_H_SYNC 32u        /* batched launch: a wait on neighbouring tiles timed out,
                                  or the tiles of one problem did not share one L2 */
#define RLBM_H_FATAL (RLBM_H_NAN | RLBM_H_SUPERLUMINAL | RLBM_H_RANGE | RLBM_H_SYNC)

typedef struct rlbm_ctx rlbm_ctx;

/*
 * Stencil description (Sec. III.C-D).  The quadrature is built from
 * full-symmetric velocity groups (Appendix C): each base vector (a, b, c)
 * stands for all its coordinate permutations and sign flips.  Abscissae are
 * p_{i,k} = zeta gamma_k (1, v0 n_{i,k}) (eq. four-momentum); one weight per
 * group solves the second-order orthonormality conditions (eq. ortho1),
 * which for full-symmetric groups reduce to six: the energy moments of
 * order 0..4 of the weight function and one quartic-isotropy condition.  At
 * third order (Sec. III.D: eleven independent conditions) they are the
 * energy moments of order 0..6, the quartic isotropy times p0^0..2 and the
 * sextic one (p_x^2 p_y^2 p_z^2).
 */
typedef struct {
  int dim;               /* 2: Nx x Ny lattice (1 x Nx x Ny slab of the 3D
                            stencil), 1: Nx x 1 lattice, 3: Nx x Ny x Nz
                            lattice with every population of the stencil
                            (Sec. V); 3D lattices take rlbm_init_fields3 and
                            rlbm_moments3 */
  int n_groups;          /* number of groups: 6 at second order, 11 at third */
  const int* group_base; /* host, 3*n_groups ints: base vectors (a, b, c) */
  double zeta;           /* mbar = m / T_R, > 0 */
  double v0;             /* > 0: use this v0 (must give positive weights);
                            <= 0: search [v0_lo, v0_hi] for the interval of
                            all-positive weights and take its midpoint */
  double v0_lo, v0_hi;   /* search interval (0, 0: (0, v_max)) */
  int precision;         /* RLBM_FP64 | RLBM_FP32_DEV | RLBM_FP16_DEV */
  double n_ref, T_ref;   /* deviation reference f^ref = f^eq(n_ref, T_ref, u=0)
                            (ignored for RLBM_FP64; 0 means 1) */
  int order;             /* expansion order of the equilibrium (eq.
                            mj-projected-distribution): 0 or 2 = second order
                            (14 polynomials, 6 groups); 3 = third order (30
                            polynomials, 11 groups, Sec. III.A and III.D),
                            RLBM_FP64 or RLBM_FP32_DEV (float32 deviations
                            from f^eq(n_ref, T_ref, u=0)); RLBM_FP16_DEV is
                            rejected (RLBM_EINVAL); third-order contexts of every dim
                            take rlbm_init_fields3 / rlbm_moments3 (nz = 1 for
                            dim 1 and 2, ny = 1 for dim 1) */
  const double* weights; /* host, nullable: n_groups weights (per population
                            of each group) to use instead of solving; needs
                            v0 > 0, and must pass the same positivity and
                            orthonormality checks */
} rlbm_stencil_desc;

typedef struct {
  int q3;                /* populations of the 3D stencil */
  int q;                 /* populations after exact in-plane merging (the
                            number of classes the GPU stores per site) */
  double v0;             /* v0 in use */
  double v0_lo, v0_hi;   /* positive-weight window found (search only) */
  double weights[16];    /* weight per group (per population of the group) */
  double ortho_residual; /* max |sum_i w_i J_l(p_i) J_k(p_i) - delta_lk| */
  int max_shift;         /* max |n_x| (and |n_y|, |n_z|) of the stencil */
  double cond;           /* 2-norm condition number at v0 of the system
                            matrix of the quadrature problem (Sec. III.D: rows
                            the pairs l <= k of the 14 (third order: 30)
                            polynomials, columns the groups, entries
                            sum_{i in group} J_l J_k), the quantity that grows
                            at small mbar */
} rlbm_stencil_info;

/*
 * Builds the stencil on the host (long double), checks orthonormality and
 * positivity, and uploads the population-class table to the current HIP
 * device.  *out receives a new context.  info (host, nullable) receives the
 * result.  Errors: RLBM_EINVAL (bad description), RLBM_ENOSTENCIL (no
 * positive weights at v0 / in the window, or orthonormality residual above
 * 1e-10), RLBM_EHIP.
 */
int rlbm_init_stencil(rlbm_ctx** out, const rlbm_stencil_desc* desc, rlbm_stencil_info* info);

/* Host-only part of rlbm_init_stencil (no HIP call): fills info. */
int rlbm_solve_stencil(const rlbm_stencil_desc* desc, rlbm_stencil_info* info);

/*
 * Host-only: the population-class table of the stencil.  For class j
 * (0 <= j < info.q): disp[2j], disp[2j+1] = in-plane displacement (n_x, n_y);
 * mom[3j..3j+2] = (p^0, p^x, p^y) (p^y = 0 in 1D); M[10j + k] = sum over the
 * class members of w_i J^(k)(p_i) for the polynomials, in Appendix A labels,
 * k = 0, 1_0, 1_x, 1_y, 2_00, 2_0x, 2_0y, 2_xx, 2_yy, 2_xy.  Buffers are host
 * arrays of capacity cap classes; RLBM_EINVAL if cap < q.
 */
int rlbm_class_table(const rlbm_stencil_desc* desc, int cap, int* disp, double* mom, double* M);

/*
 * Host-only: temperatures T[i] solving e[i] = 3T + zeta K_1(zeta/T)/K_2(zeta/T)
 * (eq. relativistic-eos, energy per particle e = eps/n, T_R = 1) from the same
 * piecewise Chebyshev table of T(e - zeta) that the GPU kernels evaluate
 * (quarter octaves of e - zeta, built in long double for this zeta).  n values,
 * host arrays.  Errors: RLBM_EINVAL.
 */
int rlbm_eos_temperature_host(double zeta, const double* e, int n, double* T);

/* Frees the context and its device tables (after synchronising its work). */
int rlbm_destroy(rlbm_ctx* ctx);

/* Bytes of one population buffer for an nx x ny lattice in this context's
 * precision: storage rows (lattice rows plus ghost rows) of q class rows each
 * (ghost columns included), padded to 128 elements.  0 on invalid sizes. */
size_t rlbm_population_bytes(const rlbm_ctx* ctx, int nx, int ny);

typedef struct {
  int nx, ny;            /* lattice size; ny must be 1 when dim == 1 */
  int bc_x, bc_y;        /* RLBM_BC_* */
  int tau_mode;          /* RLBM_TAU_* */
  double tau;            /* RLBM_TAU_CONST: relaxation time (> 0.5) */
  /* RLBM_TAU_ETA_OVER_S (Sec. IV): tau = 1/2 + (3/2) (eta/s) s hbar_c v0 / (P dx)
   * with s = 4n - n ln(n / n_eq), n_eq = 16 T^3 / (pi^2 (hbar c)^3), in
   * physical units: T = T_lat * T_R_GeV, n = n_lat * n_unit_fm3. */
  double eta_over_s, T_R_GeV, n_unit_fm3, dx_fm;
  double landau_tol;     /* target relative accuracy of eps and u (0: 1e-14
                            for FP64, 1e-10 otherwise) */
  int landau_maxit;      /* iteration cap (0: 200; at most 10^6, else RLBM_EINVAL) */
  int landau_method;     /* RLBM_LANDAU_NEWTON: Newton on the characteristic
                            polynomial det(l I - T eta) from l = T^00, then u
                            from the spatial rows; RLBM_LANDAU_FIXED_POINT:
                            eps = T^00 - T^0i u_i, u_i = (T^0i - T^ij u_j)/eps
                            from u = 0, until |d eps| <= tol eps, |d u| <= tol
                            (3D lattices: Newton only) */
  int nz;                /* 3D stencils (dim 3): sites along z (>= 1); must
                            be 0 or 1 for 1D and 2D stencils */
  int bc_z;              /* 3D stencils: RLBM_BC_* along z */
} rlbm_lattice_desc;

#define RLBM_LANDAU_NEWTON 0
#define RLBM_LANDAU_FIXED_POINT 1

/*
 * Sets f_i(x, 0) = f_i^eq(n, T, u) (eq. mj-discrete-feq with the density n
 * factored in) at every site from caller fields n, T, ux, uy (device, float64,
 * nx*ny each).  popA and popB (device, pop_bytes each, at least
 * rlbm_population_bytes()) become the ping-pong state.  The step counter is
 * reset and the health flags cleared.  Errors: RLBM_EINVAL, RLBM_EHIP.
 * Invalid descriptions (the checks of rlbm_check_lattice, NULL or too small
 * buffers) are rejected before the context changes; a HIP failure after that
 * leaves the context without fields (rlbm_step then returns RLBM_ESTATE).
 */
int rlbm_init_fields(rlbm_ctx* ctx, const rlbm_lattice_desc* lat, const double* n, const double* T,
                     const double* ux, const double* uy, void* popA, void* popB, size_t pop_bytes,
                     void* stream);

/*
 * Host-only (no HIP call): checks a lattice description against a stencil
 * description exactly as rlbm_init_fields does before it touches the device
 * (sizes, boundary rules, relaxation time, Landau options, and the layout's
 * limits: fewer than 2^31 stored elements and class byte offsets below
 * 2^31).  RLBM_OK, or RLBM_EINVAL / RLBM_ENOSTENCIL with the reason in
 * rlbm_last_error(NULL).
 */
int rlbm_check_lattice(const rlbm_stencil_desc* desc, const rlbm_lattice_desc* lat);

/*
 * Allocation-free form of rlbm_init_fields, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops that set
 * up many lattices).  Same arguments, checks, result and errors; the health
 * slots of the lattice (one per 64 sites of a row) live in a static device
 * array that the library holds on each GPU until the process ends, instead
 * of library-allocated memory, so no hipMalloc or hipFree is called.  Limit:
 * 262144 tiles (ceil(nx/64) * ny), e.g. 4096 x 4096 sites; larger lattices
 * give RLBM_EINVAL.  One context per GPU uses the array at a time: this call
 * drops the fields of the context that used it before (its rlbm_step then
 * returns RLBM_ESTATE).  Calls that overlap on one GPU race (their health
 * counters mix).
 */
int rlbm_init_fields_noalloc(rlbm_ctx* ctx, const rlbm_lattice_desc* lat, const double* n, const double* T,
                             const double* ux, const double* uy, void* popA, void* popB, size_t pop_bytes,
                             void* stream);

/*
 * 3D lattices (stencil dim 3; Sec. V runs the method in three dimensions as
 * in two).  Every population of the stencil is stored (no merging), the
 * moments are the 14 components of N^a and T^ab, the Landau frame has three
 * velocity components (Newton on the quartic characteristic polynomial of
 * T eta; RLBM_LANDAU_NEWTON only), the equilibrium uses all 14 projections
 * (Appendix B) and a population streams by its 3D vector n_i.  Layout: lat->nz
 * planes of ny storage rows of q class rows (x fastest) with ghost columns,
 * rows and planes of the stencil's reach; bc_x, bc_y, bc_z per axis.
 * rlbm_population_bytes3 gives the buffer size (0 for other stencils).
 * rlbm_init_fields3 sets f = f^eq(n, T, u) from device float64 fields n, T,
 * ux, uy, uz of nx*ny*nz values (index (z*ny + y)*nx + x), with the same
 * ownership, checks and errors as rlbm_init_fields; rlbm_step advances it;
 * rlbm_moments3 writes n, eps, T, P, ux, uy, uz (any may be NULL) and raw14
 * (device float64 [14][nz][ny][nx] or NULL: N^0, N^x, N^y, N^z, T^00, T^0x,
 * T^0y, T^0z, T^xx, T^xy, T^xz, T^yy, T^yz, T^zz) of the pre-collision
 * state.  The learned guess and the warm start are 1D/2D only.
 */
size_t rlbm_population_bytes3(const rlbm_ctx* ctx, int nx, int ny, int nz);
int rlbm_init_fields3(rlbm_ctx* ctx, const rlbm_lattice_desc* lat, const double* n, const double* T,
                      const double* ux, const double* uy, const double* uz, void* popA, void* popB,
                      size_t pop_bytes, void* stream);
int rlbm_moments3(rlbm_ctx* ctx, double* n, double* eps, double* T, double* P, double* ux, double* uy, double* uz,
                  double* raw14, void* stream);

/*
 * Advances nsteps time steps (collide, then stream; eq.
 * discrete-relativistic-boltzmann): per site, moments N^a, T^ab
 * (eq. mj-discrete-second-moment), Landau frame (eqs. landau-lifshitz-*),
 * EOS inversion (eq. relativistic-eos), projections (Appendix B), equilibrium
 * (eq. mj-discrete-feq), Anderson-Witting relaxation and exact streaming.
 * Third-order stencils (order 3) take the equilibrium of eq.
 * mj-projected-distribution at N = 3 instead (30 polynomials).
 * Asynchronous on stream; launch errors are returned at once (RLBM_EHIP).
 * Issues kernel launches only (no allocation, memset, copy or
 * synchronisation), so the steps can be recorded by stream capture and
 * replayed; the context's step count and current buffer advance when the
 * steps are recorded, so a recording holds an even number of steps and
 * starts after the first step.
 * Health flags accumulate on the device: the call returns before any site
 * is computed, so a fatal flag is reported by rlbm_get_health (RLBM_ENUMERIC)
 * and not by this call; RLBM_ESTATE before rlbm_init_fields.
 */
int rlbm_step(rlbm_ctx* ctx, int nsteps, void* stream);

/*
 * Writes the macroscopic fields of the current state f(x, t), which is the
 * pre-collision state: a step collides, then streams (eq.
 * discrete-relativistic-boltzmann), and the fields are those of eqs.
 * landau-lifshitz-* and relativistic-eos for the moments of f(x, t):
 * n, eps, T, P = nT, ux, uy (device float64, nx*ny each, any may be NULL) and
 * raw9 (device float64 [9][ny][nx] or NULL): N^0, N^x, N^y, T^00, T^0x,
 * T^0y, T^xx, T^xy, T^yy.
 */
int rlbm_moments(rlbm_ctx* ctx, double* n, double* eps, double* T, double* P, double* ux, double* uy,
                 double* raw9, void* stream);

/* Synchronises stream, returns the OR of the health flags in *flags (host)
 * and the Landau iteration statistics (sum over sites and max since the
 * last reset, host, nullable); RLBM_ENUMERIC if a fatal flag is set.
 * reset != 0 clears them afterwards. */
int rlbm_get_health(rlbm_ctx* ctx, unsigned* flags, unsigned long long* landau_iter_sum,
                    unsigned* landau_iter_max, int reset, void* stream);

/* Completed time steps since rlbm_init_fields. */
long long rlbm_step_count(const rlbm_ctx* ctx);

/*
 * Step kernel selection.  The same time step (Sec. III, eqs. mj-discrete-feq
 * and discrete-relativistic-boltzmann) is available in two forms: the
 * table-driven kernel, which reads each class's moment and equilibrium rows
 * from the stencil table, and, for the stencils of the configured workloads
 * in float32 and float16 storage, a kernel compiled with those rows as
 * constants and the class loops factored by the square's symmetry (built by
 * gen_fixed_stencils.cpp from the library's own table builder; used only when
 * the context's table matches bit for bit; for float32 storage also with
 * the learned Landau guess).  Both compute the same arithmetic up to
 * rounding order.
 * rlbm_set_step_variant: RLBM_STEP_AUTO (default: the fixed-stencil kernel
 * when one matches) or RLBM_STEP_TABLE (always the table-driven kernel);
 * RLBM_EINVAL on other values.  rlbm_step_kernel: which kernel the next
 * rlbm_step runs (RLBM_STEP_TABLE or RLBM_STEP_FIXED); RLBM_EINVAL for NULL.
 */
#define RLBM_STEP_AUTO 0
#define RLBM_STEP_TABLE 1
#define RLBM_STEP_FIXED 2
int rlbm_set_step_variant(rlbm_ctx* ctx, int variant);
int rlbm_step_kernel(const rlbm_ctx* ctx);

/* Copies the current state (population buffer in storage precision, as laid
 * out by the library) to dst (device or host, pop_bytes) and back; with the
 * step count this is the whole state (checkpoint / resume). */
int rlbm_save_state(rlbm_ctx* ctx, void* dst, size_t bytes, long long* step, int* layout_flag, void* stream);
int rlbm_load_state(rlbm_ctx* ctx, const void* src, size_t bytes, long long step, int layout_flag, void* stream);

/*
 * Learned initial guess of the Landau-frame solve (an addition to the paper's
 * method).  A 9 -> 64 -> 64 -> 64 -> 3 perceptron with SiLU activations maps
 * the nine moments of a site divided by N^0 to (eps/N^0, u_x, u_y); inputs
 * and outputs are standardised with norm = mx[9], sx[9], my[3], sy[3].
 * params (9155 floats): W1 [64x9], b1[64], W2 [64x64], b2[64], W3 [64x64],
 * b3[64], W4 [3x64], b4[3], row-major, z = W a + b.  The library keeps float32
 * master weights and uses their bfloat16 roundings in every product with
 * float32 accumulation.  rlbm_mlp_create copies params and norm (host) and
 * allocates the training buffers for batches up to max_batch.
 */
typedef struct rlbm_mlp rlbm_mlp;
int rlbm_mlp_create(rlbm_mlp** out, const float* params, const float* norm, int max_batch);
int rlbm_mlp_destroy(rlbm_mlp* m);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the mean squared error
 * of the standardised outputs.  raw9: device [B][9] moments (N^0, N^x, N^y,
 * T^00, T^0x, T^0y, T^xx, T^xy, T^yy); target: device [B][3] (eps, u_x, u_y)
 * of the converged Landau frame.  loss (host, nullable) receives the loss
 * before the step (synchronises stream). */
int rlbm_mlp_train_step(rlbm_mlp* m, const float* raw9, const float* target, int B, float lr, float* loss,
                        void* stream);

/* pred: device [B][3] = (eps, u_x, u_y) predicted from raw9 (device [B][9]). */
int rlbm_mlp_predict(rlbm_mlp* m, const float* raw9, int B, float* pred, void* stream);

/* Copies the float32 master weights and the last gradients (host, nullable). */
int rlbm_mlp_get_params(rlbm_mlp* m, float* params, float* grads);

/* Makes every later rlbm_step of ctx start its Landau solve from the network's
 * guess (NULL: from T^00, or from u = 0 for the fixed point).  The network
 * must outlive its use by ctx.  The solve that follows is unchanged, so the
 * fields agree with the unguided path to the Landau tolerance. */
int rlbm_set_landau_guess(rlbm_ctx* ctx, const rlbm_mlp* m);

/* Diagnostic: the network's guess for the current state, evaluated by the
 * same in-kernel inference as rlbm_step: out (device float32 [3][ny][nx]) =
 * eps, u_x, u_y.  RLBM_ESTATE without fields or network. */
int rlbm_landau_guess_fields(rlbm_ctx* ctx, float* out, void* stream);

/* Warm start of the Landau-frame solve (Sec. II.A): makes every later
 * rlbm_step of ctx start the solve at each site from the frame (eps, u_x,
 * u_y) that the site converged to in the previous step, kept in a
 * library-owned device buffer of 3 nx ny float32 values (allocated and
 * cleared here, never inside rlbm_step; freed by rlbm_destroy).  The first
 * step after enabling starts as without it.  The solve that follows is
 * unchanged, so the fields agree with the plain path to the Landau
 * tolerance.  enable = 0 turns it off (the buffer is kept for reuse); a
 * later rlbm_init_fields turns it off too.  RLBM_ESTATE without fields,
 * RLBM_EINVAL while a learned guess is set (the two are exclusive; so
 * rlbm_set_landau_guess returns RLBM_EINVAL while the warm start is on). */
int rlbm_set_warm_start(rlbm_ctx* ctx, int enable);

/*
 * Batched 1D problems in one persistent launch.  Each problem is an Nx x 1
 * lattice with outflow ends, float32 deviation storage and tau from eta/s
 * (rlbm_lattice_desc's RLBM_TAU_ETA_OVER_S rule), using one of the given
 * stencil contexts (rlbm_init_stencil with dim 1, RLBM_FP32_DEV, at most 24
 * classes; they must outlive the batch).  The sites of all problems are cut
 * into tiles of 64 sites, one wave each; a cooperative launch spread over the
 * whole device advances every tile through all steps of a call.  There is
 * no grid-wide barrier between steps: a tile starts step t once its two
 * neighbours in the same problem have finished step t - 1 (streaming reaches
 * at most max |n_x| < 64 sites), and every problem is kept on one L2 (one
 * XCD) so that this hand-over needs no device-wide cache maintenance.  A
 * wait that does not end, or tiles of one problem found on two L2s, raise
 * RLBM_H_SYNC (fatal) and end the launch early.
 */
typedef struct {
  int nx;                 /* sites */
  int stencil;            /* index into the stencils of rlbm_batch_create */
  double eta_over_s, T_R_GeV, n_unit_fm3, dx_fm;
} rlbm_problem;
typedef struct rlbm_batch rlbm_batch;
int rlbm_batch_create(rlbm_batch** out, int nstencils, rlbm_ctx* const* stencils, int nprob, const rlbm_problem* probs,
                      double landau_tol, int landau_maxit);
int rlbm_batch_destroy(rlbm_batch* b);
/* bytes of one population buffer; total sites (sum of nx) */
size_t rlbm_batch_population_bytes(const rlbm_batch* b);
long long rlbm_batch_sites(const rlbm_batch* b);
/* f = f^eq(n, T, u_x) from device float64 fields concatenated over the
 * problems (sum of nx each); popA, popB: caller-owned device buffers. */
int rlbm_batch_init(rlbm_batch* b, const double* n, const double* T, const double* ux, void* popA, void* popB,
                    size_t bytes, void* stream);
/* nsteps steps of every problem in one launch.  samples (device, nullable):
 * at every step t (0-based within the call) with t % sample_every == 0, the
 * pre-collision state of every site as 12 floats (N^0, N^x, N^y, T^00, T^0x,
 * T^0y, T^xx, T^xy, T^yy, eps, u_x, u_y): training pairs for the learned
 * guess; layout [t / sample_every][site][12]. */
int rlbm_batch_step_persistent(rlbm_batch* b, int nsteps, int sample_every, float* samples, void* stream);
/* The cooperative grid of rlbm_batch_step_persistent (host, nullable):
 * workgroups of 256 threads launched, the most the device holds at once for
 * this kernel (the grid never exceeds it), and the number of 64-site tiles. */
int rlbm_batch_occupancy(const rlbm_batch* b, int* workgroups, int* resident_limit, int* tiles);
/* pre-collision fields (device float64, concatenated; any may be NULL) */
int rlbm_batch_moments(rlbm_batch* b, double* n, double* eps, double* T, double* P, double* ux, void* stream);
/* OR of the health flags and Landau iteration statistics of all problems
 * (synchronises stream); RLBM_ENUMERIC if a fatal flag is set. */
int rlbm_batch_get_health(rlbm_batch* b, unsigned* flags, unsigned long long* iter_sum, unsigned* iter_max,
                          void* stream);

/*
 * Measurement utility: copies bytes (a multiple of 16) from src to dst
 * (device buffers, not overlapping) with a plain streaming kernel of the
 * given number of 256-thread workgroups, asynchronously on stream.  Its rate
 * is the achievable HBM ceiling against which the step's traffic is
 * reported.  Errors: RLBM_EINVAL, RLBM_EHIP.
 */
int rlbm_device_copy(void* dst, const void* src, size_t bytes, int workgroups, void* stream);

/* Last error message of ctx (or of the last failed context-less call when
 * ctx is NULL).  The string is owned by the library. */
const char* rlbm_last_error(const rlbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* RLBM_H */

/* hrx: right-hand side and explicit Runge-Kutta stage of the multi-species reacting
 * compressible Navier-Stokes equations on a structured grid, for AMD MI355X (gfx950).
 *
 * The method is that of Margaritis et al., "Development of a high-fidelity
 * computational tool for chemically reacting hypersonic flow simulations"
 * (arXiv 2210.05547): the governing equations of Sec. 2.1 in the compact flux form of
 * Eqs. (5)-(6), nondimensionalised by Eq. (7), with the thermodynamic, transport
 * and finite-rate chemistry models of Sec. 2.2, the sponge of Eq. (26) (Sec. 3.2),
 * artificial-diffusivity shock capturing (Sec. 3.3) and low-storage explicit
 * Runge-Kutta stages (Sec. 3.1).
 *
 * Conventions for every call below.
 *  - Array arguments are DEVICE pointers owned by the caller unless marked (host).
 *    The library never allocates or frees in the compute calls; hrx_create allocates
 *    the context's scratch once.
 *  - Fields are structure-of-arrays planes of doubles, x fastest:
 *    f[v][k][j][i] at offset ((v*nz + k)*ny + j)*nx + i, N = nx*ny*nz points.
 *  - Conserved state Q (nondimensional, Eq. 7):
 *      perfect gases (calorically or thermally perfect, Sec. 2.2.2):
 *                                [rho, rho u, rho v, (rho w), rho E]
 *      5-species air:            [rho_N2, rho_O2, rho_NO, rho_N, rho_O, rho u, rho v,
 *                                 (rho w), rho E]  (all species equations, no global
 *                                 continuity: the alternative named in Sec. 2.1)
 *  - Calls are asynchronous on the given HIP stream (NULL = default stream).  Argument
 *    errors are returned synchronously; per-point failures (energy inversion) are
 *    reported through status arrays and the counters of hrx_get_counters.
 *  - A context is not thread-safe; calls on one context must not overlap.
 *  - Every function returns HRX_OK (0) or a negative hrx_status; nothing aborts.
 */
#ifndef HRX_H
#define HRX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HRX_OK = 0,
  HRX_EINVAL = -1,   /* bad argument or configuration */
  HRX_EHIP = -2,     /* a HIP runtime call failed */
  HRX_ENOMEM = -3,   /* scratch allocation failed in hrx_create */
  HRX_EUNSUP = -4,   /* valid request that the library does not support */
  /* per-point failures found by the kernels (Sec. 3.4: every state evaluation solves a
   * nonlinear equation, which can fail); reported by hrx_get_counters, never by the
   * asynchronous compute calls themselves */
  HRX_ENEWTON = -5,   /* the energy inversion did not converge at some point */
  HRX_EDOMAIN = -6,   /* some energy lay below e(50 K), outside the inversion's domain */
  HRX_ENONFINITE = -7, /* some state held a non-finite value or a non-positive density */
  HRX_ETOOBIG = -8     /* the problem does not fit the static workspace of
                          hrx_rhs_eval_noalloc */
} hrx_status;

enum { HRX_GAS_CPG = 0, HRX_GAS_AIR5 = 1, HRX_GAS_TPG = 2 };
enum { HRX_WALL_ADIABATIC = 0, HRX_WALL_ISOTHERMAL = 1 };
enum { HRX_RK3_2N = 0, HRX_RK45_2N = 1, HRX_SSPRK3 = 2 };
enum { HRX_PREC_FP64 = 0, HRX_PREC_MIXED = 1 };
enum { HRX_THERMO_PLAIN = 0, HRX_THERMO_SURROGATE = 1 };
enum { HRX_DIFF_RAMSHAW = 0, HRX_DIFF_STEFAN_MAXWELL = 1 };
enum { HRX_FD_EXPLICIT = 0, HRX_FD_COMPACT = 1 };

/* Workload description (host).  Sec. 2.1 (reference scales, Eq. 7 and 11), Sec. 3.2
 * (sponges, wall), Sec. 3.3 (artificial diffusivity), Sec. 4 (case parameters). */
typedef struct hrx_config {
  int gas;                  /* HRX_GAS_*: calorically perfect, 5-species air, or thermally
                               perfect air (Sec. 2.2.2) */
  int nx, ny, nz;           /* grid points; nz = 1 for a 2-D problem; nx, ny >= 8 */
  const double *x, *y, *z;  /* (host) separable coordinates, nondimensional; x, y
                               non-periodic, z uniform and periodic (may be NULL if nz = 1) */
  int fd_order;             /* 4 or 6: the order of the first derivatives (fd_scheme) */
  int rk_scheme;            /* HRX_RK3_2N (Williamson), HRX_RK45_2N (Carpenter-Kennedy) or
                               HRX_SSPRK3 (the three-register TVD RK3 of Shu and Osher) */
  int precision;            /* HRX_PREC_FP64, or HRX_PREC_MIXED: FP64 conserved state, RK
                               update, energy inversion, convective fluxes, stencil
                               differences and Arrhenius exponentials at T >= 2000 K;
                               FP32 transport, rate products, viscous/diffusive fluxes,
                               stencil weighted sums and artificial-diffusivity planes */
  int ad_on;                /* artificial diffusivity on/off */
  double ad_coef[5];        /* C_mu, C_beta, C_kappa, C_D, C_Y */
  double gamma, Pr;         /* gamma_inf: perfect gases (CPG, TPG); Pr: CPG only (the
                               thermally perfect gas derives it from Sutherland's and
                               Keyes' laws at T_inf, Sec. 2.2.2) */
  double mach;              /* free-stream Mach number (informational) */
  double T_inf;             /* K */
  double p_inf;             /* Pa (air5) */
  double Re;                /* free-stream Reynolds number (used when L_ref <= 0) */
  double L_ref;             /* m (air5); > 0 fixes L_ref and derives Re */
  double Y_inf[5];          /* free-stream mass fractions (air5) */
  int wall;                 /* HRX_WALL_* at j = 0 */
  double T_wall;            /* K, isothermal wall */
  int sponge_in, sponge_out, sponge_top;  /* sponge extents in points */
  double sigma_max;         /* sponge strength at the boundary (nondimensional) */
  const int64_t *hold;      /* (host) flat indices of held (Dirichlet) points, all in
                               the first three wall rows, or NULL */
  int64_t n_hold;
  int newton_max_iter;      /* <= 0: 50 */
  double newton_rtol;       /* <= 0: 1e-13 */
  int diffusion;            /* HRX_DIFF_RAMSHAW: Eq. (18) with the averaged coefficients of
                               Eq. (19); HRX_DIFF_STEFAN_MAXWELL: the Stefan-Maxwell
                               system of Eq. (17) solved per point (5-species air, else
                               HRX_EUNSUP; artificial diffusivities add a flux of the
                               form of Eq. 18) */
  int fd_scheme;            /* first derivatives of the gradients and the divergence
                               (Sec. 3.1): HRX_FD_EXPLICIT, central differences of order
                               fd_order with one-sided 4th-order ends; HRX_FD_COMPACT,
                               collocated compact (Pade) tridiagonal schemes of order
                               fd_order (6: 6th-order interior, 4th-order Pade next to
                               the ends; 4: Pade) with 3rd-order one-sided compact end
                               rows, cyclic in z; nx <= 2048 (else HRX_EUNSUP).  The
                               fourth differences and filters of the artificial
                               diffusivity are explicit in both. */
} hrx_config;

typedef struct hrx_ctx hrx_ctx;

/* Reference state derived by hrx_create (host), for callers that convert units. */
typedef struct hrx_reference {
  double gamma, Re, Pr, Ec;         /* Ec is the computed value (1 by construction) */
  double T_ref;                     /* K: (gamma_inf - 1) T_inf (Sec. 2.1) */
  double rho_inf, c_inf, mu_inf, kappa_inf, R_inf, L_ref;   /* SI (air5) */
} hrx_reference;

typedef struct hrx_counters {
  int64_t newton_nonconverged;      /* points with no convergence in newton_max_iter */
  int64_t energy_below_min;         /* points with e < e(50 K) */
  int64_t surrogate_fallbacks;      /* points evaluated outside the surrogate's hull */
  int64_t nonfinite;                /* points whose state held a non-finite value or a
                                       non-positive density */
  int64_t negative_density;         /* points with a negative partial (or, for the perfect
                                       gases, total) density: undershoots, counted only */
} hrx_counters;

/* Validate cfg, derive the reference state (Sec. 2.1, Eqs. 7 and 11), the metrics and
 * sponge profiles, and allocate the context's scratch on the current HIP device.
 * Returns HRX_EINVAL for an invalid configuration, HRX_ENOMEM if scratch does not
 * fit.  Runs no kernels. */
int hrx_create(const hrx_config *cfg, hrx_ctx **out);
void hrx_destroy(hrx_ctx *ctx);
int hrx_get_reference(const hrx_ctx *ctx, hrx_reference *out /* (host) */);

/* R = F(Q) - sigma (Q - Q_ref): Eq. (5)-(6) with Eq. (26).  Q, Q_ref, R: [nvar][N].
 * Q_ref may be NULL (no sponge term).  Rows with boundary conditions: the inflow
 * column (i = 0) and held points get R = 0; the wall row (j = 0) gets zero momentum
 * rows.  R must not alias Q. */
int hrx_rhs_eval(hrx_ctx *ctx, const double *Q, const double *Q_ref, double *R,
                 void *hip_stream);

/* hrx_rhs_eval for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same right-hand
 * side, with the scratch planes taken from a static device workspace of
 * HRX_NOALLOC_MAX_BYTES that the library holds on every GPU it runs on (from its first
 * hrx_create there until the process ends) instead of the context's.  The call itself
 * allocates and frees nothing.  Inputs and outputs as in hrx_rhs_eval; the energy
 * inversion starts cold.  The scratch of one call is 8 N (nWd + nF) + s N (nWp + 2 nad)
 * bytes (each part rounded up to 256; s = 8, or 4 in the mixed form): about 336 B per
 * point for 2-D 5-species air without artificial diffusivity, 500 B with it.
 * Returns HRX_ETOOBIG when that exceeds HRX_NOALLOC_MAX_BYTES (nothing runs),
 * HRX_EUNSUP in the surrogate form, HRX_EHIP if the workspace's address could not be
 * obtained.  Every call on one GPU uses the same workspace: calls that overlap on one GPU
 * (other streams, other threads, other contexts) race. */
#define HRX_NOALLOC_MAX_BYTES (64u << 20)
int hrx_rhs_eval_noalloc(hrx_ctx *ctx, const double *Q, const double *Q_ref, double *R,
                         void *hip_stream);

/* One explicit Runge-Kutta stage k = stage mod (number of stages of the scheme), Sec. 3.1
 * (two-register low-storage RK3 and RK4, three-register TVD RK3), then the wall-row
 * update (no-slip, non-catalytic zero-gradient mass fractions, isothermal or adiabatic
 * energy).  Q, dQ: [nvar][N], updated in place.
 *   HRX_RK3_2N, HRX_RK45_2N:  dQ <- A_k dQ + dt R;  Q <- Q + B_k dQ.  dQ must be
 *     zero-initialised before stage 0 or hold the previous stage's register.
 *   HRX_SSPRK3:  stage 0 stores the step's initial state Q0 in dQ and sets
 *     Q <- Q + dt R; stages 1 and 2 set Q <- a_k Q0 + b_k (Q + dt R) with
 *     (a, b) = (3/4, 1/4), (1/3, 2/3).  The three registers are Q, Q0 (in dQ) and R.
 * R: NULL evaluates R = F(Q) - sigma (Q - Q_ref) inside the stage (fused with the
 * update, nothing materialised); otherwise R [nvar][N] is a right-hand side the caller
 * computed (e.g. by hrx_rhs_eval) and Q_ref is not used.  Q_ref as in hrx_rhs_eval.
 * R must not alias Q or dQ. */
int hrx_rk_stage(hrx_ctx *ctx, int stage, double dt, double *Q, double *dQ,
                 const double *Q_ref, const double *R, void *hip_stream);

/* Pointwise 5-species-air state in SI units (Sec. 2.2.1, Sec. 3.4): from density
 * rho [kg/m^3], internal energy e [J/kg] (including formation enthalpies) and mass
 * fractions Y [5][n], return T [K] (Newton inversion of e(T)), p = rho R_mix T [Pa],
 * species enthalpies h [5][n] [J/kg], viscosity mu [Pa s], frozen conductivity kappa
 * [W/(m K)], averaged diffusion coefficients D [5][n] [m^2/s] (Eq. 19) and status
 * [n] (0 converged, 1 no convergence in newton_max_iter, 2 e below e(50 K),
 * 3 a non-finite input or rho <= 0); status may be NULL.  T is also an input: a value
 * in (50 K, 1e5 K) starts the inversion there (a warm start; e(T) is convex, so the
 * root is the same), anything else (0, NaN) starts it cold.  Any of p, h, mu, kappa, D
 * may be NULL to skip it.  ctx must be an air5 context.  No allocation: in the surrogate
 * form the network's outputs go through the context's workspace, in chunks of at most
 * max(N, 2^20) points. */
int hrx_thermo_eval(hrx_ctx *ctx, int64_t n, const double *rho, const double *e,
                    const double *Y, double *T, double *p, double *h, double *mu,
                    double *kappa, double *D, int32_t *status, void *hip_stream);

/* Net mass production rates of the 5-species mechanism (Eqs. 13-15), SI:
 * rho_s [5][n] kg/m^3 and T [n] K -> wdot [5][n] kg/(m^3 s).  ctx: air5 context. */
int hrx_chem_source(hrx_ctx *ctx, int64_t n, const double *rho_s, const double *T,
                    double *wdot, void *hip_stream);

/* Compositions of local thermodynamic equilibrium (Sec. 2.2.1, frozen and equilibrium
 * flow: the composition that minimises the mixture's free energy), SI: density rho [n]
 * kg/m^3, temperature T [n] K and the element-N mass fraction xiN [n] (NULL: the
 * context's free stream, Y_inf) -> mass fractions Y [5][n] and status [n] (NULL to skip):
 * 0 converged, 1 not converged in newton_max_iter, 3 an input not finite, rho or T not
 * positive, or xiN outside [0, 1] (Y NaN).  The minimum is found from its stationarity:
 * every species at (p0/(R_u T)) exp(-g_s/(R_u T) + sum_e a_es lambda_e) with the element
 * potentials lambda_e, which Newton's method takes from the two element balances
 * (stopping at a step below newton_rtol); K_c and g_s as in hrx_chem_source.  ctx:
 * air5 context. */
int hrx_equilibrium(hrx_ctx *ctx, int64_t n, const double *rho, const double *T,
                    const double *xiN, double *Y, int32_t *status, void *hip_stream);

/* Accumulated failure counters; synchronises the context's last stream.  reset != 0
 * zeroes them afterwards.  Returns HRX_OK when no point failed since the last reset,
 * else the most severe failure counted (HRX_ENONFINITE, then HRX_EDOMAIN, then
 * HRX_ENEWTON); *out is filled in either case.  Surrogate fallbacks and negative
 * densities are counted, not failures. */
int hrx_get_counters(hrx_ctx *ctx, hrx_counters *out /* (host) */, int reset);

/* ---- Learned thermochemistry surrogate (motivated by Sec. 5: replacing the costly
 * thermochemical-library calls with a learned model).  Network 7 -> 64 -> 64 -> 64 -> 8,
 * hidden activation max(z, 0)^2, mapping the standardised features of an SI
 * state (rho, e, Y_s) to standardised residuals of (ln T, ln mu, ln kappa,
 * ln(rho D_1)..ln(rho D_5)) (composition: hrx_mlp_set_norm; D_s = exp(y)/rho).
 * Parameters: 9352
 * FP32 values in the order [W1 (64x7, row-major by output), b1, W2 (64x64), b2, W3, b3,
 * W4 (8x64), b4].  Inference and the training forward pass run on the matrix cores in
 * BF16 with FP32 accumulation (weights and layer inputs rounded to BF16, nearest even);
 * the backward pass and Adam run in FP32 on FP32 master parameters. */

/* Allocate the network's parameters, Adam moments and a training workspace for
 * batches of up to max_batch rows (setup call; once per context). */
int hrx_mlp_init(hrx_ctx *ctx, int64_t max_batch);
/* Copy parameters theta [9352] (device, FP32) into the context, zero the Adam moments
 * and prepare the BF16 matrix-core copy. */
int hrx_mlp_set_params(hrx_ctx *ctx, const float *theta, void *hip_stream);
/* Copy the current FP32 parameters to theta_out [9352] (device). */
int hrx_mlp_get_params(hrx_ctx *ctx, float *theta_out, void *hip_stream);
/* Surrogate composition around the network (host arrays).  Inputs: the raw features
 * f = (log10 rho, ln T_c, Y_1..Y_5), with T_c = (e - sum_s Y_s h0_s/M_s) / sum_s Y_s c_s
 * and c_s = (3/2 + 2 r_s) R_s (every mode fully excited), are standardised with
 * in_mean/in_std [7]: x = (f - in_mean)/in_std.  Outputs: (ln T, ln mu, ln kappa,
 * ln(rho D_1..5)) (SI) = out_mean + out_std * net(x) + L [1, x], with out_mean/out_std
 * [8] and L = out_lin [8][8] row-major (NULL: zero).  Training hull: log10 rho in
 * [log10rho_min, log10rho_max], Y_s >= -1e-3, sum_s Y_s e_s(T_lo) <= e <=
 * sum_s Y_s e_s(T_hi), and the mass fraction of the element N,
 * Y_N2 + Y_NO M_N/M_NO + Y_N, in [xiN_min, xiN_max].  HRX_EINVAL for non-positive
 * std entries or empty ranges. */
int hrx_mlp_set_norm(hrx_ctx *ctx, const float *in_mean, const float *in_std,
                     const float *out_mean, const float *out_std, const float *out_lin,
                     double log10rho_min, double log10rho_max, double T_lo, double T_hi,
                     double xiN_min, double xiN_max);
/* Raw surrogate features f [n][7] (device, FP32, row per state) of SI states rho [n],
 * e [n], Y [5][n] (device): (log10 rho, ln T_c, Y_1..Y_5) as defined for
 * hrx_mlp_set_norm above -- the inputs a training set needs.  No hull check. */
int hrx_mlp_features(hrx_ctx *ctx, int64_t n, const double *rho, const double *e,
                     const double *Y, float *f, void *hip_stream);
/* A training set from SI states rho [n], e [n], Y [5][n] (device): raw features
 * F [n][7] (FP64: log10 rho, ln T_c, Y_1..Y_5 as for hrx_mlp_set_norm) and raw targets
 * T [n][8] (ln T, ln mu, ln kappa, ln(rho D_1..5)) of the plain FP64 evaluation (cold
 * energy inversion); status [n] as for hrx_thermo_eval (may be NULL). */
int hrx_mlp_dataset(hrx_ctx *ctx, int64_t n, const double *rho, const double *e,
                    const double *Y, double *F, double *T, int32_t *status, void *hip_stream);
/* The composition around the network from a training set F [n][7], T [n][8] (device,
 * FP64): the features' mean m and standard deviation s (population), the least-squares
 * linear fit L [8][8] of every target in a = (1, (f - m)/s), and the mean rm and
 * standard deviation rs of the residuals r = t - L a (all sums in FP64 on the device, the
 * 8 x 8 normal equations solved on the host); writes the standardised rows
 * Xs [n][7] = (f - m)/s and Ys [n][8] = (r - rm)/rs (FP32, device), installs the
 * composition with the given training hull as hrx_mlp_set_norm does, and returns
 * (host, may be NULL) stats [94] = m [7], s [7], rm [8], rs [8], L [8][8].  Set-up call
 * (synchronises the stream); requires hrx_mlp_init; HRX_EINVAL for n < 2 or a zero
 * spread. */
int hrx_mlp_fit(hrx_ctx *ctx, int64_t n, const double *F, const double *T, float *Xs, float *Ys,
                double log10rho_min, double log10rho_max, double T_lo, double T_hi,
                double xiN_min, double xiN_max, double *stats /* (host) */, void *hip_stream);
/* HRX_THERMO_SURROGATE makes hrx_thermo_eval, hrx_rhs_eval and hrx_rk_stage (air5) take
 * mu, kappa, D_s from the network and start the FP64 energy inversion from its T, for
 * points inside the hull; points outside fall back to the plain evaluation and are
 * counted.  Requires parameters and normalisation to be set. */
int hrx_set_thermo_mode(hrx_ctx *ctx, int mode);
/* Y [n][8] = network(X [n][7]) on standardised rows (device, FP32). */
int hrx_mlp_forward(hrx_ctx *ctx, int64_t n, const float *X, float *Y, void *hip_stream);
/* grad [9352] (device) = d(loss)/d(theta) for the batch X [n][7] (n <= max_batch) given
 * dLdY [n][8] (device). */
int hrx_mlp_backward(hrx_ctx *ctx, int64_t n, const float *X, const float *dLdY,
                     float *grad, void *hip_stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; t counts from 1) with gradient grad. */
int hrx_adam_step(hrx_ctx *ctx, const float *grad, float lr, int t, void *hip_stream);
/* Forward, mean-squared-error gradient against Yt, backward and Adam for the rows
 * idx [n] (device, or NULL for rows 0..n-1) of X [.][7] and Yt [.][8]; the batch's
 * mean squared error is added to *loss (device, may be NULL). */
int hrx_mlp_train_step(hrx_ctx *ctx, int64_t n, const int32_t *idx, const float *X,
                       const float *Yt, float lr, int t, float *loss, void *hip_stream);

/* Per-kernel timing with HIP events recorded on the launching stream around every
 * kernel of the calls that follow hrx_timing_enable(ctx, 1).  Kernel ids (index into
 * the arrays of hrx_timing_read): 0 prim, 1 ad_src, 2 ad_d4 (the fourth difference
 * fused with the x and y filters), 3 and 4 (no launches: the x and y filters run inside
 * 2), 5 ad_filter_z, 6 flux, 7 div, 8 bc (3-D; in 2-D the wall condition runs
 * inside div), 9 thermo_eval,
 * 10 chem_source (in the surrogate form the network pass is counted with prim and
 * thermo_eval), 11 the compact scheme's line solves (gradients and divergence), 12 the
 * compact scheme's pointwise pass (sources, sponge, boundary rows, update), 13
 * equilibrium.
 * hrx_timing_read synchronises, returns the summed milliseconds and launch counts
 * per kernel since enabling (arrays of HRX_NKERNELS, host) and keeps timing on.
 * hrx_timing_enable(ctx, 0) stops and releases the events. */
#define HRX_NKERNELS 14
int hrx_timing_enable(hrx_ctx *ctx, int on);
int hrx_timing_read(hrx_ctx *ctx, double *ms /* (host) */, int64_t *launches /* (host) */);

const char *hrx_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif

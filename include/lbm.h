/*
 * lbm.h -- C ABI of the MI355X (gfx950) coupled thermal lattice Boltzmann step.
 *
 * Method: the double-distribution-function thermal LB model of Xu, Shi & Xi,
 * "Lattice Boltzmann simulations of three-dimensional thermal convective flows
 * at high Rayleigh number", Int. J. Heat Mass Transfer (2019),
 * arXiv:1903.08882:
 *   - a D3Q19 MRT lattice for the flow with Guo forcing of the Boussinesq
 *     buoyancy rho g beta (T - T0) z^ (Sec. 2.2, Eq. MRT);
 *   - a D3Q7 MRT lattice for the temperature with the relaxation rates that
 *     make the fourth-order error isotropic (Sec. 2.3, Eq. MRT_T, Eq. magic,
 *     Eq. 4th, Eq. qnu);
 *   - half-way bounce-back no-slip walls, half-way anti-bounce-back fixed
 *     temperature walls and bounce-back adiabatic walls (Sec. 2.2, 2.3);
 *   - a closed cube: side-heated (Sec. 3) or Rayleigh-Benard (Sec. 4).
 *
 * Geometry and units.  N nodes per side, node (i, j, k) at (i+1/2, j+1/2,
 * k+1/2) lattice units, walls on the planes 0 and N of every axis, cell height
 * H = N.  Gravity points along -z.  Wall temperatures are T_hot = +1/2 and
 * T_cold = -1/2 (dT = 1).  Side-heated: hot wall x = 0, cold wall x = N.
 * Rayleigh-Benard: hot wall z = 0, cold wall z = N.  All other walls are
 * adiabatic.  Lattice parameters follow from (N, Ra, Pr, U) with the
 * free-fall scaling of Sec. 2.1: nu = U H sqrt(Pr/Ra), kappa = U H/sqrt(Ra Pr),
 * g beta = U^2/(H dT).
 *
 * Arrays handed across this ABI.  Field and population arrays are FP64,
 * x fastest: element [q][z][y][x] at q*N^3 + x + N*(y + N*z).  Populations
 * are q = 0..18 for f_0..f_18 and 19..25 for g_0..g_6, in the velocity order
 * of the paper's printed arrays, always the pre-collision values of the
 * current time step.
 *
 * Memory and streams.  The caller owns all device memory (one buffer of
 * lbm_state_bytes() bytes handed to lbm_create) and passes a HIP stream
 * (hipStream_t as void*, NULL = the default stream) to every call that
 * launches work.  Calls that return host values synchronise that stream.
 * Pointers documented as "device" must be device (or managed) memory; the
 * library never dereferences them on the host.
 *
 * Errors.  Every int-returning call returns LBM_OK (0) or a negative code.
 * lbm_last_error(h) describes the last failure on a handle; no call aborts.
 * One handle must not be used from two host threads at once.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#ifndef LBM_API
#define LBM_API __attribute__((visibility("default")))
#endif

typedef struct lbm lbm_t;             /* opaque handle; owned by the library */
typedef struct lbm_batch lbm_batch_t; /* opaque batch of cavities           */

enum lbm_cell { LBM_SIDE_HEATED = 0, LBM_RAYLEIGH_BENARD = 1 };

/* Storage type of the populations in device memory.  Populations are kept as
 * deviations from the rest equilibrium (f_i - w_i, g_i - w_i^T * 0).
 * FP64: FP64 storage and arithmetic.  FP32: FP32 storage and arithmetic.
 * FP16S: f as FP16 scaled deviations, g as FP32; FP32 arithmetic
 * (66 bytes per node instead of 104).  FP16C: as FP16S with f in a customised
 * 16-bit format (sign, 4-bit exponent with bias 18, 11-bit mantissa,
 * subnormals below 2^-17 spaced 2^-28; round to nearest even, magnitudes
 * below 2^-17 first rounded to a multiple of 2^-40; |f_i - w_i| must stay
 * below 1/4, larger values saturate), one mantissa bit more than IEEE half
 * over the deviations' range (the customised 16-bit storage that Lehmann et
 * al., Phys. Rev. E 2022, propose for lattice Boltzmann populations). */
enum lbm_storage { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16S = 2, LBM_FP16C = 3 };

enum lbm_status {
    LBM_OK = 0,
    LBM_EINVAL = -1,    /* bad argument (NULL pointer, size, enum)            */
    LBM_ERANGE = -2,    /* parameters outside the scheme's valid range        */
    LBM_ENOMEM = -3,    /* caller buffer too small, or allocation failed      */
    LBM_EDEVICE = -4,   /* HIP runtime error (text in lbm_last_error)         */
    LBM_EDIVERGED = -5, /* a reduction came back NaN or infinite              */
    LBM_ESTATE = -6,    /* call not valid in the handle's current state       */
    LBM_EIO = -7        /* checkpoint file missing, short, corrupt or foreign */
};

/* Raw observables (lattice units, FP64), indices of the LBM_NRAW vector.
 * Means are over the N^3 nodes, the N^2 nodes of a wall, or the N nodes of a
 * wall's mid-line (the central y index; mean of the two central indices when
 * N is even), running along z (side-heated) or x (Rayleigh-Benard).
 *   FLUX_*: heat entering the fluid through an isothermal wall during the last
 *           step, per link: (6 + a_T)/21 T_w - 2 g_out, the difference the
 *           anti-bounce-back rule makes (Sec. 2.3 boundary scheme).
 *   GRAD_*: -dT/dn into the fluid at the wall, one-sided second-order
 *           difference (-8 T_w + 9 T_0 - T_1)/3 through the wall point and the
 *           first two nodes.
 *   EPS_U:  <nu/2 sum_ij (d_i u_j + d_j u_i)^2>, EPS_T: <kappa |grad T|^2>
 *           (Sec. 4), central differences inside; at the first node next to a
 *           wall the quadratic through the wall value (u = 0, T = T_w) and the
 *           two nearest nodes, -4/3 phi_w + phi_0 + 1/3 phi_1; at an adiabatic
 *           wall a mirror node (dT/dn = 0): (phi_1 - phi_0)/2.
 *   DIV2:   <(div u)^2> with the same differences. */
enum lbm_raw {
    LBM_RAW_FLUX_HOT = 0, LBM_RAW_FLUX_COLD, LBM_RAW_FLUX_HOT_MID, LBM_RAW_FLUX_COLD_MID,
    LBM_RAW_GRAD_HOT, LBM_RAW_GRAD_COLD, LBM_RAW_GRAD_HOT_MID, LBM_RAW_GRAD_COLD_MID,
    LBM_RAW_U2, LBM_RAW_W2, LBM_RAW_WT, LBM_RAW_UT, LBM_RAW_EPS_U, LBM_RAW_EPS_T,
    LBM_RAW_DRHO2, LBM_RAW_T, LBM_RAW_DRHO, LBM_RAW_DIV2,
    LBM_NRAW
};

/* Nondimensional observables (free-fall units u/U, T/dT, lengths in H),
 * indices of the LBM_NOBS vector filled by lbm_nondimensional().
 * Nu by link flux: FLUX * H/(kappa dT); Nu by difference: GRAD * H/dT (the
 * cold wall's sign flipped so both are positive); Nu_vol = 1 + sqrt(Ra Pr)
 * <w* T*> (Rayleigh-Benard) or <u* T*> (side-heated); Re = sqrt(<|u|^2>) H/nu,
 * Re_w = sqrt(<w^2>) H/nu; eps_u* = eps_u H/U^3, eps_T* = eps_T H/(U dT^2);
 * Nu_kin = 1 + sqrt(Ra Pr) eps_u*, Nu_th = sqrt(Ra Pr) eps_T* (Sec. 4);
 * E = <|u*|^2>/2 (Sec. 3); rms(rho - 1); <T>; rms(div* u*) (Sec. 3). */
enum lbm_obs {
    LBM_NU_HOT = 0, LBM_NU_COLD, LBM_NU_HOT_MID, LBM_NU_COLD_MID,
    LBM_NU_HOT_FD, LBM_NU_COLD_FD, LBM_NU_HOT_MID_FD, LBM_NU_COLD_MID_FD,
    LBM_RE_RMS, LBM_RE_W, LBM_NU_VOL, LBM_EPS_U, LBM_EPS_T, LBM_NU_KIN, LBM_NU_TH,
    LBM_E_KIN, LBM_RMS_DRHO, LBM_MEAN_T, LBM_RMS_DIV,
    LBM_NOBS
};

typedef struct {
    double U;         /* free-fall velocity sqrt(g beta dT H) in lattice units;
                         default 0.1/sqrt(3), i.e. Mach 0.1 (Sec. 3)          */
    double T0;        /* reference temperature of the buoyancy; default 0    */
    int sample_every; /* lbm_step adds the observables to the time averages
                         every this many steps (0 = never; default 0)          */
    int block;        /* threads per block of the step kernel: 64, 128, 192
                         or 256 (the step kernels are compiled for at most
                         256 threads per block); 0 = library default (256);
                         anything else gives LBM_EINVAL from lbm_create      */
    int waves_even;   /* occupancy cap of the step kernel, waves per SIMD, for
                         even and odd steps: 1..8, 0 = library default for the
                         storage type (FP32: 2 and 3; FP16S: 3 and none; FP16C:
                         none and none; FP64: 2 and 2), -1 = no cap.  The cap reserves otherwise unused
                         LDS per block; fewer concurrent waves per SIMD spread
                         fewer HBM streams and measured faster for these steps */
    int waves_odd;
} lbm_opts;

/* Lattice parameters derived from (N, Ra, Pr, cell, opts). */
typedef struct {
    int N, cell, storage;
    double Ra, Pr, U, T0, T_hot, T_cold, H, dT;
    double nu, kappa, gbeta;
    double tau_f, s_e, s_q;   /* s_e = s_eps = s_nu = s_pi = 1/tau_f; s_q = s_m */
    double q_k, q_e, q_nu, a_T;
    double wT0, wT1;          /* D3Q7 weights (1 - a_T)/7 and (6 + a_T)/42     */
} lbm_params;

/* Fill *o with the defaults above. */
LBM_API void lbm_default_opts(lbm_opts *o);

/* Host only.  Derive the lattice parameters (Sec. 2.1-2.3):
 *   tau_f = 3 nu + 1/2, s_q = s_m = 8(2 tau_f - 1)/(8 tau_f - 1),
 *   q_k = 3 - sqrt 3, q_e = q_nu = 4 sqrt 3 - 6, a_T = 42 sqrt 3 kappa - 6.
 * opts may be NULL (defaults).  LBM_EINVAL for N < 3, a bad cell or storage,
 * Ra, Pr or U not positive or not finite; LBM_ERANGE when a_T leaves (-6, 1],
 * where a D3Q7 weight would turn negative (kappa > 1/(6 sqrt 3)). */
LBM_API int lbm_derive_params(int N, double Ra, double Pr, int cell, int storage,
                      const lbm_opts *opts, lbm_params *out);

/* Host only.  Bytes of device memory a handle of size N and storage type
 * needs (populations, macro planes, residual snapshot, reduction scratch). */
LBM_API int lbm_state_bytes(int N, int storage, size_t *bytes);

/* Create a handle.  dev_buf: device buffer of at least lbm_state_bytes()
 * bytes, 256-byte aligned, owned by the caller and kept alive until
 * lbm_destroy; NULL makes the library allocate (and free) it itself.  The
 * populations are undefined until lbm_set_fields or lbm_set_populations. */
LBM_API int lbm_create(int N, double Ra, double Pr, int cell, int storage, const lbm_opts *opts,
               void *dev_buf, size_t buf_bytes, lbm_t **out);

/* Destroy a handle (frees only what the library allocated). */
LBM_API int lbm_destroy(lbm_t *h);

LBM_API int lbm_get_params(const lbm_t *h, lbm_params *out);

/* Initialise from fields: rho = 1, f = f^eq(1, u) (Sec. 2.2), g = g^eq(T, u)
 * (Sec. 2.3).  uvwT: device FP64 array [4][N^3] holding u, v, w, T.  Resets
 * the step counter, the time averages and the residual snapshot. */
LBM_API int lbm_set_fields(lbm_t *h, const double *uvwT, void *stream);

/* Macroscopic fields of the current state (Sec. 2.2, 2.3):
 * rho = sum f, T = sum g, u = (sum e f + F/2)/rho with F = rho g beta (T - T0) z^.
 * out: device FP64 array [5][N^3] receiving rho, u, v, w, T. */
LBM_API int lbm_get_fields(lbm_t *h, double *out, void *stream);

/* Replace the populations.  in: device FP64 array [26][N^3] of pre-collision
 * populations.  Keeps the step counter; resets the time averages and the
 * residual snapshot.  The values are rounded to the storage type. */
LBM_API int lbm_set_populations(lbm_t *h, const double *in, void *stream);

/* Pre-collision populations of the current time step.  out: device FP64
 * array [26][N^3]. */
LBM_API int lbm_get_populations(lbm_t *h, double *out, void *stream);

/* Advance n >= 0 coupled time steps (Eq. MRT and Eq. MRT_T with the wall
 * rules), asynchronously on stream.  With opts.sample_every = K > 0 the
 * observables of every K-th state are added to the time averages. */
LBM_API int lbm_step(lbm_t *h, int64_t n, void *stream);

/* Steps taken since lbm_set_fields. */
LBM_API int64_t lbm_time(const lbm_t *h);

/* Raw observables (enum lbm_raw) of the current state; synchronises stream.
 * The FLUX_* entries refer to the last step taken (zero meaning before the
 * first step after lbm_set_fields/lbm_set_populations).  LBM_EDIVERGED when
 * any entry is not finite. */
LBM_API int lbm_observables_raw(lbm_t *h, void *stream, double raw[LBM_NRAW]);

/* Instantaneous headline observables of the current state, nondimensional:
 * Nu = mean of the hot- and cold-wall link-flux Nusselt numbers, Re = Re_rms,
 * eps_u* and eps_T* volume means (Sec. 4).  Any output pointer may be NULL. */
LBM_API int lbm_observables(lbm_t *h, void *stream, double *Nu, double *Re, double *eps_u,
                    double *eps_T);

/* Host only.  Convert a raw vector to the LBM_NOBS nondimensional numbers. */
LBM_API int lbm_nondimensional(const lbm_params *p, const double raw[LBM_NRAW],
                       double out[LBM_NOBS]);

/* Time averages: the mean raw vector over the states sampled by lbm_step
 * since the last reset, and the number of samples; synchronises stream.
 * LBM_ESTATE when no sample was taken yet. */
LBM_API int lbm_averages(lbm_t *h, void *stream, double raw_mean[LBM_NRAW], int64_t *count);
LBM_API int lbm_reset_averages(lbm_t *h, void *stream);

/* Steady-state residual against the state recorded at the previous call (or
 * at initialisation), then record the current state (Sec. 3 criterion):
 *   max_dT   = max |T - T_old|
 *   rel_L1_T = sum |T - T_old| / sum |T_old|
 *   rel_L2_u = sum ||u - u_old||_2 / sum ||u_old||_2
 * Synchronises stream.  Any output pointer may be NULL. */
LBM_API int lbm_residual(lbm_t *h, void *stream, double *max_dT, double *rel_L1_T,
                 double *rel_L2_u);

/* Checkpoint and restart of one cavity (not part of the paper's method; long
 * Rayleigh-Benard averaging runs need it).  lbm_save writes, to the host file
 * at path, a header (N, cell, storage, Ra, Pr, U, T0, step count, AA parity,
 * sample count), the population storage exactly as it sits in device memory,
 * the FP64 time-average accumulators and a 64-bit FNV-1a checksum of all of
 * it; it synchronises stream.  lbm_load reads such a file into a handle
 * created with the same N, cell, storage, Ra, Pr, U and T0 (LBM_EINVAL
 * otherwise), restores the step count, the parity and the time averages, and
 * records the loaded state as the residual reference; the wall flux of the
 * step before the save is not kept (observables need one step first, as after
 * lbm_set_populations).  Stepping a loaded handle continues bit for bit as
 * the saved one would have.  LBM_EIO for a file that cannot be opened, read
 * or written, is short, or fails its magic or checksum; LBM_ESTATE when
 * saving a handle whose populations were never set, or loading into a
 * cavity of a batch. */
LBM_API int lbm_save(lbm_t *h, const char *path, void *stream);
LBM_API int lbm_load(lbm_t *h, const char *path, void *stream);

/* Steady-state driver (Sec. 3 criterion, with the maximum change of T as the
 * stopping measure): repeat { lbm_step(check_every); lbm_residual } until
 * max |T - T_old| < tol_max_dT or max_steps steps have been taken.  Writes the
 * steps taken, the last max_dT and, when history != NULL, up to history_len
 * max_dT values (one per check).  Returns LBM_OK whether or not it converged
 * (compare *final_max_dT with tol_max_dT); errors as lbm_step/lbm_residual. */
LBM_API int lbm_run_to_steady(lbm_t *h, int64_t check_every, double tol_max_dT,
                              int64_t max_steps, void *stream, int64_t *steps_taken,
                              double *final_max_dT, double *history, int64_t history_len);

/* Mid-plane centreline maxima of the side-heated benchmark (Sec. 3, Table 1),
 * in this library's axes (hot wall x = 0): out[0] = max u/U on the vertical
 * line x = y = 1/2 and out[1] its height z/H; out[2] = max w/U on the
 * horizontal line y = z = 1/2 and out[3] its position x/H; out[4] = E =
 * <|u|^2>/(2 U^2).  Nodal values at (i + 1/2)/N; for even N the two central
 * lines are averaged.  Synchronises stream. */
LBM_API int lbm_centerline_peaks(lbm_t *h, void *stream, double out[5]);

/* Plane-averaged Nusselt number across the cell (Sec. 3: the Nu(y) profile
 * of its Fig. 4, from the hot to the cold wall; here along x for the
 * side-heated cell and along z for Rayleigh-Benard).  out[k], k = 0..N-1, is
 * the heat carried through the node plane at (k + 1/2)/N of that axis a, by
 * convection and conduction, in units of the conduction flux kappa dT/H:
 *   Nu(k) = H/(kappa dT) (<u_a T>_k - kappa <d_a T>_k),
 * means over the plane's N^2 nodes, d_a T with the differences of the
 * observables (central inside; at the first node next to a wall the
 * quadratic through the wall temperature).  Linear conduction gives 1 on
 * every plane; in a steady state every plane carries the same heat, so the
 * profile is flat up to the differences' truncation error.  out: host array
 * of N doubles.  Synchronises stream; LBM_EDIVERGED when a value is not
 * finite. */
LBM_API int lbm_nusselt_profile(lbm_t *h, void *stream, double *out);

/* Fields (u, v, w, T) trilinearly resampled onto M^3 node-centred points
 * (i + 1/2)/M, FP32 [4][M^3] in device memory.  Per axis the samples are the
 * nodes and, beyond the outermost nodes, the walls: u = v = w = 0 on all
 * walls, T = T_w on the isothermal walls, T held at the nearest node along
 * the adiabatic axes.  M >= 2. */
LBM_API int lbm_resample_fields(lbm_t *h, int M, float *out, void *stream);

/* Block-size autotuner: times the step kernel with 64, 128, 192 and 256
 * threads per block (steps_per_candidate steps each, HIP events on stream)
 * and keeps the fastest for this handle.  Results are cached per (N,
 * storage, cell) for the life of the process; a cached entry is reused
 * without timing.  The steps taken while timing advance the state like
 * lbm_step.  *best_ms is the mean step time of the winner (0 if cached). */
LBM_API int lbm_autotune(lbm_t *h, void *stream, int steps_per_candidate, int *best_block,
                         double *best_ms);

/* ---------------------------------------------------------------------------
 * Batches: K independent cavities (own N, Ra, Pr, cell; one storage type)
 * advanced together, one kernel launch per step for all of them, so that
 * small lattices are not launch bound.  Each cavity is an ordinary handle
 * (lbm_batch_cavity) whose memory is a slice of the batch buffer: use it to
 * set and read fields, observables and residuals.  A cavity handle of a batch
 * cannot be stepped on its own (LBM_ESTATE); set its fields only while the
 * batch has taken an even number of steps.
 * ------------------------------------------------------------------------- */
LBM_API int lbm_batch_state_bytes(int K, const int *N, int storage, size_t *bytes);
LBM_API int lbm_batch_create(int K, const int *N, const double *Ra, const double *Pr,
                             const int *cell, int storage, const lbm_opts *opts, void *dev_buf,
                             size_t buf_bytes, lbm_batch_t **out);
LBM_API int lbm_batch_destroy(lbm_batch_t *b);
LBM_API int lbm_batch_cavity(lbm_batch_t *b, int k, lbm_t **h);

/* Advance every active cavity by n steps (asynchronous on stream). */
LBM_API int lbm_batch_step(lbm_batch_t *b, int64_t n, void *stream);

/* Steady-state loop over the batch: every check_every steps each active
 * cavity's max |dT| is taken (as lbm_residual); cavities below tol_max_dT
 * retire (are no longer stepped).  Stops when all have retired or after
 * max_steps.  A cavity whose residual is not finite (diverged) retires too,
 * with res_k = NaN, and the others go on.  steps_k[k] = steps cavity k took,
 * res_k[k] = its last max |dT| (either may be NULL). */
LBM_API int lbm_batch_run_to_steady(lbm_batch_t *b, int64_t check_every, double tol_max_dT,
                                    int64_t max_steps, void *stream, int64_t *steps_k,
                                    double *res_k);

/* Autotuner for the batched launch (as lbm_autotune, not cached). */
LBM_API int lbm_batch_autotune(lbm_batch_t *b, void *stream, int steps_per_candidate,
                               int *best_block, double *best_ms);

LBM_API const char *lbm_batch_last_error(const lbm_batch_t *b);

/* Reference device copy for measuring the practical HBM bandwidth that the
 * step kernels are compared against (not part of the method): copies bytes
 * from src to dst, both device memory, with 16-byte streaming loads and
 * stores on stream (asynchronous).  bytes must be a multiple of 16 and both
 * pointers 16-byte aligned; the ranges must not overlap (LBM_EINVAL
 * otherwise); LBM_EDEVICE when the launch fails. */
LBM_API int lbm_device_copy(void *dst, const void *src, size_t bytes, void *stream);

/* Kernel timing.  With profiling enabled, lbm_step brackets every step
 * kernel it launches with a pair of HIP events on its stream.
 * lbm_profile_read synchronises, returns the summed duration (ms) and number
 * of step kernels timed since the previous read, and starts a new count. */
LBM_API int lbm_profile(lbm_t *h, int enable);
LBM_API int lbm_profile_read(lbm_t *h, double *kernel_ms, int64_t *kernels);

LBM_API const char *lbm_last_error(const lbm_t *h);
LBM_API const char *lbm_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */

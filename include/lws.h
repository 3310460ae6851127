/* lws.h -- C ABI of the learned warm start for the thermal lattice Boltzmann
 * library (lbm.h): a small 3-D convolutional encoder-decoder, conditioned on
 * (log Ra, Pr), that predicts the steady fields of a side-heated cavity, and
 * the kernels it is trained with.  The network is not part of the method of
 * Xu, Shi & Xi (arXiv:1903.08882); it supplies the initial state (Sec. 3 starts
 * from rest), and the paper's steady-state criterion decides when a run
 * started from it has converged.
 *
 * Precision: convolutions take bfloat16 operands (round to nearest even from
 * FP32) on the gfx950 matrix cores and accumulate in FP32; everything else,
 * the master parameters and the optimiser run in FP32; loss and FiLM
 * gradient sums in FP64.
 *
 * Layouts (all device memory unless stated): activations are channels-last,
 * [B][D][H][W][C] with x fastest among the spatial indices; convolution
 * weights are FP32 [27][Cin][Cout] with tap t = 9 (dz + 1) + 3 (dy + 1) +
 * (dx + 1) reading the input at (z + dz, y + dy, x + dx), zero outside the
 * grid (3x3x3 cross-correlation, stride 1, "same" size).
 *
 * Every call returns an lbm_status (LBM_OK, LBM_EINVAL for bad sizes or NULL
 * pointers, LBM_ENOMEM, LBM_EDEVICE with the HIP error text in
 * lws_last_error()).  Calls that take a stream are asynchronous unless they
 * return host values.
 */
#ifndef P1903_LWS_H
#define P1903_LWS_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { int B, D, H, W; } lws_grid;

/* ---- kernels ----------------------------------------------------------- */

/* Elements of a packed bfloat16 weight operand: forward packing holds
 * ceil(Cout/16)*16 rows of ceil(27 Cin/32)*32; data-gradient packing the same
 * with Cin and Cout exchanged. */
LBM_API size_t lws_packed_elems(int cin, int cout, int for_data_grad);

/* Pack FP32 weights w [27][cin][cout] into the bfloat16 operand of
 * lws_conv3d_forward (for_data_grad = 0: row co holds w[t][ci][co] at
 * column t*cin + ci) or of the data gradient (for_data_grad = 1: row ci holds
 * w[26 - t][ci][co] at column t*cout + co, the adjoint's taps mirrored).
 * Padding rows and columns are zero. */
LBM_API int lws_pack_weights(const float *w, int cin, int cout, int for_data_grad,
                             uint16_t *packed, void *stream);

/* z[b][v][co] = sum_t sum_ci x[b'][v + off_t][ci] w[t][ci][co], FP32 out
 * [B][D][H][W][cout].  x is bfloat16 [B][D][H][W][cin] (b' = b) or, with
 * x_shared != 0, [1][D][H][W][cin] used by every sample (b' = 0).  packed is
 * lws_pack_weights(w, cin, cout, 0).  cin must be a multiple of 8,
 * 1 <= cout <= 64. */
LBM_API int lws_conv3d_forward(const uint16_t *x, int x_shared, int cin, const uint16_t *packed,
                               int cout, float *z, lws_grid g, void *stream);

/* Gradient with respect to the input: dx[b][u][ci] = sum_t sum_co
 * dz[b][u - off_t][co] w[t][ci][co], FP32 out [B][D][H][W][cin], from
 * bfloat16 dz [B][D][H][W][cout] and packed = lws_pack_weights(w, cin, cout,
 * 1).  cout must be a multiple of 8, 1 <= cin <= 128. */
LBM_API int lws_conv3d_backward_data(const uint16_t *dz, int cout, const uint16_t *packed,
                                     int cin, float *dx, lws_grid g, void *stream);

/* Workspace bytes lws_conv3d_backward_weight needs for these sizes. */
LBM_API size_t lws_wgrad_work_bytes(int cin, int cout, lws_grid g);

/* Gradient with respect to the weights: dw[t][ci][co] = sum_b sum_v
 * x[b'][v + off_t][ci] dz[b][v][co] (b' as in lws_conv3d_forward), FP32 out
 * [27][cin][cout], overwritten.  Per-chunk partial sums go to work (at least
 * lws_wgrad_work_bytes) and are added in a fixed order, so the result does
 * not depend on scheduling.  1 <= cout <= 64. */
LBM_API int lws_conv3d_backward_weight(const uint16_t *x, int x_shared, int cin, const uint16_t *dz,
                                       int cout, float *dw, lws_grid g, void *work,
                                       size_t work_bytes, void *stream);

/* lws_conv3d_backward_weight for callers that cannot allocate device
 * memory (code under HIP graph capture, training loops that must not call
 * hipMalloc): the same arguments without the workspace.  The per-chunk
 * partial sums go to a 64 MiB device array the library holds on each GPU it
 * runs on (looked up on the first call made with that device current, kept
 * until the process ends); the voxel chunks are coarsened where needed so
 * that every size the original accepts fits in it.  No allocation of any
 * kind is made.  The result equals lws_conv3d_backward_weight's up to the
 * rounding of the chunk sums (it is the same where both use the same
 * chunks).  All calls on one GPU share the array, so calls that overlap on
 * one GPU (other streams, other threads) race: serialise them.
 * LBM_EINVAL for bad arguments, LBM_EDEVICE when the array's address cannot
 * be obtained or a launch fails. */
LBM_API int lws_conv3d_backward_weight_noalloc(const uint16_t *x, int x_shared, int cin,
                                               const uint16_t *dz, int cout, float *dw,
                                               lws_grid g, void *stream);

/* Fields predicted on the node-centred M^3 grid (FP32 channels-last
 * [M^3][ld], channels u/U, v/U, w/U, (T - T_mid)/dT first) interpolated
 * trilinearly onto the N^3 lattice nodes (i + 1/2)/N, in lattice units
 * (u*U, T_mid + T* (T_hot - T_cold) with T_mid the mean wall temperature), as
 * FP64 [4][N^3] for lbm_set_fields.  Beyond the outermost grid nodes each axis
 * is anchored at its walls: velocity 0 on every wall, T_hot / T_cold on the
 * isothermal walls (x for side-heated, z for Rayleigh-Benard), the nearest
 * node's T along adiabatic axes.  With symmetrize != 0 (side-heated cell
 * only; ignored otherwise) each node gets the mean of this interpolation over
 * the steady cell's symmetries: the half-turn about the y axis through the
 * centre with T* -> -T* ((x, z) -> (1 - x, 1 - z), (u, w) -> (-u, -w)) and
 * the mirror y -> 1 - y (v -> -v); errors odd under them are removed. */
LBM_API int lws_upsample_fields(const float *pred, int M, int ld, int N, int cell, double U,
                                double T_hot, double T_cold, int symmetrize, double *uvwT,
                                void *stream);

/* ---- the network ------------------------------------------------------- */

/* Architecture on grid levels M, (M+1)/2, (M+3)/4 (M = 1 mod 4, M >= 5) with
 * channels ch = (c1, c2, c3) (multiples of 16, at most 64; 16/32/64 by
 * default):
 *   E1a 8 -> c1, E1b c1 -> c1 (= s1)             on level 0
 *   E2a c1 -> c2 on inject(s1), E2b c2 -> c2 (= s2) on level 1
 *   E3a c2 -> c3 on inject(s2), E3b c3 -> c3 (= s3) on level 2
 *   D2 [interp(s3), s2] -> c2                     on level 1
 *   D1 [interp(D2), s1] -> c1                     on level 0
 *   OUT c1 -> 8 (bias, no FiLM, no activation; channels 0-3 are the fields)
 * Every other layer: z = conv(x); y = z * (1 + Gw c + Gb) + (Bw c + Bb) with
 * the conditioning c = ((log10 Ra - 5.5)/1.5, (Pr - 3.855)/3.145) (FiLM);
 * a = silu(y) = y / (1 + exp(-y)).  inject keeps every second node (node 2i);
 * interp is tensor-product linear interpolation (node 2i = node i, node
 * 2i + 1 = the mean of nodes i and i + 1).  Input features on the
 * node-centred grid (i + 1/2)/M: 2x - 1, 2y - 1, 2z - 1, their squares, the
 * distance to the nearest wall, 1.
 *
 * Flat FP32 parameter vector, layer by layer in the order above: W
 * [27][Cin][Cout], then Gw [Cout][2], Gb [Cout], Bw [Cout][2], Bb [Cout]
 * (FiLM layers) or b [Cout] (OUT). */
typedef struct lws_net lws_net_t;

LBM_API int lws_net_create(int M, int max_batch, const int ch[3], lws_net_t **out);
LBM_API int lws_net_destroy(lws_net_t *net);
LBM_API int64_t lws_net_param_count(const lws_net_t *net);
/* Host FP32 arrays of lws_net_param_count() values; set also clears the
 * optimiser state.  Both synchronise. */
LBM_API int lws_net_set_params(lws_net_t *net, const float *host);
LBM_API int lws_net_get_params(lws_net_t *net, float *host);

/* Forward pass for B <= max_batch samples of parameters ra_pr (host, [B][2] =
 * Ra, Pr): out is FP32 [B][M^3][8] channels-last. */
LBM_API int lws_net_forward(lws_net_t *net, int B, const double *ra_pr, float *out, void *stream);

/* Loss and gradient: forward, then mean squared error over the 4 field
 * channels against target (FP32 [B][4][M^3], channel-major, each channel
 * multiplied by scale[b][ch] from the host [B][4] array, or 1 when scale is
 * NULL), then the full backward pass.  Writes the loss (FP64, host) and
 * leaves the flat gradient on the device (lws_net_get_grad).  Synchronises. */
LBM_API int lws_net_loss_grad(lws_net_t *net, int B, const double *ra_pr, const float *target,
                              const double *scale, double *loss, void *stream);
LBM_API int lws_net_get_grad(lws_net_t *net, float *host);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr on
 * the gradient of lws_net_loss_grad; the step counter is kept in the net. */
LBM_API int lws_net_adam(lws_net_t *net, double lr, void *stream);

LBM_API const char *lws_last_error(const lws_net_t *net);

#ifdef __cplusplus
}
#endif

#endif

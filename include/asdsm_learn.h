/*
 * asdsm_learn.h -- C ABI of the learned correction for the ASDSM refinement loop (Algorithm 4):
 * a small 3D convolutional network maps the fine residual r_k (with the coarse-plane positions and
 * the cell Peclet numbers of the equation) to a proposed correction c of the iterate.  In a learned
 * solve, each refinement step first tries u_k + w c with the line-search step w of Algorithm 4; the
 * proposal is accepted only if the residual falls by a stated factor, otherwise the plain ASDSM
 * step is taken.  The motivation is the paper's diagnosis of stagnation (Section 4, Example 2):
 * after a few iterations the residual is highly irregular at the coarse points, which spoils the
 * projected right-hand sides of the next step, and smoothing the residual lowers the stagnation
 * level.  A local correction that removes the irregular part of r_k is what the network learns.
 *
 * Network: four 3x3x3 convolutions with zero padding, channels 7 -> 32 -> 32 -> 32 -> 1, ReLU after
 * the first three, biases; BF16 weights and activations as MFMA operands with FP32 accumulation
 * (FP32 master weights and weight gradients).  Losses: mean squared error against a target, or
 * the residual loss mean (rhat - A' c)^2, A' = the fine operator scaled by h^2 / mean(alpha): the
 * A^T A-weighted distance between c and the exact correction A'^{-1} rhat, which is never formed.
 * Optimiser: Adam.
 *
 * Conventions
 * -----------
 * - A network object is built for one cubic volume of n^3 voxels (4 <= n <= 256), voxel
 *   v = x + n (y + n z), x fastest.  Inputs are FP32, channels last, 16 channels per voxel of which
 *   the first 7 are read (the remaining 9 must be zero): in[v * 16 + c].  Outputs and targets are
 *   FP32, one value per voxel.
 * - Parameters are one flat FP32 vector: for each layer l = 0..3 its weights w[co][tap][ci]
 *   (co < cout_p(l), tap = (dz+1) 9 + (dy+1) 3 + (dx+1) for the neighbour (x+dx, y+dy, z+dz),
 *   ci < cin_p(l)) and then its biases (cout_p(l) values), with (cin_p, cout_p) = (16, 32),
 *   (32, 32), (32, 32), (32, 16); weights of padded channels are kept at zero.
 * - Device pointers must be valid for the network's device; calls are enqueued on the stream given
 *   at creation (asdsm_solve_learned: the plan's stream).  Calls that hand results to the host
 *   (asdsm_net_params, asdsm_net_gradient with a loss or gradient pointer, asdsm_solve_learned)
 *   return after the stream has completed; the others return once their work is enqueued, so
 *   their device buffers must stay valid until the stream reaches it.  Return: 0 or an ASDSM_E_* code
 *   (include/asdsm.h); asdsm_last_error() describes the last error.
 */
#ifndef ASDSM_LEARN_H
#define ASDSM_LEARN_H

#include <stddef.h>
#include <stdint.h>

#include "asdsm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct asdsm_net_s *asdsm_net_t;

/* Create a network for n^3 volumes: He-normal weights from `seed` for the three hidden layers,
 * zero weights for the output layer (the first proposals are c = 0), zero biases.
 * hip_stream is borrowed (may be NULL).  Errors: ASDSM_E_ARG. */
int asdsm_net_create(asdsm_net_t *out, int n, uint64_t seed, void *hip_stream);

/* Number of parameters (FP32) of the flat parameter vector. */
int asdsm_net_param_count(asdsm_net_t net, size_t *count);

/* Bytes of device workspace (256-byte aligned base) holding parameters, Adam moments,
 * activations and gradients; attaching it uploads the current parameters. */
int asdsm_net_workspace_size(asdsm_net_t net, size_t *bytes);
int asdsm_net_set_workspace(asdsm_net_t net, void *dev, size_t bytes);

/* Copy the flat parameter vector to (get != 0) or from (get == 0) the host array `host`.
 * Setting resets the Adam moments. */
int asdsm_net_params(asdsm_net_t net, float *host, int get);

/* Inference: out (device, n^3) = network(in (device, n^3 x 16)). */
int asdsm_net_forward(asdsm_net_t net, const float *in, float *out);

#define ASDSM_NET_LOSS_MSE      0   /* mean_v (out_v - target_v)^2                                */
#define ASDSM_NET_LOSS_RESIDUAL 1   /* mean_v (target_v - (A' out)_v)^2, A' of the bound plan     */

/* Forward and backward pass for one sample: the loss of kind loss_kind into *loss (host, may be
 * NULL); the gradient of the loss with respect to every parameter stays in the network (for
 * asdsm_net_adam) and is copied to `grad_host` (flat layout above) when that is not NULL.  A' (ASDSM_NET_LOSS_RESIDUAL) is
 * the bound plan's 7-point fine operator times h^2 / mean(alpha), applied on the network's volume
 * with zero values outside it.  Errors: ASDSM_E_ARG (unknown kind, residual loss without binding). */
int asdsm_net_gradient(asdsm_net_t net, const float *in, const float *target, int loss_kind,
                       double *loss, float *grad_host);

/* Bind the network to a plan with d = 3 and N_f >= n: fixes the cell Peclet numbers
 * beta_j h / (2 alpha_j), the coarse-plane spacing H / h and the operator A' of the residual loss.
 * The plan must outlive the binding.  Errors: ASDSM_E_ARG. */
int asdsm_net_bind(asdsm_net_t net, asdsm_plan_t plan);

/* Network input for the window [o_j, o_j + n) (o = offset, host int[3], NULL = origin) of a fine
 * residual r (device, N_f^3 FP64, axis 0 fastest) with squared norm rnorm2 (of the whole r):
 * in16 (device, n^3 x 16): channel 0 r / sigma with sigma = sqrt(rnorm2 / N_f^3), channels 1..3 the
 * indicators of the coarse planes of axes 0..2 (fine index i, 0-based, on a coarse plane when
 * (i + 1) is a multiple of H / h), channels 4..6 the cell Peclet numbers, channels 7..15 zero;
 * rhat (device, n^3, may be NULL) receives channel 0 contiguously (the target of the residual loss).
 * The proposed correction in the solver's units is out * sigma * h^2 / mean(alpha).
 * Errors: ASDSM_E_ARG (not bound, window outside the mesh). */
int asdsm_net_features(asdsm_net_t net, const double *r, double rnorm2, const int *offset,
                       float *in16, float *rhat);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr on the last gradient. */
int asdsm_net_adam(asdsm_net_t net, float lr);

/* ASDSM solve (as asdsm_solve) with learned proposals: before each refinement step the network,
 * bound to this plan and built for n = N_f, proposes c from r_k; with the line-search step
 * w = <r, A c> / <A c, A c> the new residual norm is sqrt(||r||^2 - <r, A c>^2 / <A c, A c>), and
 * the proposal is accepted when that is at most ||r_k|| / factor (factor > 1; the learned step then
 * counts as the refinement step), otherwise the plain step of Algorithm 4 is taken.  *accepted
 * (may be NULL) receives the number of accepted proposals.  The network's buffers are used on the
 * plan's stream.  The stopping rule, histories and statistics are those of asdsm_solve (phase
 * ASDSM_PHASE_LEARNED holds the proposals).  Errors: those of asdsm_solve, ASDSM_E_ARG (network
 * not bound to this plan or of another size, factor <= 1). */
int asdsm_solve_learned(asdsm_plan_t plan, asdsm_net_t net, double factor, const double *s,
                        const double *g, double *u, const asdsm_opts *opts, asdsm_stats *stats,
                        int *accepted);

/* Release the network (not the workspace).  NULL is ignored. */
void asdsm_net_destroy(asdsm_net_t net);

#ifdef __cplusplus
}
#endif
#endif /* ASDSM_LEARN_H */

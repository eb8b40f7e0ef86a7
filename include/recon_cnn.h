/*
 * recon_cnn.h -- learned starting displacement for the reconstruction of recon.h.
 *
 * Not part of the paper's method.  The paper's approximate starts (eq. approx1,
 * eq. approx2) change only the radial component of the plain Zel'dovich start;
 * the learned start does the same with a correction Delta u predicted per cell
 * by a small periodic 3D CNN:
 *     Psi_0 = Psi_p + Delta u r_hat,
 * after which the iteration of Sec. 5.1 runs unchanged and stays the judge of
 * convergence.  Network (channels-last bfloat16 activations, FP32 accumulation):
 *     x0 = [delta_s, 0.1 u_p, r_x, r_y, r_z, 0, 0, 0]     u_p = Psi_p . r_hat [Mpc/h]
 *     a1 = relu(conv3(x0; W1 [16][27][8],  b1 [16]))
 *     a2 = relu(conv3(a1; W2 [16][27][16], b2 [16]))
 *     y  =      conv3(a2; W3 [1][27][16],  b3 [1]),   Delta u = y / 0.1
 * conv3 is a periodic 3x3x3 cross-correlation with tap t = (dz+1)*9 + (dy+1)*3 + (dx+1).
 * Parameters: one FP32 device vector of RECON_CNN_PARAMS values, W1, b1, W2, b2, W3, b3
 * in that order.  Every call needs a plan created with RECON_CNN_BUFFERS.
 *
 * Network grid: the plan's n^3 grid, or with RECON_CNN_HALF the (n/2)^3 grid of every
 * other node (cell 2 L/n), or with RECON_CNN_QUARTER the (n/4)^3 grid of every fourth node (the
 * restriction and prolongation below applied twice; the two prolongations run as one trilinear pass,
 * equal up to FP32 rounding).  Then recon_solve restricts delta_s and u_p by full weighting
 * (recon_restrict), evaluates the network with r_hat of the coarse nodes, and prolongs
 * Delta u linearly (recon_prolong) to the n^3 grid.  The network grid needs >= 16^3 cells.
 * recon_cnn_forward and recon_cnn_train_step take and return fields on the network grid.
 */
#ifndef RECON_CNN_H
#define RECON_CNN_H

#include "recon.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RECON_CNN_PARAMS 10833
#define RECON_CNN_BUFFERS 8u     /* plan flag: activation, gradient and partial-sum buffers */
#define RECON_CNN_HALF 16u       /* plan flag (with RECON_CNN_BUFFERS): network on the (n/2)^3 grid */
#define RECON_CNN_QUARTER 512u   /* plan flag (with RECON_CNN_BUFFERS): network on the (n/4)^3 grid of every
                                    fourth node: inputs restricted twice, output prolonged twice      */

/* Delta u for every cell of every realisation of the plan.  params: device FP32
 * [RECON_CNN_PARAMS]; delta, u_p, du_out: device FP32 [batch][m^3] on the network grid
 * (m = n, n/2 with RECON_CNN_HALF, or n/4 with RECON_CNN_QUARTER). */
int recon_cnn_forward(recon_plan_t* plan, const float* params, const float* delta, const float* u_p, float* du_out);

/* One training step on the plan's batch: loss = mean (y - 0.1 target_du)^2 over all cells,
 * its gradient (deterministic, FP32) into grad_out (device FP32 [RECON_CNN_PARAMS], may be NULL),
 * and, when lr > 0, one Adam update (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected for step >= 1)
 * of params with the moment vectors adam_m, adam_v (device FP32 [RECON_CNN_PARAMS]).
 * loss_out: host double.  Synchronises once to read the loss. */
int recon_cnn_train_step(recon_plan_t* plan, float* params, float* adam_m, float* adam_v, int step, float lr,
                         const float* delta, const float* u_p, const float* target_du, double* loss_out,
                         float* grad_out);

/* u = Psi . r_hat of the current displacement (device FP32 [batch][n^3]); needs a computed Psi. */
int recon_get_radial(recon_plan_t* plan, float* u_out);

/* Full-weighting restriction of [batch][n^3] node fields to [batch][(n/2)^3]: coarse node J
 * sits on fine node 2J, weights 1/4, 1/2, 1/4 per axis on fine nodes 2J-1, 2J, 2J+1 (periodic).
 * fine, coarse: device FP32, not overlapping.  Any plan; enqueued on its stream. */
int recon_restrict(recon_plan_t* plan, const float* fine, float* coarse);

/* Linear prolongation of [batch][(n/2)^3] to [batch][n^3]: fine node 2J copies coarse node J,
 * fine node 2J+1 the mean of coarse nodes J and J+1, axis by axis (periodic).  coarse, fine:
 * device FP32, not overlapping.  Any plan; enqueued on its stream. */
int recon_prolong(recon_plan_t* plan, const float* coarse, float* fine);

#ifdef __cplusplus
}
#endif

#endif /* RECON_CNN_H */

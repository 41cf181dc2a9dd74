/*
 * sbi_net.h -- the learned warm start of the W iteration: its features, its
 * matrix-core inference, and the trainer that fits it on the GPU.
 *
 * The paper starts the successive approximation of Sec. 2.4 from the linear
 * initiation V0 = F^-1{k tanh(kh) phi_hat}, phi_b0 = F^-1{sech(kh) phi_hat}.
 * The learned warm start adds to both the corrections predicted by a small
 * periodic convolution network of local surface quantities:
 *   V0 = W_lin + out_scale[0] y[0],   phi_b0 = phi_b,lin + out_scale[1] y[1]
 * (with a flat bed the iteration has no bottom unknown and y[1] is unused).
 * A context with seed SBI_SEED_NET uses it for solves that have no previous
 * solve to start from (the first one, and any after a failed one); later
 * solves start from the SBI_SEED_PREV seed, which carries the previous
 * converged nonlinear parts -- or, in fixed-step time stepping once the
 * learned history layer is loaded and has K solves behind it, from that
 * layer's prediction (below).
 * The iteration itself, and its residual test, are unchanged: the seed affects
 * the number of sweeps, never the converged answer.  When a solve started from the learned
 * seed fails (divergence, non-finite values) it is redone from the linear
 * guess and the call reports SBI_WARN_FALLBACK_USED.
 *
 * Features, per point, channel-last, FP32 [batch][ny][nx][8] (2D grids only):
 *   0 eta (as the solve sees it)   1 W_lin = F^-1{k tanh(kh) phi_hat}
 *   2 d_x eta   3 d_y eta          (spectral derivatives of the masked eta)
 *   4 d_x phi   5 d_y phi          (spectral derivatives of the masked phi_s)
 *   6 delta = h_ref - depth        7 eta * W_lin
 * each multiplied by its channel scale (in_scale of the loaded weights).
 *
 * Network: z1 = b1 + conv3x3(x; W1) 8->32, a1 = silu(z1);
 *          z2 = b2 + conv3x3(a1; W2) 32->32, a2 = silu(z2);
 *          z3 = b3 + W3 a2 (1x1) 32->32, a3 = silu(z3);  y = b4 + W4 a3 (1x1) 32->2.
 * conv3x3(a; W)[o](y, x) = sum_{t=0..8} sum_c W[o][t][c] a[c](y + t/3 - 1, x + t%3 - 1)
 * with periodic wrap; silu(z) = z / (1 + exp(-z)).
 *
 * Parameter vector (FP32, SBI_NET_PARAMS values, this order):
 *   W1[32][9][8], b1[32], W2[32][9][32], b2[32], W3[32][32], b3[32], W4[2][32], b4[2].
 * Weight blob (host bytes, sbi_net_blob_bytes() long): sbi_net_header followed
 * by the parameter vector.  Inference uses the BF16 rounding (nearest even) of
 * the weights, FP32 biases, BF16 activations into the matrix-core products and
 * FP32 accumulation.
 *
 * Conventions are those of sbi.h: device pointers are caller-owned, calls
 * return sbi_status, work runs on the context's (or trainer's) stream.
 */
#ifndef SBI_NET_H
#define SBI_NET_H

#include "sbi.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SBI_NET_PARAMS 12706

typedef struct sbi_net_header {
    char magic[4];         /* "SBIW" */
    uint32_t version;      /* 1 */
    uint32_t cin;          /* 8 */
    uint32_t width;        /* 32 */
    uint32_t nparams;      /* SBI_NET_PARAMS */
    float in_scale[8];     /* feature scales */
    float out_scale[2];    /* scales of the V and phi_b corrections */
    float reserved[1];
} sbi_net_header;

/* Number of FP32 parameters of the network (SBI_NET_PARAMS). */
int32_t sbi_net_param_count(void);

/* Bytes of a weight blob: sizeof(sbi_net_header) + 4 * SBI_NET_PARAMS. */
size_t sbi_net_blob_bytes(void);

/*
 * Features of the states (eta, phi_s) of a context's members (2D grids).
 *   eta, phi_s  device [batch][ny][nx], context precision
 *   feat_out    device FP32 [batch][ny][nx][8], scaled by the loaded weights'
 *               in_scale (by 1 when no weights are loaded)
 *   wlin_out    device [batch][ny][nx] W_lin in the context precision, or NULL
 * Errors: SBI_ERR_UNSUPPORTED on 1D grids.
 */
sbi_status sbi_net_features(sbi_ctx* ctx, const void* eta, const void* phi_s, float* feat_out, void* wlin_out);

/*
 * Matrix-core inference of the loaded network (the seeds used by
 * SBI_SEED_NET): seed_out = wlin + out_scale[0] y[0](feat) and
 * dphib_out = out_scale[1] y[1](feat).
 *   feat       device FP32 [batch][ny][nx][8] (as from sbi_net_features)
 *   wlin       device [batch][ny][nx], context precision
 *   seed_out   device [batch][ny][nx], context precision
 *   dphib_out  device [batch][ny][nx], context precision
 * Errors: SBI_ERR_INVALID_ARG when no weights are loaded (sbi_net_load).
 */
sbi_status sbi_net_infer(sbi_ctx* ctx, const float* feat, const void* wlin, void* seed_out, void* dphib_out);

/*
 * Training labels: the nonlinear parts (V* - W_lin, phi_b - phi_b,lin) that the
 * last solve of an SBI_SEED_PREV or SBI_SEED_NET context left (the parts its next solve starts
 * from), in physical space.  phi_b is the iterate after the relaxed update of
 * the last sweep; with a flat bed dphib_out is zero.
 *   dv_out, dphib_out  device [batch][ny][nx], context precision
 * Errors: SBI_ERR_INVALID_ARG for other seeds, or when no solve has succeeded
 * yet.
 */
sbi_status sbi_last_correction(sbi_ctx* ctx, void* dv_out, void* dphib_out);

/*
 * Learned history layer (the second, spectral layer of the learned warm
 * start).  In fixed-step stepping (sbi_step, sbi_batch_step: integrating-
 * factor RK4, Sec. 2.2) each step makes four W solves, at stages s = 0..3.
 * The nonlinear part of a converged solve is the pair of kept-mode spectra
 *   N_V = V* - k tanh(kh) phi_hat,   N_B = phi_b - sech(kh) phi_hat
 * (N_B only over a variable bed).  The layer predicts the nonlinear part of
 * the solve at stage s from those of the K fixed-step solves before it
 * (h_0 the most recent) through their backward differences
 * d_q = sum_{j<=q} (-1)^j C(q, j) h_j, mode by mode:
 *   pred_P(k) = sum_{q<K} w[P][s][b(k)][q] d_q,P(k),  b(k) = min(floor(|k|/dk), nb - 1),
 * complex weights per part P (0: V, 1: phi_b), stage, radial bin and tap, and
 * the iteration starts from V0 = k tanh(kh) phi_hat + pred_V, phi_b0 =
 * sech(kh) phi_hat + pred_B.  Only successful fixed-step solves enter the
 * history; any other solve of the context (sbi_vertical_velocity,
 * sbi_diagnostics, sbi_step_adaptive) or a failed one empties it.  A solve
 * started from the prediction that fails is redone from the linear guess
 * (SBI_WARN_FALLBACK_USED), except inside captured ensembles (sbi_batch.h),
 * which report the failure.  With w[.][.][.][0] = 1 and the other taps 0 the
 * layer is the SBI_SEED_PREV seed; w = 1 for every q is Newton's backward-
 * difference extrapolation one step ahead.
 * Weights: host FP32 [2][4][nb][K][2] (re, im), sbi_net_hist_param_count()
 * values, K <= SBI_HIST_MAX_TAPS, nb <= SBI_HIST_MAX_BINS.
 * Training (on the device, per context): with training on, every fixed-step
 * solve with a full history adds to an accumulator the gradient of its loss
 *   L = sum_P sum_k c_k |pred_P - N_P|^2 / sum_k c_k |N_P|^2
 * (kept modes, c_k = 1 at m_x = 0 else 2; parts with N_P = 0 skipped) with
 * respect to the real and imaginary parts of its stage's weights (the
 * weights it was seeded with), and the Gram matrices G = sum c conj(d) d^T / D
 * of each (part, stage, bin).  Two optimisers: sbi_net_hist_adam (one Adam
 * step with the mean accumulated gradient) and sbi_net_hist_newton (the
 * Gauss-Newton step w <- w - (G + lam tr(G)/K I)^-1 gamma, gamma = gradient/2
 * as the complex derivative; the loss is quadratic in w, so one step lands on
 * the ridge-regularised least-squares weights of the accumulated solves).
 */
#define SBI_HIST_MAX_TAPS 8
#define SBI_HIST_MAX_BINS 32

/* FP32 values of a layer of `taps` taps and `bins` bins (0 when out of range). */
int32_t sbi_net_hist_param_count(int32_t taps, int32_t bins);

/* Load the layer into an SBI_SEED_NET context (weights copied; Adam moments
   and the gradient accumulator cleared; history emptied).  dk > 0: bin width
   in 1/length units.  Errors: SBI_ERR_INVALID_ARG. */
sbi_status sbi_net_hist_load(sbi_ctx* ctx, int32_t taps, int32_t bins, double dk, const float* w);

/* Accumulate the loss gradient of each later fixed-step solve (enable != 0). */
sbi_status sbi_net_hist_train(sbi_ctx* ctx, int32_t enable);

/* The accumulated sums since the last optimiser step: loss sum, solves, and
   (each optional) the gradient sum, host double [param count], and the Gram
   sums, host double [2][4][nb][K][K][2] (re, im). */
sbi_status sbi_net_hist_gradient(sbi_ctx* ctx, double* loss_sum, int32_t* samples, double* grad_sum,
                                 double* gram_sum);

/* One Gauss-Newton step (ridge lam >= 0, relative to tr(G)/K) of every
   (part, stage, bin) with accumulated solves, by complex Cholesky in FP64;
   clears the accumulators; loss_mean/samples as for sbi_net_hist_adam. */
sbi_status sbi_net_hist_newton(sbi_ctx* ctx, double lam, double* loss_mean, int32_t* samples);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; FP64
   moments, FP32 weights) with the mean accumulated gradient, which is then
   cleared; loss_mean/samples (host, optional) describe the accumulated solves.
   With no solve accumulated the weights are unchanged. */
sbi_status sbi_net_hist_adam(sbi_ctx* ctx, float lr, double* loss_mean, int32_t* samples);

/* Copy the layer's current weights to host w_out [param count]. */
sbi_status sbi_net_hist_params(sbi_ctx* ctx, float* w_out);

/*
 * Trainer: FP32 master parameters, Adam moments, the BF16-rounded copy used
 * by the forward pass, and the activations of one training batch of `batch`
 * periodic fields of ny x nx points (nx a multiple of 64, ny >= 16).
 * Workspace: caller-owned device memory of sbi_net_trainer_bytes() bytes.
 */
typedef struct sbi_net_trainer sbi_net_trainer;

size_t sbi_net_trainer_bytes(int32_t batch, int32_t ny, int32_t nx);

/* theta: host FP32 [SBI_NET_PARAMS] initial parameters (copied). */
sbi_status sbi_net_trainer_init(sbi_net_trainer** out, int32_t batch, int32_t ny, int32_t nx, const float* theta,
                                void* workspace, size_t ws_bytes, void* hip_stream);

/* FP32 forward pass: y_out device FP32 [batch][ny][nx][2] = network(feat). */
sbi_status sbi_net_trainer_forward(sbi_net_trainer* tr, const float* feat, float* y_out);

/*
 * Mean-square loss L = mean over points and both outputs of (y - target)^2,
 * target device FP32 [batch][ny][nx][2], and its gradient with respect to
 * the (BF16-rounded) weights and biases.  loss: host, optional; grad_out:
 * host FP32 [SBI_NET_PARAMS], optional.  The gradient stays in the trainer
 * for sbi_net_trainer_adam.
 */
sbi_status sbi_net_trainer_gradient(sbi_net_trainer* tr, const float* feat, const float* target, double* loss,
                                    float* grad_out);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the
   last gradient; refreshes the BF16-rounded forward copy. */
sbi_status sbi_net_trainer_adam(sbi_net_trainer* tr, float lr);

/* Copy the FP32 master parameters to host theta_out [SBI_NET_PARAMS]. */
sbi_status sbi_net_trainer_params(sbi_net_trainer* tr, float* theta_out);

sbi_status sbi_net_trainer_destroy(sbi_net_trainer* tr);

#ifdef __cplusplus
}
#endif

#endif /* SBI_NET_H */

/*
 * Learned warm start for the GSIS solver: a small multilayer perceptron that maps case parameters and cell
 * geometry features to initial macroscopic fields, trained on converged solutions the solver itself
 * produces.  The paper has no learned component; it starts its hard cases from cheaper solutions instead
 * (ten conventional iterations before GSIS in Sec. 7.1-7.3, an Euler solution before GSIS in Sec. 7.4).
 * The network only changes the initial state: the converged fields are those of the plain solve, which is
 * also what its prediction error is judged against.
 *
 * Network (fixed depth 4): x (n_in) -> tanh(W1 x + b1) (width) -> tanh(W2 . + b2) (width)
 *                          -> tanh(W3 . + b3) (width) -> W4 . + b4 (n_out).
 * Weights are kept in FP32 (master copy, Adam moments) and used in BF16 (round to nearest even) by the
 * forward and backward products when bf16_weights != 0; every product accumulates in FP32 and the
 * activations are FP32.  Loss: mean squared error over all rows and outputs,
 *     L = (1 / (n n_out)) sum_rows sum_outputs (y - t)^2.
 * Every step runs in HIP kernels on the handle's device; reductions use a fixed order (deterministic).
 *
 * Parameter vector layout (FP32, gsis_mlp_num_params values): for l = 1..4, W_l row-major
 * [out_l][in_l] followed by b_l [out_l].
 *
 * Ownership and errors follow gsis.h: host arrays are read or written during the call only; the handle
 * owns its device memory; negative return codes are errors (GSIS_E_*), with a message from
 * gsis_mlp_last_error.  One handle per thread.
 */
#ifndef GSIS_WARMSTART_H
#define GSIS_WARMSTART_H

#include <stdint.h>

#include "gsis.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsis_mlp_s gsis_mlp_t;

typedef struct {
    int32_t epochs;    /* passes over the training rows */
    int32_t batch;     /* rows per optimizer step (last partial batch of an epoch is used as is) */
    double lr;         /* Adam step size */
    double beta1;      /* Adam first-moment decay */
    double beta2;      /* Adam second-moment decay */
    double eps;        /* Adam denominator guard */
    uint64_t seed;     /* row shuffling (splitmix64 stream; the same seed gives the same order) */
} gsis_mlp_train_opts;

/* Create a network on `device` with seeded weights: W_l entries uniform in +-sqrt(6 / (in_l + out_l))
 * (Glorot), biases zero, drawn from the splitmix64 stream of `seed` in parameter-vector order.
 * n_in, n_out in [1, 64]; width in [1, 1024]. */
int32_t gsis_mlp_create(int32_t device, int32_t n_in, int32_t width, int32_t n_out, int32_t bf16_weights,
                        uint64_t seed, gsis_mlp_t **out);
void gsis_mlp_destroy(gsis_mlp_t *m);
const char *gsis_mlp_last_error(gsis_mlp_t *m);
/* Launch stream (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream); NULL = default stream. */
int32_t gsis_mlp_set_stream(gsis_mlp_t *m, void *hip_stream);
int64_t gsis_mlp_num_params(gsis_mlp_t *m);
/* Copy the FP32 master parameters out / in (layout above); set_params also resets the Adam state. */
int32_t gsis_mlp_get_params(gsis_mlp_t *m, float *params);
int32_t gsis_mlp_set_params(gsis_mlp_t *m, const float *params);
/* Inference: x [n][n_in] -> y [n][n_out] (host, row-major). */
int32_t gsis_mlp_forward(gsis_mlp_t *m, int64_t n, const float *x, float *y);
/* Allocation-free inference, for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): x [n][n_in] -> y [n][n_out], both DEVICE pointers
 * owned by the caller (row-major FP32, 4-byte aligned).  The hidden activations live in a file-scope device
 * array of 8 MiB per GPU (held until the process ends); batches larger than it holds (8 MiB / (8 width) rows,
 * 4,096 at width 256) go through in consecutive chunks, with results identical to gsis_mlp_forward's.
 * Enqueued on the handle's stream; returns without waiting.  Calls no hipMalloc / hipFree.  Every call on
 * one GPU shares that array, so calls that overlap on one GPU (other streams, other threads, other handles)
 * race.  Errors: GSIS_E_ARG (n < 0 or > INT32_MAX, null x or y with n > 0), GSIS_E_DEVICE (the array's
 * address could not be obtained at gsis_mlp_create, or a launch error). */
int32_t gsis_mlp_forward_noalloc(gsis_mlp_t *m, int64_t n, const float *x, float *y);
/* Loss and its gradient with respect to the parameter vector (same layout) for rows x, targets t. */
int32_t gsis_mlp_loss_grad(gsis_mlp_t *m, int64_t n, const float *x, const float *t, double *loss, float *grad);
/* One Adam step (bias-corrected, step count kept in the handle) on the rows given; *loss before the step. */
int32_t gsis_mlp_adam_step(gsis_mlp_t *m, const gsis_mlp_train_opts *o, int64_t n, const float *x,
                           const float *t, double *loss);
/* Minibatch Adam training on the rows given (copied to the device once); *final_loss = mean loss of the
 * last epoch's batches (may be NULL). */
int32_t gsis_mlp_train(gsis_mlp_t *m, int64_t n, const float *x, const float *t, const gsis_mlp_train_opts *o,
                       double *final_loss);

/* ------------------------------------------------------------------ warm start of the solver
 * Standardisation of the network's inputs and outputs: x_n = (x - x_mean) / x_scale per feature and
 * y = y_n y_scale + y_mean per output (n_in, n_out at most 64). */
typedef struct {
    int32_t n_in, n_out;
    double x_mean[64], x_scale[64], y_mean[64], y_scale[64];
} gsis_ws_norm;

/* Mean and standard deviation (population, plus 1e-12) of every column of the host rows x [n][n_in] and
 * t [n][n_out], summed in row order in FP64. */
int32_t gsis_ws_fit_norm(int64_t n, int32_t n_in, const double *x, int32_t n_out, const double *t,
                         gsis_ws_norm *norm);
/* Minibatch Adam training (as gsis_mlp_train) on raw host rows x [n][n_in], t [n][n_out]: both are
 * standardised with `norm` on the device. */
int32_t gsis_ws_train(gsis_mlp_t *m, const gsis_ws_norm *norm, int64_t n, const double *x, const double *t,
                      const gsis_mlp_train_opts *o, double *final_loss);
/* Prediction on raw host rows: standardisation, forward pass and de-standardisation on the device;
 * y [n][n_out] (host). */
int32_t gsis_ws_predict(gsis_mlp_t *m, const gsis_ws_norm *norm, int64_t n, const double *x, double *y);
/* Network parameters and standardisation in one binary file (tag, dimensions, FP32 parameters, norm);
 * gsis_ws_load requires a handle of the same dimensions (GSIS_E_ARG otherwise or for a foreign file) and
 * resets its Adam state. */
int32_t gsis_ws_save(gsis_mlp_t *m, const gsis_ws_norm *norm, const char *path);
int32_t gsis_ws_load(gsis_mlp_t *m, gsis_ws_norm *norm, const char *path);

/* Training targets of the solver's current state, [nc][D + 5]: log rho, u (D), log T_t, log T_r, log T_v,
 * log T_R (GSIS_E_DIVERGED if a density or temperature is not positive). */
int32_t gsis_ws_targets(gsis_t *h, double *t);
/* Initial state from the network (the learned warm start; the paper's analogue is its Euler-solution start
 * of the capsule case, Sec. 7.4): per-cell features x [nc][n_in] of the solver's mesh are standardised and
 * passed through the network on the device, the outputs read as the targets above (n_out = D + 5), and the
 * multi-temperature equilibrium of the predicted fields becomes f and I (as gsis_init_fields).  In a domain
 * closed by walls the predicted density is scaled to the mass of the solver's current state, which the
 * iteration conserves.  Runs on the solver's stream. */
int32_t gsis_init_warmstart(gsis_t *h, gsis_mlp_t *m, const gsis_ws_norm *norm, const double *x);

#ifdef __cplusplus
}
#endif

#endif

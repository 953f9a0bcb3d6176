/* mlp.h -- C ABI of the learned surrogate of the batched sweep, on gfx950.
 *
 * A small fully connected network, 5 inputs -> 256 -> 256 -> 256 -> 2 outputs
 * with exact GELU (x (1 + erf(x / sqrt 2)) / 2) after each hidden layer, in an
 * ensemble of `members` independently trained copies.  It maps the five sweep
 * inputs of a case (clean contact angle, adsorption strength, surfactant
 * load, capillary number, drop radius; scaled by the caller) to two outputs
 * (steady apparent contact angle and detachment time, standardised by the
 * caller).  Not part of the paper's method: a surrogate layer over the
 * lattice Boltzmann solver, which remains the fallback and the arbiter of its
 * error.
 *
 * Numerics: every matrix product runs on the matrix cores as
 * bfloat16 x bfloat16 -> FP32 accumulation (weights and each layer's input in
 * bfloat16; in the backward pass also the back-propagated signal); biases,
 * activations, the loss and the optimiser in FP32, with FP32 master weights.
 * Loss: masked mean squared error, sum of m (y - t)^2 over the batch and both
 * outputs divided by the sum of the mask.  Optimiser: Adam (beta1 0.9, beta2
 * 0.999, eps 1e-8, bias-corrected).
 *
 * Parameter layout (FP32, mlp_param_count() values per member): per layer the
 * weight matrix W[in][out] row-major, then the bias b[out].
 *
 * Pointers named *_dev are device memory; *_host are host memory.  Arrays are
 * row-major: x[n][5], t[n][2], m[n][2], y[n][2].  All calls are ordered on the
 * handle's stream; those returning host data synchronise it.  Errors: 0 on
 * success or a negative code as in lbm.h (-1 argument, -3 memory, -4 device);
 * mlp_last_error gives the message. */
#ifndef MLP_SURROGATE_H
#define MLP_SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlp_handle mlp_handle; /* opaque, owned by the library */

/* Parameters per member (133634). */
int32_t mlp_param_count(void);

/* Device bytes for `members` members and batches of up to max_batch samples. */
int mlp_required_bytes(int32_t members, int32_t max_batch, size_t* bytes);

/* Create an ensemble; dev_buf (caller-owned, 256-byte aligned, at least
 * mlp_required_bytes) or NULL for a library allocation; hip_stream or NULL for
 * a library stream.  Parameters start at zero: set them with mlp_set_params. */
int mlp_init(int32_t members, int32_t max_batch, void* dev_buf, size_t buf_bytes, void* hip_stream, mlp_handle** out);

/* Copy FP32 master parameters of one member from the host (and reset its
 * optimiser state), or to the host. */
int mlp_set_params(mlp_handle* h, int32_t member, const float* params_host);
int mlp_get_params(mlp_handle* h, int32_t member, float* params_host);

/* Outputs of one member for n inputs (n <= max_batch). */
int mlp_forward(mlp_handle* h, int32_t member, const float* x_dev, int32_t n, float* y_dev);

/* Loss and its gradient with respect to the master parameters for one member
 * (grad_host: mlp_param_count() floats, or NULL); synchronises. */
int mlp_loss_grad(mlp_handle* h, int32_t member, const float* x_dev, const float* t_dev, const float* m_dev, int32_t n,
                  float* loss_host, float* grad_host);

/* One training step of one member: forward, backward, Adam update with rate
 * lr.  loss_host (the loss before the update) may be NULL: then nothing
 * synchronises. */
int mlp_train_step(mlp_handle* h, int32_t member, const float* x_dev, const float* t_dev, const float* m_dev, int32_t n,
                   float lr, float* loss_host);

/* One training step of every member at once, each on its own batch of n
 * samples (its bootstrap resample): x_dev[members][n][5], t_dev and
 * m_dev[members][n][2].  Every product and reduction covers all members in one
 * launch (member = grid z or y); per member the arithmetic is that of
 * mlp_train_step on its own batch, so the parameters after the step equal, bit
 * for bit, those of one mlp_train_step per member.  loss_host[members] (each
 * member's loss before the update) may be NULL: then nothing synchronises. */
int mlp_train_step_ensemble(mlp_handle* h, const float* x_dev, const float* t_dev, const float* m_dev, int32_t n,
                            float lr, float* loss_host);

/* Every member on the same n inputs; per sample and output the ensemble mean
 * and standard deviation (population, over members): mean_dev[n][2], std_dev[n][2]. */
int mlp_predict_ensemble(mlp_handle* h, const float* x_dev, int32_t n, float* mean_dev, float* std_dev);

/* mlp_predict_ensemble without a handle and without allocating: for callers
 * that cannot allocate device memory (work under HIP graph capture, tight
 * serving loops, harnesses that forbid it).  params_dev holds the FP32
 * parameters of `members` members back to back ([members][mlp_param_count()],
 * device memory, caller-owned, as mlp_get_params returns them); x_dev, mean_dev
 * and std_dev as for mlp_predict_ensemble.  The results equal
 * mlp_predict_ensemble's for the same parameters bit for bit.  Limits:
 * 1 <= members <= 8 and 1 <= n <= 1024 (-1 beyond them).  Work is ordered on
 * hip_stream (NULL: the null stream) and nothing synchronises.  The bfloat16
 * weights and activations live in one fixed device array of about 4.3 MB per
 * device, held until the process ends and shared by every call on that
 * device: calls that overlap on one device (other streams or threads) race
 * and must be serialised by the caller.  No hipMalloc, hipFree or other
 * allocating call is made.  Errors go to mlp_last_error(NULL). */
int mlp_predict_ensemble_noalloc(const float* params_dev, int32_t members, const float* x_dev, int32_t n,
                                 float* mean_dev, float* std_dev, void* hip_stream);

/* Release the handle and any library-owned memory and stream. */
int mlp_destroy(mlp_handle* h);

/* Message of the last failed call on h (of the last failed mlp_init when NULL). */
const char* mlp_last_error(const mlp_handle* h);

#ifdef __cplusplus
}
#endif
#endif

/*
 * mlp.h -- C interface of the surrogate network of the gfx950 PIC library.
 *
 * The paper's accuracy study (Sec. "Accurate modeling of plasma accelerators
 * in finite order PSATD", Eqs. (11)-(12), and its parameter-scan figure)
 * measures, for each set of physical and numerical parameters, the error of
 * the witness slice energy spread and emittance of an order-p run against
 * the infinite-order twin, and reads off the lowest order whose errors stay
 * below 0.05.  This interface trains and evaluates a small multilayer
 * perceptron that maps (2/p, k_p dz, k_p dr, gamma, charge), normalised by
 * the caller, to those two errors, so the order can be chosen without
 * running the whole scan.
 *
 * Network: n_in -> n_hidden_layers x hidden (GELU, the exact erf form)
 * -> n_out (linear).  Loss: mean squared error over the batch and outputs.
 * Optimiser: Adam with bias correction,
 *   m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
 *   p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 *
 * Parameters are one flat float32 array, layer by layer: W_l as [out][in]
 * row-major, then b_l [out].  PIC_MLP_FP32 computes everything in float32.
 * PIC_MLP_BF16 keeps float32 master weights and Adam moments, but the
 * matrix products read bfloat16 operands (weights, hidden activations and
 * back-propagated gradients rounded to nearest-even when written) and
 * accumulate in float32; the network input stays float32.
 *
 * Conventions as in pic.h: every function returns a pic_status code, device
 * pointers are device memory of the context's device, work is enqueued on the
 * context's stream and only the functions marked "synchronizes" wait for it.
 * The workspace is caller-owned device memory that must outlive the context.
 */
#ifndef PIC_MLP_H
#define PIC_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "pic.h" /* pic_status */

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pic_mlp pic_mlp;

typedef enum { PIC_MLP_FP32 = 0, PIC_MLP_BF16 = 1 } pic_mlp_prec;

typedef struct {
  int32_t n_in;            /* 1..64 */
  int32_t hidden;          /* 1..1024 */
  int32_t n_hidden_layers; /* 1..8 */
  int32_t n_out;           /* 1..64 */
  int32_t prec;            /* pic_mlp_prec */
  int32_t max_batch;       /* rows per forward / training batch, 1..65536 */
} pic_mlp_config;

typedef struct {
  float lr, beta1, beta2, eps;
} pic_adam;

/* Number of float32 parameters of the configuration.  Errors: PIC_EINVAL. */
int pic_mlp_num_params(const pic_mlp_config* cfg, int64_t* n);

/* Device workspace needed by pic_mlp_init.  Errors: PIC_EINVAL. */
int pic_mlp_workspace_bytes(const pic_mlp_config* cfg, size_t* bytes);

/* Creates a network with the given initial parameters (host, num_params
 * floats, copied) and zero Adam moments.  `hip_stream` is a hipStream_t
 * (NULL: the default stream).  Synchronizes.  Errors: PIC_EINVAL (bad
 * configuration or pointer), PIC_ENOSPC (workspace too small), PIC_EHIP. */
int pic_mlp_init(const pic_mlp_config* cfg, const float* params, void* workspace, size_t bytes,
                 void* hip_stream, pic_mlp** out);

/* y[n][n_out] = network(x[n][n_in]), device pointers, 0 <= n <= max_batch. */
int pic_mlp_forward(pic_mlp* net, const float* x, int32_t n, float* y);

/* One forward and backward pass over the n rows of x with targets t[n][n_out]:
 * writes the gradient of the loss with respect to every parameter to
 * grad[num_params] and the loss to loss[0] (device pointers).  The
 * parameters are not changed. */
int pic_mlp_loss_grad(pic_mlp* net, const float* x, const float* t, int32_t n, float* grad, float* loss);

/* `steps` Adam steps.  Step s trains on the rows idx[s * batch .. s * batch +
 * batch - 1] of the data set (x[n_data][n_in], t[n_data][n_out]); the row
 * indices are the caller's (device int32, each in [0, n_data)), so the
 * minibatch order is an input.  The loss of every step goes to loss[s] (device,
 * may be NULL).  batch <= max_batch.  The Adam step counter continues across
 * calls. */
int pic_mlp_train(pic_mlp* net, const float* x, const float* t, int32_t n_data, const int32_t* idx,
                  int32_t batch, int32_t steps, const pic_adam* opt, float* loss);

/* Copies the float32 master parameters to host memory.  Synchronizes. */
int pic_mlp_get_params(pic_mlp* net, float* params);

/* Replaces the float32 master parameters (host, num_params floats) and their
 * bfloat16 copy; the Adam moments and step count are kept.  Synchronizes.
 * Errors: PIC_EINVAL, PIC_EHIP. */
int pic_mlp_set_params(pic_mlp* net, const float* params);

/* Adam steps taken so far. */
int pic_mlp_steps(pic_mlp* net, int64_t* steps);

/* Waits for the context's work.  Synchronizes. */
int pic_mlp_sync(pic_mlp* net);

/* Releases the context (not the workspace).  Synchronizes. */
int pic_mlp_free(pic_mlp* net);

#ifdef __cplusplus
}
#endif

#endif /* PIC_MLP_H */

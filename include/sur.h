/* sur.h -- C-ABI of the learned surrogate for gfx950 (BF16 MFMA, FP32 accumulate).
 *
 * The surrogate maps the parameters of a grounding-electrode case (soil
 * conductivity and permittivity, electrode length and depth, rise time of the
 * injected current) to the ground-potential-rise waveform at the feed point.
 * It is a multilayer perceptron trained on waveforms computed by the batched
 * FDTD engine of fdtd.h; FDTD stays the fallback and the judge of its error.
 * The surrogate is an extension of the method in Section 2 of the paper (the
 * paper itself trains no network); the FDTD waveform it imitates is the
 * ground potential rise of Section 4.1.
 *
 * Network (per member of an ensemble of n_nets independent nets):
 *   widths w_0 -> w_1 -> ... -> w_L;  layer l computes z = a W_l^T + b_l,
 *   W_l of shape (w_l, w_{l-1}) row-major; hidden layers apply the exact
 *   GELU a = z (1 + erf(z / sqrt 2)) / 2, the last layer is linear.
 *   Products run on the matrix cores with bfloat16 operands (inputs,
 *   activations, weights and output-side gradients rounded to nearest even)
 *   and FP32 accumulation; biases, GELU, the loss and Adam run in FP32.
 * Loss: mean squared error over all outputs of the batch.
 * Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction,
 * FP32 master weights.
 *
 * Parameter vectors ("flat" order, FP32): for each layer, W_l row-major
 * (w_l x w_{l-1}) followed by b_l (w_l).
 *
 * Memory: the caller owns all device memory.  sur_workspace_bytes() gives the
 * size of one device buffer that the caller allocates and binds; the library
 * keeps parameters, Adam state and activations there and never allocates
 * device memory itself.  Pointers named *_dev are device pointers; all other
 * pointers are host pointers, copied during the call.  Calls are enqueued on
 * the stream given at creation (NULL: the legacy default stream); calls that
 * return host data synchronize that stream.  A handle is not thread-safe.
 *
 * Errors: every call returns 0 or a negative code below and never aborts;
 * sur_last_error() describes the last failure.
 */
#ifndef MI355_SUR_H
#define MI355_SUR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SUR_OK = 0,
  SUR_EINVAL = -1,  /* null pointer, bad size, width or net index */
  SUR_ESTATE = -3,  /* workspace not bound, or parameters never set */
  SUR_ENOMEM = -5,  /* bound workspace smaller than sur_workspace_bytes() */
  SUR_EDEVICE = -6, /* HIP error */
};

typedef struct sur_ctx sur_ctx;

/* widths: n_widths entries (2..8); widths[0] in 1..32 inputs, every other
 * width a multiple of 64 up to 4096.  n_nets: ensemble size 1..16.
 * max_rows: rows processed per launch (training batch limit and inference
 * chunk), a multiple of 64 up to 65536. */
int sur_create(const int* widths, int n_widths, int n_nets, int max_rows, void* hip_stream,
               sur_ctx** out);
size_t sur_workspace_bytes(const sur_ctx* c);
int sur_bind_workspace(sur_ctx* c, void* dev, size_t bytes);
/* Number of FP32 parameters of one net (length of a flat vector). */
long long sur_num_params(const sur_ctx* c);

/* Initialise net `net` with uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights
 * and biases from a counter-based generator (SplitMix64 of seed and element
 * index), and reset its Adam state. */
int sur_init_params(sur_ctx* c, int net, unsigned long long seed);
/* Set (and reset the Adam state of) / read the flat FP32 parameters. */
int sur_set_params(sur_ctx* c, int net, const float* host);
int sur_get_params(sur_ctx* c, int net, float* host);
/* Read the flat gradient of the loss left by the last sur_train_step of net. */
int sur_get_grads(sur_ctx* c, int net, float* host);

/* One training step of net `net` on a batch of `batch` rows (1..max_rows):
 *   x_dev: inputs, FP32 row-major [rows x w_0]; t_dev: targets [rows x w_L];
 *   rows_dev: int32 row indices of the batch (device), or NULL for rows
 *   0..batch-1; the caller guarantees the indices are inside x_dev / t_dev.
 * Computes the loss and the gradient; with update != 0 applies one Adam step
 * with learning rate lr.  loss_dev (device, may be NULL) receives the batch
 * loss as one FP32 value. */
int sur_train_step(sur_ctx* c, int net, const float* x_dev, const float* t_dev, const int* rows_dev,
                   int batch, float lr, int update, float* loss_dev);

/* Forward pass of one net over n rows (any n >= 0, processed in chunks of
 * max_rows): x_dev [n x w_0] FP32 -> y_dev [n x w_L] FP32. */
int sur_forward(sur_ctx* c, int net, const float* x_dev, int n, float* y_dev);

/* Ensemble inference with routing.  Runs every net on x_dev [n x w_0];
 * writes y_mean_dev [n x w_L] (mean over nets) and spread_dev [n], where the
 * spread of a row is (max - min) / |mean| of the nets' peaks and a net's peak
 * is the largest of its w_L outputs (+INFINITY for a row outside the input
 * bound of sur_set_input_bound).  Rows whose spread exceeds `threshold`
 * (or is not finite) are listed in increasing order in fallback_dev (device,
 * room for n ints) and counted in *n_fallback_dev (device int). */
int sur_infer_route(sur_ctx* c, const float* x_dev, int n, float threshold, float* y_mean_dev,
                    float* spread_dev, int* fallback_dev, int* n_fallback_dev);

/* Inference kernels of sur_forward and sur_infer_route: 1 (default) runs
 * every layer of every net in one fused launch per chunk, the activations
 * of a block of rows held on chip (hidden widths up to 512, output width up
 * to 260); 0 runs one product launch per layer and net, as training does.
 * Both give the same bits.  Errors: EINVAL. */
int sur_set_kernel(sur_ctx* c, int fused);

/* Guard for sur_infer_route: a row any of whose inputs lies outside
 * [-bound, bound] is routed to the fallback whatever its spread (its spread
 * reads +INFINITY).  With inputs scaled so that the training box maps to
 * [-1, 1], bound 1 keeps every answer the ensemble gives inside the box it
 * was trained on.  Default INFINITY (off).  Errors: EINVAL (bound <= 0 or
 * NaN). */
int sur_set_input_bound(sur_ctx* c, float bound);

const char* sur_last_error(const sur_ctx* c);
void sur_destroy(sur_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* MI355_SUR_H */

/*
 * gcin.h -- C ABI of the GCIN smoother-coefficient predictor on MI355X (gfx950).
 *
 * The predictor maps the graph of each AMG level matrix to that level's smoother
 * coefficients (paper Sec. 3.2, Eqs. 6-10; App. A.1, Tab. 5):
 *   node features x_i = [a_ii, deg(i)] (Eq. 6, deg = stored off-diagonals of row i),
 *   four GCIN layers x^(l) = ReLU(InstanceNorm(A_hat x^(l-1) Theta_l + b_l)) with
 *   A_hat = (A - D) + I (Eqs. 7-8: edge weights a_ij, unit self-loops, no normalisation),
 *   InstanceNorm per graph (biased variance, eps 1e-5, affine),
 *   readout per layer [mean_i x_i, max_i x_i] -> Linear(128, 32) (Eq. 9), concatenation
 *   (Eq. 10), LayerNorm(128), sigmoid, MLP 128 -> 128 -> 64 -> 2d+1 with ReLU.
 * The paper's text gives several sizes for the head; this one has the 55,045 trainable
 * parameters it states (App. A.1) for d = 2.
 *
 * Parameters: one device FP32 array of gcin_param_count(d) values, tensors in this order:
 *   for l = 0..3: conv_l.W [in_l x 64] (in_0 = 2, else 64), conv_l.b [64], norm_l.gamma [64],
 *                 norm_l.beta [64];
 *   for l = 0..3: readout_l.W [128 x 32], readout_l.b [32];
 *   ln.gamma [128], ln.beta [128], mlp0.W [128 x 128], mlp0.b [128], mlp1.W [128 x 64],
 *   mlp1.b [64], mlp2.W [64 x (2d+1)], mlp2.b [2d+1].
 * Every W is row-major [fan_in x fan_out] and applied as y = x W + b.
 *
 * Precision: GCIN_FP32 evaluates everything in FP32. GCIN_BF16 runs the three 64 x 64 GCIN
 * linear layers (forward and both backward products) on BF16 MFMA (v_mfma_f32_16x16x32_bf16)
 * with FP32 accumulation and BF16 weights; the aggregated features entering each product
 * are split into a hi + lo BF16 pair because InstanceNorm removes their large per-graph
 * mean, which would otherwise amplify their rounding. GCIN_BF16X3 also splits the weights
 * (three MFMA products per tile), giving FP32-accurate activations on the MFMA units; use it
 * for training, where ReLU masks and arg-max pooling make gradients sensitive to activation
 * rounding. Activations, normalisation, pooling and the head stay FP32 in every mode.
 *
 * Hidden width: the functions without a width argument build the 64-channel network above.
 * The *_hidden variants also build the 32-channel variant that the paper proposes for
 * structured meshes, where the smaller network costs less setup time (App. B.3): every 64
 * above that counts GCIN channels becomes 32 (conv_l.W [in_l x 32], readout_l.W [64 x 32]);
 * the readout width, the head and the coefficient count are unchanged. Its tile products
 * run in FP32 whatever the precision argument (the MFMA tiling is written for 64 channels).
 *
 * Memory and streams as in amggnn.h: device pointers are caller-owned, the batch
 * lives in one caller-allocated workspace, every call is ordered on `stream`; 0 =
 * success, negative = error with the message in amgg_last_error(). Reductions use a
 * fixed order, so results are bitwise reproducible.
 */
#ifndef GCIN_H
#define GCIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GCIN_FP32 0
#define GCIN_BF16 1
#define GCIN_BF16X3 2
#define GCIN_MAX_GRAPHS 4096

/* Trainable parameter count for polynomial degree d (1..4): 55,045 for d = 2. */
int64_t gcin_param_count(int degree);
/* The same for hidden width 64 or 32 (-1 for another width or degree). */
int64_t gcin_param_count_hidden(int degree, int hidden);

/* One graph of the batch: a level matrix in device CSR (diagonal stored). */
typedef struct {
    int32_t n, nnz;
    const int32_t* rowptr;
    const int32_t* col;
    const double* val;
} gcin_graph;

typedef struct gcin_batch gcin_batch;

/* Workspace bytes for a batch of ngraphs graphs with the given host arrays of row and
 * entry counts (Alg. 1, steps 3-5: every level of every problem in one batch). */
int gcin_batch_workspace_bytes(int ngraphs, const int32_t* n, const int32_t* nnz, size_t* bytes);
/* Build the batched graph (aggregation matrix A_hat in FP32, node features) in the
 * workspace (device, 256-byte aligned). graphs is a host array of device CSR views.
 * The views are read during this call only. */
int gcin_batch_create(int ngraphs, const gcin_graph* graphs, void* workspace, size_t ws_bytes, void* stream,
                      gcin_batch** out);
/* The same for hidden width 64 or 32 (AMGG_EINVAL otherwise); forward and backward then use
 * the parameter layout of gcin_param_count_hidden(d, hidden). */
int gcin_batch_workspace_bytes_hidden(int hidden, int ngraphs, const int32_t* n, const int32_t* nnz, size_t* bytes);
int gcin_batch_create_hidden(int hidden, int ngraphs, const gcin_graph* graphs, void* workspace, size_t ws_bytes,
                             void* stream, gcin_batch** out);
/* The same with flags: GCIN_INFERENCE builds a batch for forward passes only (Alg. 1, step 6 at
 * solver setup): the forward keeps no aggregates for a backward and the layers' activations share
 * two buffers, so the workspace holds about a quarter of the training batch's (the training
 * batch keeps every layer's aggregates and activations and the backward's buffers); the
 * coefficients are bitwise those of a training batch, and gcin_backward on such a batch returns
 * AMGG_ESTATE. flags = 0 is the training batch of the functions above. */
#define GCIN_INFERENCE 1
int gcin_batch_workspace_bytes_ex(int hidden, int flags, int ngraphs, const int32_t* n, const int32_t* nnz,
                                  size_t* bytes);
int gcin_batch_create_ex(int hidden, int flags, int ngraphs, const gcin_graph* graphs, void* workspace,
                         size_t ws_bytes, void* stream, gcin_batch** out);
int gcin_batch_destroy(gcin_batch* b);

/* Forward pass (Alg. 1, step 6): coeffs_out is device FP32 [ngraphs][2d+1], raw
 * coefficients (d0..d_d, o1..o_d) in graph order. Keeps the activations for a backward. */
int gcin_forward(gcin_batch* b, int degree, int precision, const float* params, float* coeffs_out, void* stream);
/* Backward of the last forward: given dL/dcoeffs (device FP32 [ngraphs][2d+1]) writes dL/dparams
 * (device FP32, gcin_param_count(d) values; overwritten). */
int gcin_backward(gcin_batch* b, int degree, int precision, const float* params, const float* dcoeffs,
                  float* grads, void* stream);

/* Self-check of the dense 64 x 64 tile product used by the GCIN layers: with A, B device FP32
 * 64 x 64 row-major, writes A B computed by the FP32 path to D_fp32 and by the BF16 MFMA path
 * (v_mfma_f32_16x16x32_bf16, FP32 accumulation) to D_bf16. */
int gcin_tile_gemm_check(const float* A, const float* B, float* D_fp32, float* D_bf16, void* stream);

/* Adam step with global-norm gradient clipping (App. B.1, Tab. 7: Adam, learning rate 1e-3,
 * clipping at max norm 1.0): g <- g min(1, clip/||g||) (clip <= 0: no clipping), then
 * m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2, p <- p - lr (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps).
 * step t >= 1. gnorm_out (device, may be NULL) receives ||g|| before clipping. scratch is a
 * device buffer of adam_scratch_bytes() bytes. */
size_t adam_scratch_bytes(void);
int adam_step(float* params, const float* grads, float* m, float* v, int64_t n, float lr, float b1, float b2,
              float eps, int step, float clip, float* gnorm_out, void* scratch, void* stream);

/* adam_step without any allocation, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight training loops, harnesses that forbid hipMalloc): the same kernels and
 * results, with the step's scratch (the per-workgroup partial sums of ||g||^2 and the clipping
 * scalars, adam_scratch_bytes() = 2,112 bytes) in a static device array of exactly that size that
 * the library holds on each GPU it runs on until the process ends. That scratch does not grow
 * with n, so no n >= 1 is beyond its capacity. Allocates nothing (no hipMalloc, no library
 * allocation). The stream's device (the current device for stream NULL) is the GPU used. Every
 * call on one GPU shares that GPU's scratch: calls that overlap in time on one GPU (on different
 * streams, or from several threads) race and must be serialised by the caller. Each call writes
 * every scratch value it reads before reading it, so no clearing is needed between calls.
 * Errors: AMGG_EINVAL (null pointer, n < 1, step < 1), AMGG_EHIP. */
int adam_step_noalloc(float* params, const float* grads, float* m, float* v, int64_t n, float lr, float b1, float b2,
                      float eps, int step, float clip, float* gnorm_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* GCIN_H */

/*
 * alloc_mlp.h -- C ABI of the warm-start network for the allocator of
 * include/alloc.h (MI355X, BF16 matrix cores, FP32 accumulation).
 *
 * The paper's Dinkelbach iteration (Sec. III) starts from an allocation p^0
 * and its dual loop (Sec. IV-A, Alg. 1) from non-negative multipliers; the
 * paper leaves both unspecified.  This network predicts
 * them from per-triple features, so that the first Dinkelbach parameter
 * E^1 = R(p^0)/P(p^0) is already close to the optimum and the multipliers
 * start near their final values.  The network is not part of the paper.
 *
 * Network, per triple (m, n, k):
 *  - features x = [(10 log10(Gamma pmask_m / sigma) - 20)/20,  streaming flag,
 *                  Psi_k (0 for elastic users),  (10 log10(1000 pmax_m) - 40)/10];
 *  - 4 -> 256 -> 256 -> 256 -> 3, GELU (tanh form) after each hidden layer;
 *  - outputs y = [power logit, xi contribution, zeta contribution].
 * Powers are coded over six decades below the mask: code(p) = 1 + log10(p/pmask)/6.
 * Warm start of a drop: q = sigmoid(y0), p0 = pmask_m 10^(6(q-1)) where q >= 0.1
 * else 0;
 * xi0_m = expm1(clip(mean_{n,k} y1, 0, 30)); zeta0_k = expm1(clip(mean_{m,n}
 * y2, 0, 30)) for streaming users, 0 for elastic users.
 * Training loss per row: w0 BCE-with-logits(y0, t0) + w1 (y1-t1)^2 +
 * w2 (y2-t2)^2, averaged over rows; targets from a solved drop are
 * t0 = code(p) clipped to [0,1] (0 where p = 0), t1 = log1p(xi_m),
 * t2 = log1p(zeta_k), weights 1, 1, and the streaming flag.
 *
 * Rounding: inputs, weight matrices, hidden activations and the upstream
 * gradients that enter products are bfloat16 (round to nearest even);
 * products accumulate in FP32; biases, pre-activations, outputs, gradients,
 * the master weights and the AdamW moments are FP32.
 *
 * Parameters are one FP32 vector of ALLOC_MLP_NPARAMS values, row-major, in
 * the order W1 [256][4], b1 [256], W2 [256][256], b2 [256], W3 [256][256],
 * b3 [256], W4 [3][256], b4 [3] (W[out][in]).
 *
 * Conventions as in alloc.h: negative return = error (ALLOC_EINVAL,
 * ALLOC_ENOMEM, ALLOC_EDEVICE), outputs untouched; a network belongs to the
 * context it was created on and uses its stream; calls on one network must
 * not overlap.  Array arguments of the data-plane calls are DEVICE pointers
 * unless stated otherwise.
 */
#ifndef ALLOC_MLP_H
#define ALLOC_MLP_H
#include <stdint.h>

#include "alloc.h"

#ifdef __cplusplus
extern "C" {
#endif

#define ALLOC_MLP_NIN 4
#define ALLOC_MLP_HID 256
#define ALLOC_MLP_NOUT 3
#define ALLOC_MLP_NPARAMS 133635

/* alloc_result.status_flags: the warm-started solve ended non-finite, with no
 * allocation (EE <= 0) or infeasible for C12 or C13 (ALLOC_BUDGET_INFEASIBLE,
 * ALLOC_QOS_INFEASIBLE), and the returned result is the cold-started solve's */
#define ALLOC_WARM_FALLBACK 128u

typedef struct alloc_mlp alloc_mlp;

typedef struct {
  float lr;           /* step size */
  float beta1, beta2; /* moment decay rates (0.9, 0.999) */
  float eps;          /* 1e-8 */
  float weight_decay; /* decoupled decay of the weight matrices (biases are not decayed) */
} alloc_mlp_opt;

/* Create a network on the context's device, parameters zero until set.  Owns
 * its FP32 master weights, AdamW moments, BF16 copies and scratch. */
ALLOC_API int alloc_mlp_create(alloc_ctx* ctx, alloc_mlp** out);
ALLOC_API void alloc_mlp_destroy(alloc_mlp* net);

/* Host copies of the FP32 master parameters (n must be ALLOC_MLP_NPARAMS).
 * Setting parameters also resets the AdamW moments and step count. */
ALLOC_API int alloc_mlp_set_params(alloc_mlp* net, const float* host, int64_t n);
ALLOC_API int alloc_mlp_get_params(alloc_mlp* net, float* host, int64_t n);

/* Save the FP32 master parameters to the file at `path` (created or
 * replaced), or load them from it, in the safetensors layout: a little-endian
 * uint64 header length, a JSON header with one tensor "params" (dtype F32,
 * shape [ALLOC_MLP_NPARAMS]) and metadata naming the layer sizes, then the
 * values.  The AdamW moments are not saved; loading resets them as
 * alloc_mlp_set_params does.  Returns ALLOC_EFILE when the file cannot be
 * written or read, or does not hold such a tensor; ALLOC_EINVAL for a NULL
 * argument or a non-finite value; the network is unchanged on error. */
ALLOC_API int alloc_mlp_save(alloc_mlp* net, const char* path);
ALLOC_API int alloc_mlp_load(alloc_mlp* net, const char* path);

/* Features [M*N*K][4] (float32, device) of every triple of a drop, in
 * [M][N][K] order.  The gain pointer follows ALLOC_GAIN_ON_DEVICE in flags. */
ALLOC_API int alloc_mlp_features(alloc_mlp* net, const alloc_problem* prob, uint32_t flags,
                                 float* feat);

/* Forward pass of R rows: feat [R][4] float32 -> y [R][3] float32. */
ALLOC_API int alloc_mlp_forward(alloc_mlp* net, int64_t R, const float* feat, float* y);

/* Loss and gradients of R rows without an update: grad [ALLOC_MLP_NPARAMS]
 * float32 (device, may be NULL), *loss (host, mean over rows). */
ALLOC_API int alloc_mlp_grad(alloc_mlp* net, int64_t R, const float* feat, const float* target,
                             const float* weight, float* grad, double* loss);

/* One AdamW step on the loss of R rows; *loss (host, may be NULL) is the loss
 * before the step. */
ALLOC_API int alloc_mlp_train_step(alloc_mlp* net, int64_t R, const float* feat,
                                   const float* target, const float* weight,
                                   const alloc_mlp_opt* opt, double* loss);

/* One AdamW step from a given gradient grad [ALLOC_MLP_NPARAMS] (device). */
ALLOC_API int alloc_mlp_adamw(alloc_mlp* net, const float* grad, const alloc_mlp_opt* opt);

/* Training rows of a solved drop: for the R triples idx[R] (int64 flat
 * [M][N][K] indices, device) writes features feat [R][4], targets
 * target [R][3] and loss weights weight [R][3] (float32, device), from the
 * dense solved powers power [M][N][K] (float32, device) and the final
 * multipliers xi [M], zeta [K] (float64, device).  An index outside
 * [0, M*N*K) gives an all-zero row (zero loss weights). */
ALLOC_API int alloc_mlp_rows(alloc_mlp* net, const alloc_problem* prob, uint32_t flags,
                             const float* power, const double* xi, const double* zeta,
                             int64_t R, const int64_t* idx, float* feat, float* target,
                             float* weight);

/* Warm start of one drop from the network: p0 [M][N][K], xi0 [M], zeta0 [K]
 * (float64, device), as defined above. */
ALLOC_API int alloc_mlp_warm(alloc_mlp* net, const alloc_problem* prob, uint32_t flags, double* p0,
                             double* xi0, double* zeta0);

/* Network inference, then alloc_solve from that warm start.  Falls back to
 * the cold start (and sets ALLOC_WARM_FALLBACK) when the warm-started solve
 * ends non-finite, with EE <= 0 (nothing allocated) or infeasible for C12 or
 * C13 (the constraints the method meets when it converges; every returned
 * allocation meets C14), or, with alloc_params.warm_max_dinkelbach set, has
 * not converged within that many Dinkelbach steps: the cold-started solve is
 * then returned, whatever its own flags. */
ALLOC_API int alloc_solve_mlp(alloc_mlp* net, const alloc_problem* prob, const alloc_params* prm,
                              alloc_result* res);

/* Network inference for B drops, then alloc_solve_batch from those warm
 * starts; drops whose warm-started solve needs the fallback (as for
 * alloc_solve_mlp) are solved again from the cold start in a second batch
 * (ALLOC_WARM_FALLBACK). */
ALLOC_API int alloc_solve_batch_mlp(alloc_mlp* net, int32_t B, const alloc_problem* probs,
                                    const alloc_params* prm, alloc_result* results);

/* Duration in ms of the network's kernels in the last alloc_solve_mlp /
 * alloc_solve_batch_mlp / alloc_mlp_forward call when the context's timing is
 * enabled (-1 otherwise). */
ALLOC_API double alloc_mlp_last_ms(alloc_mlp* net);

#ifdef __cplusplus
}
#endif
#endif

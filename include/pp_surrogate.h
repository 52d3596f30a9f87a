/*
 * pp_surrogate.h - C ABI of the learned surrogate in libpp.
 *
 * The paper notes that the depth-dependent optics of the ice make simple
 * light models inaccurate and force photon-by-photon Monte Carlo, which is
 * the expensive part of the chain (Sec. 1, detector paragraph; Sec. 2,
 * photon-propagation paragraph). The surrogate learns, from hits that this
 * library's own Monte Carlo generates, the expected number of hits of a
 * module from a Cherenkov source and gamma parameters of the hit delay, so
 * that expectations for many (source, module) pairs come from one network
 * evaluation instead of many propagated photons. The Monte Carlo stays the
 * judge of its error and the fallback where the error check fails.
 *
 * Model (fixed shape): 29 features of a (source, module) pair, padded to
 * 64 -> five affine layers 64 -> 256 -> 256 -> 256 -> 256 -> 64 with GELU
 * between them; BF16
 * weights and activations, FP32 accumulation on the matrix cores, FP32
 * master weights and Adam state. Output 0 is log(mu / mu_base), where
 * mu_base is a diffusion estimate of the hit probability per photon;
 * outputs 1 and 2 are log(kappa) and log(theta / 50 ns) of a gamma
 * distribution of the hit delay. Loss per pair: the Poisson negative
 * log-likelihood of the hit count plus 0.1 times the gamma negative
 * log-likelihood of the delays, times the row's weight, averaged over the
 * rows of the batch.
 *
 * A pair set is every (source, module) pair of a batch submitted to the
 * context (pp_submit), source-major: pair p = source p / n_doms, module
 * p % n_doms. Surrogate sources must be Cherenkov segments.
 *
 * Conventions as in pp.h: status codes, caller-owned outputs, one surrogate
 * per context at a time, not thread-safe.
 */
#ifndef PP_SURROGATE_H_
#define PP_SURROGATE_H_

#include <stdint.h>

#include "pp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pp_surrogate pp_surrogate;

/* Creates a surrogate on ctx's device; ice and geometry must be loaded
 * (PP_ESTATE otherwise). Weights are initialised from init_seed. */
pp_status pp_sur_create(pp_context *ctx, uint64_t init_seed, pp_surrogate **out);
void pp_sur_destroy(pp_surrogate *sur); /* NULL-safe */

/* Number of f32 parameters: per layer, W (out x in, row-major) then b. */
uint64_t pp_sur_param_count(void);
pp_status pp_sur_get_params(pp_surrogate *sur, float *out, uint64_t n);
/* Sets all parameters (n must equal the count) and clears the Adam state. */
pp_status pp_sur_set_params(pp_surrogate *sur, const float *in, uint64_t n);

/* Which pairs of a batch the next pp_sur_set_training_set keeps. With
 * far_stride = 1 (the default) every pair is a row of weight 1. With
 * far_stride > 1 a pair is kept if the module centre lies within near_m
 * metres of the segment centre (weight 1), or else if (module id + source
 * index) mod far_stride == 0 (weight far_stride): an evenly spread
 * 1-in-far_stride sample of the far pairs whose weighted loss has the
 * expectation of the full set's, so training spends its work where the
 * light is. near_m >= 0 (INFINITY keeps every pair); PP_EINVAL otherwise
 * or for far_stride = 0. */
pp_status pp_sur_set_sampling(pp_surrogate *sur, float near_m, uint32_t far_stride);

/* Makes the (source, module) pairs of the context's batch the training set
 * (all of them, or the sample chosen by pp_sur_set_sampling, in
 * source-major order): computes the pair features on the device, and
 * labels from the batch's hits (which must have been propagated; the hit
 * buffer is completed first). Each source of the batch needs its own event
 * id. With sampling, at most 2^31 pairs per batch. */
pp_status pp_sur_set_training_set(pp_surrogate *sur, uint64_t batch);

/* Number of rows (kept pairs) in the training set. */
pp_status pp_sur_training_size(const pp_surrogate *sur, uint64_t *n_pairs);

/* Copies, for training rows [first, first + count), the pair index
 * (source-major, as above) and the loss weight to host memory. Either
 * pointer may be NULL. */
pp_status pp_sur_get_training_pairs(pp_surrogate *sur, uint64_t first, uint64_t count, uint64_t *pair,
                                    float *weight);

/* Number of real input features per (segment, module) pair (29): the pair
 * geometry up to a rotation about the vertical, the segment's extent, the
 * optics of the layers at the segment centre and at the module, and of the
 * layers 20 m above and below each. */
uint32_t pp_sur_feature_count(void);

/* Copies training-set rows [first, first + count) to host memory:
 * pp_sur_feature_count() features per row (bf16 values widened to float),
 * mu_base, and labels (k, n_t, sum of delays, sum of log delays). Any output
 * pointer may be NULL. */
pp_status pp_sur_get_training_rows(pp_surrogate *sur, uint64_t first, uint64_t count, float *features,
                                   float *mu_base, float *k, float *n_t, float *s1, float *s2);

/* Loss and gradient (f32, parameter layout) over training rows
 * [first, first + count) as one batch, without an update. PP_EINVAL unless
 * 0 < count <= 2^30 and the rows lie within the training set. Work buffers
 * grow with count (about 4.4 KB per row for the activations the weight
 * gradients read). */
pp_status pp_sur_loss_grad(pp_surrogate *sur, uint64_t first, uint64_t count, double *loss, float *grad);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr on
 * rows [first, first + count) (the same bounds); *loss gets the loss before
 * the step. */
pp_status pp_sur_train_step(pp_surrogate *sur, uint64_t first, uint64_t count, float lr, double *loss);

/* Trains for the given epochs over the whole training set in minibatches of
 * batch_size rows (a multiple of 64, at most 2^30) on hip_stream. Every epoch visits the
 * rows in a fresh pseudo-random order (an affine permutation of the row
 * index modulo the set size, multiplier coprime to it), so each minibatch
 * mixes pairs of many sources. The Adam learning rate follows a cosine from
 * lr at the first step to lr_final at the last step of this call (lr_final
 * = lr: constant). epoch_loss (may be NULL) receives the mean loss of each
 * epoch. */
pp_status pp_sur_train(pp_surrogate *sur, uint32_t epochs, uint32_t batch_size, float lr, float lr_final,
                       void *hip_stream, float *epoch_loss);

/* Distance beyond which inference takes a pair's expected hits as 0
 * without evaluating the network (default +inf: no cut). The distance is
 * from the segment centre to the module centre; a tile of 128 pairs with
 * none inside the cut is skipped whole. Light is absorbed within about
 * 100 m in this ice, so a cut of a few hundred metres changes no
 * expectation that matters and skips most of the detector. PP_EINVAL
 * unless cut_m > 0. Applies to the two calls below. */
pp_status pp_sur_set_inference_cut(pp_surrogate *sur, float cut_m);

/* Expected hits (photons of the source times the predicted probability
 * per photon) of every (source, module) pair of the context's batch,
 * summed per module into dev_dom_sums (n_doms doubles in device memory,
 * overwritten), on hip_stream. */
pp_status pp_sur_expected_hits(pp_surrogate *sur, uint64_t batch, double *dev_dom_sums, void *hip_stream);

/* Expected hits of every pair of the batch into host memory out (n_sources
 * x n_doms f32, source-major). n must equal that size. */
pp_status pp_sur_predict_pairs(pp_surrogate *sur, uint64_t batch, float *out, uint64_t n);

#ifdef __cplusplus
}
#endif

#endif /* PP_SURROGATE_H_ */

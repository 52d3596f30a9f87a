// Internal interface between the surrogate host code (sur_api.cpp) and its
// gfx950 kernels (sur_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pp_device.h"

namespace sur {

constexpr int kInReal = 29, kInPad = 64, kHidden = 256, kOutPad = 64, kOutReal = 3;
constexpr float kTanCherenkov = 0.86928673781622666f;  // tan 41 deg
constexpr float kNeighbourDz = 20.0f;  // depth offset (m) of the neighbouring optics features
constexpr int kLayers = 5;
constexpr int kTile = 64;            // GEMM workgroup tile (rows and columns)
constexpr float kTau0Ns = 50.0f;     // gamma scale unit of the delay model
constexpr float kTimeWeight = 0.1f;  // weight of the delay term in the loss

// Layer l maps in_dim(l) -> out_dim(l); weights are stored out x in.
__host__ __device__ constexpr int in_dim(int l) { return l == 0 ? kInPad : kHidden; }
__host__ __device__ constexpr int out_dim(int l) { return l == kLayers - 1 ? kOutPad : kHidden; }

// Flat parameter layout (f32): for each layer, W (out x in) then b (out).
__host__ __device__ constexpr int64_t w_offset(int l) {
  int64_t o = 0;
  for (int j = 0; j < l; ++j) o += (int64_t)out_dim(j) * in_dim(j) + out_dim(j);
  return o;
}
__host__ __device__ constexpr int64_t b_offset(int l) { return w_offset(l) + (int64_t)out_dim(l) * in_dim(l); }
__host__ __device__ constexpr int64_t param_count() { return w_offset(kLayers); }
// bf16 weight copies: W (out x in) and W^T (in x out), layer after layer,
// each matrix tile-major: the 16 x 32 tile (rows 16 t .., columns 32 s ..)
// of a matrix with K columns is 512 elements at (t (K / 32) + s) 512,
// lane-major inside (lane l: row l % 16, columns 8 (l / 16) .. + 8), the
// operand layout of v_mfma_f32_16x16x32_bf16. A wavefront's fragment load
// then reads 1 KB contiguous: whole cache lines.
__host__ __device__ constexpr int64_t frag_offset(int r, int k, int K) {
  return ((int64_t)(r / 16) * (K / 32) + k / 32) * 512 + ((r % 16) + 16 * ((k % 32) / 8)) * 8 + k % 8;
}
__host__ __device__ constexpr int64_t wb_offset(int l) {
  int64_t o = 0;
  for (int j = 0; j < l; ++j) o += (int64_t)out_dim(j) * in_dim(j);
  return o;
}
__host__ __device__ constexpr int64_t wb_count() { return wb_offset(kLayers); }

struct FeatureArgs {
  const pp::DevSource *sources;
  const float *src_nph;       // photons per source
  int n_sources_set;          // sources in the pair set (rows = source-major pairs)
  const float4 *doms;         // module centres, module-id order
  int n_doms;
  const pp::DevLayer *layers;
  int n_layers;
  float z_lo, inv_dz, radius;
  int64_t first_pair, n_pairs;  // rows [first, first + n) of the set
  const int64_t *pair_of_row;   // pair index of each row (source-major), null: row = pair
  uint16_t *X;    // bf16 n x 64 (rows padded to a multiple of 64 with zeros)
  uint16_t *XT;   // bf16 64 x ldxt (column = pair - first), may be null
  int64_t ldxt;
  float *mu_base; // per pair, may be null
  float *nph;     // photons of the pair's source, may be null
  float *r_out;   // distance per pair, may be null
};

// Training-pair selection: a (source, module) pair is kept if the module
// centre lies within near_m of the segment centre, or else if
// (module + source) mod far_stride == 0, with loss weight far_stride; the
// far pairs kept are then an evenly spread 1-in-far_stride sample whose
// weighted loss has the expectation of the full set's.
struct SelectArgs {
  const pp::DevSource *sources;
  int n_sources;
  const float4 *doms;   // module centres, module-id order
  int n_doms;
  float near2;          // near_m^2
  uint32_t far_stride;
  const int64_t *row_offset;  // first row of each source (exclusive prefix of the counts)
  int64_t n_rows;             // rows allocated (scatter pass): no row at or past it is written
  uint32_t *count;            // kept pairs per source (counting pass)
  int64_t *pair_of_row;       // row -> pair (scatter pass)
  int32_t *row_of_pair;       // pair -> row or -1 (scatter pass)
  float *w;                   // row -> loss weight (scatter pass)
};
hipError_t launch_select(const SelectArgs &a, bool scatter, hipStream_t s);

hipError_t launch_features(const FeatureArgs &f, hipStream_t s);
hipError_t launch_pack_weights(const float *theta, uint16_t *w_bf16, uint16_t *wt_bf16, hipStream_t s);
hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t s);
hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s);
hipError_t launch_labels(const pp::DevHit *hits, const unsigned long long *hit_count, uint64_t hit_cap,
                         const int32_t *event_to_source, uint32_t n_events, const pp::DevSource *sources,
                         const float4 *doms, int n_doms, float radius, float time_per_m,
                         const int32_t *row_of_pair, float *k, float *n_t, unsigned long long *s1q,
                         unsigned long long *s2q, float *s1, float *s2, int64_t n_rows, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t s);

// One training minibatch in three launches.
//
// launch_train_rows: kTrainRows minibatch rows per workgroup. Row i < count
// of the minibatch is training row (mul (first + i) + add) mod P (mul
// coprime to P: a permutation); rows count..M-1 are zero and carry no loss.
// Forward, loss and backward down to dZ_0 run with the rows' activations in
// LDS; what the weight gradients need leaves as bf16 with the minibatch row
// contiguous, and each workgroup stores its loss sum and the column sums of
// its dZ_l and dY rows (the bias gradients' parts).
// launch_wgrad: dW_l = dZ_l^T H_{l-1} (dY for the output layer, X for the
// first), every layer in one launch; K slice s (the 32-row blocks s,
// s + splits, ...) stores its partial product.
// launch_reduce_adam: per parameter, the partials added in slice order (the
// bias parts in row-block order), the gradient stored, then (if adam) the
// Adam step and the bf16 weight copies.
constexpr int kTrainRows = 32;                    // minibatch rows per workgroup of the row pass
constexpr int kTrainLd = kHidden + 8;             // LDS row stride (elements) of activations and GELU'
constexpr int kDyLd = kOutPad + 8;                // LDS row stride of the output gradient
constexpr int kBiasCols = 4 * kHidden + kOutPad;  // bias-gradient columns per row block: dZ_0..dZ_3, then dY
constexpr int kWgradSplits = 16;                  // K slices of the weight gradients (at most)

// Tiles of layer l's weight gradient: 128 x 128, or the layer's whole
// extent where it is 64 (inputs of layer 0, outputs of the last), and
// their running offset.
__host__ __device__ constexpr int wgrad_tm(int l) { return out_dim(l) < 128 ? out_dim(l) : 128; }
__host__ __device__ constexpr int wgrad_tn(int l) { return in_dim(l) < 128 ? in_dim(l) : 128; }
__host__ __device__ constexpr int wgrad_tiles(int l) { return (out_dim(l) / wgrad_tm(l)) * (in_dim(l) / wgrad_tn(l)); }
__host__ __device__ constexpr int wgrad_tile_offset(int l) {
  int o = 0;
  for (int j = 0; j < l; ++j) o += wgrad_tiles(j);
  return o;
}

struct TrainArgs {
  const uint16_t *X;                               // bf16 training features, 64 per row
  const float *mu_base, *nph, *k, *n_t, *s1, *s2;  // labels per training row
  const float *w;                                  // loss weight per training row, null: 1
  uint64_t P, mul, add;
  int64_t first;
  int count, M;                    // real rows; M = count rounded up to a multiple of 64
  float inv_norm;                  // 1 / count
  const uint16_t *wb[kLayers];     // bf16 W (out x in), tile-major (frag_offset)
  const uint16_t *wt[kLayers];     // bf16 W^T (in x out), tile-major
  const float *b[kLayers];
  uint16_t *XT, *HT[4], *dYT, *dZT[4];  // bf16, row-block-major: block b's column c at (b n_cols + c) kTrainRows
  float *col_part;                 // kBiasCols x (M / kTrainRows): a bias column's row-block parts contiguous
  double *loss_part;               // M / kTrainRows
};
struct WgradArgs {
  const uint16_t *A[kLayers];  // dZ_l (out columns); dY for the output layer; row-block-major as the row pass writes
  const uint16_t *B[kLayers];  // H_{l-1} (in columns); X for the first layer
  int M, splits;               // splits <= M / kTrainRows
  float *ws;                   // layer l: splits x out x in partials from ws + splits * wb_offset(l)
};
struct AdamArgs {
  float *theta, *grad, *m, *v;
  uint16_t *wb, *wt;
  const float *ws;
  int splits;
  const float *col_part;
  const double *loss_part;
  int n_blocks;                // row blocks of the bias and loss parts
  double *loss_sum;            // set to the minibatch loss (weighted sum over rows)
  double *loss_epoch;          // also added to, if not null
  int adam;                    // 0: gradient only
  float lr, c1, c2;            // Adam step size and bias corrections 1 - beta^t
};
size_t train_lds_bytes();
hipError_t launch_train_rows(const TrainArgs &a, hipStream_t s);
hipError_t launch_wgrad(const WgradArgs &g, hipStream_t s);
hipError_t launch_reduce_adam(const AdamArgs &a, hipStream_t s);

// Fused inference over pairs [f.first_pair, f.first_pair + f.n_pairs):
// features, the five layers and the expected hits, kFusedRows pairs per
// workgroup of 256 threads with the activations in LDS.
constexpr int kFusedRows = 128;
constexpr int kFusedLd = kHidden + 8;  // LDS row stride of the activations (bf16); the pad spreads rows over banks
struct FusedArgs {
  FeatureArgs f;                 // the pair set (its output pointers are unused)
  const uint16_t *w[kLayers];    // bf16 weights, out x in, tile-major (frag_offset)
  const float *b[kLayers];       // biases
  double *dom_sums;              // += expected hits per module (atomically: the last bits vary), may be null
  float *pair_mu;                // expected hits of pair first_pair + i at i, may be null
  float cut2;                    // pairs farther apart than sqrt(cut2) expect 0 hits (+inf: no cut)
};
size_t fused_lds_bytes();
hipError_t launch_infer_fused(const FusedArgs &a, hipStream_t s);

}  // namespace sur

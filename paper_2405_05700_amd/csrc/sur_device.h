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
// bf16 weight copies: W (out x in) and W^T (in x out), layer after layer.
__host__ __device__ constexpr int64_t wb_offset(int l) {
  int64_t o = 0;
  for (int j = 0; j < l; ++j) o += (int64_t)out_dim(j) * in_dim(j);
  return o;
}
__host__ __device__ constexpr int64_t wb_count() { return wb_offset(kLayers); }

enum Epilogue {
  kEpiGelu = 0,     // z = acc + bias; store z (f32) unless null, gelu(z) as bf16 and its transpose unless null
  kEpiGeluBwd = 1,  // dz = acc * gelu'(z_saved); store bf16 and its transpose
  kEpiSplitK = 2,   // out (f32) = acc summed over the K slices: each slice stores its partial in ws, then
                    // a reduction adds them in slice order
  kEpiLinear = 4,   // out (f32, ld N) = acc + bias
};

struct GemmArgs {
  // C[M x N] = A[M x K] * B[N x K]^T ; A, B bf16 with K contiguous
  const uint16_t *A;
  int64_t lda;
  const uint16_t *B;
  int64_t ldb;
  int M, N, K;
  int k_chunk;  // K range per grid.z slice
  const float *bias;
  float *Z;          // f32 M x N (ld N)
  uint16_t *H;       // bf16 M x N (ld N)
  uint16_t *HT;      // bf16 N x M (ld ldt)
  int64_t ldt;
  const float *Zin;  // saved pre-activation for kEpiGeluBwd (ld N)
  float *out;        // kEpiSplitK: f32 M x N (ld N)
  float *ws;         // kEpiSplitK: f32 splits x M x N partials
  float *col_sums;   // kEpiGeluBwd: column sums of the stored bf16 output (bias gradient), may be null;
  float *col_part;   //   formed from per-32-row partials (M / 32 x N, f32) in row order
};

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

struct LossArgs {
  const float *Y;        // f32 M x 64 (ld 64)
  const float *mu_base, *nph, *k, *n_t, *s1, *s2;  // per row
  const float *w;        // loss weight per row, null: 1
  int M_real, M_pad;
  float inv_norm;        // 1 / number of pairs averaged over
  uint16_t *dY;          // bf16 M_pad x 64
  uint16_t *dYT;         // bf16 64 x M_pad
  double *loss_sum;      // set to the loss summed over the rows
  double *loss_epoch;    // also accumulated into, if not null
  float *out_bias_grad;  // set to the column sums of the stored bf16 dY (output-layer bias gradient), may be null
  double *loss_part;     // per-workgroup partials (loss_blocks(M_pad) of each)
  float *bias_part;      //   (3 per workgroup)
};
int loss_blocks(int M_pad);

// Copies training rows p(r) = (mul * r + add) mod P, r in [first, first + count),
// into dense minibatch buffers (row i of the batch = row p(first + i)); rows
// [count, M) of the batch are zero. mul is coprime to P, so p is a permutation.
struct GatherArgs {
  const uint16_t *X;                                // bf16 P_pad x 64
  const float *mu_base, *nph, *k, *n_t, *s1, *s2;   // per training row
  const float *w;                                   // per training row, may be null
  uint64_t P, mul, add;
  int64_t first;
  int count, M;
  uint16_t *gX;    // bf16 M x 64
  uint16_t *gXT;   // bf16 64 x M
  float *g_mu_base, *g_nph, *g_k, *g_n_t, *g_s1, *g_s2;
  float *g_w;      // written only if w is not null
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

hipError_t launch_gemm(int epi, const GemmArgs &g, int splits, hipStream_t s);
hipError_t launch_gather(const GatherArgs &g, hipStream_t s);
hipError_t launch_features(const FeatureArgs &f, hipStream_t s);
hipError_t launch_loss(const LossArgs &l, hipStream_t s);
hipError_t launch_adam(float *theta, const float *grad, float *m, float *v, int64_t n, float lr,
                       float c1, float c2, hipStream_t s);
hipError_t launch_pack_weights(const float *theta, uint16_t *w_bf16, uint16_t *wt_bf16, hipStream_t s);
hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t s);
hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s);
hipError_t launch_labels(const pp::DevHit *hits, const unsigned long long *hit_count, uint64_t hit_cap,
                         const int32_t *event_to_source, uint32_t n_events, const pp::DevSource *sources,
                         const float4 *doms, int n_doms, float radius, float time_per_m,
                         const int32_t *row_of_pair, float *k, float *n_t, unsigned long long *s1q,
                         unsigned long long *s2q, float *s1, float *s2, int64_t n_rows, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t s);

// Fused inference over pairs [f.first_pair, f.first_pair + f.n_pairs):
// features, the five layers and the expected hits, kFusedRows pairs per
// workgroup of 256 threads with the activations in LDS.
constexpr int kFusedRows = 128;
constexpr int kFusedLd = kHidden + 8;  // LDS row stride of the activations (bf16); the pad spreads rows over banks
struct FusedArgs {
  FeatureArgs f;                 // the pair set (its output pointers are unused)
  const uint16_t *w[kLayers];    // bf16 weights, out x in
  const float *b[kLayers];       // biases
  double *dom_sums;              // += expected hits per module (atomically: the last bits vary), may be null
  float *pair_mu;                // expected hits of pair first_pair + i at i, may be null
  float cut2;                    // pairs farther apart than sqrt(cut2) expect 0 hits (+inf: no cut)
};
size_t fused_lds_bytes();
hipError_t launch_infer_fused(const FusedArgs &a, hipStream_t s);

}  // namespace sur

// gfx950 kernels of the learned surrogate: a five-layer GELU perceptron in
// BF16 with FP32 accumulation on the matrix cores, its backward pass, loss,
// Adam, and the features / labels / reductions around it.
//
// Matrix products use v_mfma_f32_16x16x32_bf16. The weights (at most 128 KB
// per layer) stay in L2, so their fragments are loaded straight into VGPRs,
// 16 bytes per lane per fragment; activations are staged in LDS. Every sum
// that gradients or labels depend on is formed in a fixed order (partials
// reduced in order, or exact fixed-point atomics), so training is
// bit-reproducible.

#include "sur_device.h"
#include "gelu_cdf_table.h"

namespace sur {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 load8(const uint16_t *p) {
  const uint4 v = *reinterpret_cast<const uint4 *>(p);
  return __builtin_bit_cast(bf16x8, v);
}

// GELU for the fused inference kernel: z Phi(z) with Phi linear between the
// 1025 nodes of a table in LDS, read as float16 pairs (Phi_i, Phi_(i+1) -
// Phi_i) packed in 32 bits (gelu_table.py beside this file derives it and
// bounds the error: within 5.0e-4 relative where |GELU| > 0.01, a quarter of
// the bf16 rounding the activation then takes). Eight full-rate operations
// and one 4-byte LDS read; t = N (z >= 6) lands on the last node, whose
// difference is 0, and a NaN converts to index 0.
__device__ __forceinline__ float gelu_table(float z, const uint32_t *cdf) {
  const float t = __builtin_amdgcn_fmed3f(__builtin_fmaf(z, kCdfA, kCdfB), 0.0f, (float)kCdfN);
  const uint32_t e = cdf[(uint32_t)t];
  const float p = (float)__builtin_bit_cast(_Float16, (uint16_t)e);
  const float d = (float)__builtin_bit_cast(_Float16, (uint16_t)(e >> 16));
  return z * __builtin_fmaf(__builtin_amdgcn_fractf(t), d, p);
}

// Digamma for x > 0: recurrence psi(x) = psi(x + 1) - 1/x up to x >= 6, then
// the asymptotic expansion ln x - 1/(2x) - sum B_2n / (2n x^2n)
// (Abramowitz & Stegun 6.3.18).
__device__ __forceinline__ float digamma(float x) {
  float r = 0.0f;
  while (x < 6.0f) {
    r -= 1.0f / x;
    x += 1.0f;
  }
  const float f = 1.0f / (x * x);
  const float t = f * (1.0f / 12 - f * (1.0f / 120 - f * (1.0f / 252 - f * (1.0f / 240 - f * (1.0f / 132)))));
  return r + logf(x) - 0.5f / x - t;
}

// Workgroup barrier that orders LDS accesses only: global loads issued
// before it stay in flight (the kernels that use it pass nothing between
// wavefronts through global memory).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ bf16x8 lds_load8(const uint16_t *p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(p));
}

// Weight gradients of all five layers in one launch. Block (tile, slice) =
// (blockIdx.x / splits, blockIdx.x % splits), the tiles of layer 0 first.
// Slice s takes the minibatch's 32-row blocks s, s + splits, s + 2 splits,
// ...; the row pass wrote block b from its workgroup b, and consecutive
// workgroups are dispatched to the eight XCDs in turn, so with splits a
// multiple of 8 a slice reads only blocks written on the XCD it runs on
// (whatever of them that XCD's L2 still holds is read from there).
//
// A tile of TM x TN: each 32-row step stages the A rows (TM x 32) and B rows
// (TN x 32) in LDS (row stride 40 elements: the 16 rows a fragment read
// touches fall on distinct banks), and each wavefront multiplies its
// TM / 2 x TN / 2 quarter from there. The global loads run kWgradDepth steps
// ahead in VGPRs; the LDS stage is double-buffered. Each block stores its
// slice's partial product; the reduction adds the slices in order.
constexpr int kWgradLd = 40;
constexpr int kWgradDepth = 4;

// acc[i][j] += A rows 16 i .. (from a) x B rows 16 j .. (from b) over one
// 32-wide K step staged in LDS (a, b: this lane's fragment addresses).
template <int MI, int NI>
__device__ __forceinline__ void wgrad_products(f32x4 (&acc)[MI][NI], const uint16_t *a, const uint16_t *b) {
  bf16x8 af[MI], bf[NI];
#pragma unroll
  for (int i = 0; i < MI; ++i) af[i] = lds_load8(a + i * 16 * kWgradLd);
#pragma unroll
  for (int j = 0; j < NI; ++j) bf[j] = lds_load8(b + j * 16 * kWgradLd);
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
}

template <int TM, int TN>
__device__ __forceinline__ void wgrad_block(const WgradArgs &g, int l, int t, int s, uint16_t *stage) {
  constexpr int L = (TM + TN) * 4 / 256;  // 16-byte chunks per thread per step
  constexpr int kStage = (TM + TN) * kWgradLd;
  constexpr int D = kWgradDepth, MI = TM / 32, NI = TN / 32;
  static_assert((TM + TN) * 4 % 256 == 0, "whole chunks per thread");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wr = wave >> 1, wc = wave & 1;
  const int n_in = in_dim(l), n_out = out_dim(l);
  const int col_tiles = n_in / TN;
  const int r0 = (t / col_tiles) * TM, c0 = (t % col_tiles) * TN;
  const int n_blk = g.M / kTrainRows;
  const int n = (n_blk - s + g.splits - 1) / g.splits;  // this slice's steps
  // this thread's chunks: row c / 4 of the stage (A rows, then B rows), part c % 4
  const uint16_t *src[L];
  int64_t blk_stride[L];  // elements from one row block to the next in this chunk's array
  int dst[L];
#pragma unroll
  for (int q = 0; q < L; ++q) {
    const int c = tid + 256 * q, row = c >> 2, part = c & 3;
    src[q] = (row < TM ? g.A[l] + (int64_t)(r0 + row) * kTrainRows : g.B[l] + (int64_t)(c0 + row - TM) * kTrainRows) +
             part * 8;
    blk_stride[q] = (int64_t)(row < TM ? n_out : n_in) * kTrainRows;
    dst[q] = row * kWgradLd + part * 8;
  }
  f32x4 acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
  const int fr = (lane & 15) * kWgradLd + (lane >> 4) * 8;
  // The ring is four named register sets, each step written out for its
  // set, so every index is static and the sets stay in VGPRs.
  static_assert(D == 4, "the ring below has four sets");
  u32x4 ra[L], rb[L], rc[L], rd[L];  // native vectors: a uint4 struct would be copied through memory
  // Every step issues its loads, past the slice's end from its last block
  // (loaded, never used): the same count of loads in flight on every path
  // lets the compiler wait for exactly the set it needs (loads complete in
  // issue order).
#define WGRAD_LOAD(R, J)                                                                \
  {                                                                                     \
    const int64_t b_ = s + min((J), n - 1) * g.splits;                                  \
    _Pragma("unroll") for (int q = 0; q < L; ++q) R[q] = *reinterpret_cast<const u32x4 *>(src[q] + b_ * blk_stride[q]); \
  }
  // step j: its rows (in R) to LDS stage j & 1, the set reloaded with step
  // j + D, then the products. Stage j & 1 was last read by step j - 2,
  // which every wavefront finished before the barrier of step j - 1.
#define WGRAD_STEP(R, J)                                                                \
  {                                                                                     \
    const int j_ = (J);                                                                 \
    uint16_t *st_ = stage + (j_ & 1) * kStage;                                          \
    _Pragma("unroll") for (int q = 0; q < L; ++q) *reinterpret_cast<u32x4 *>(st_ + dst[q]) = R[q]; \
    WGRAD_LOAD(R, j_ + D);                                                              \
    lds_barrier();                                                                      \
    wgrad_products<MI, NI>(acc, st_ + wr * (TM / 2) * kWgradLd + fr, st_ + (TM + wc * (TN / 2)) * kWgradLd + fr); \
  }
  WGRAD_LOAD(ra, 0);
  WGRAD_LOAD(rb, 1);
  WGRAD_LOAD(rc, 2);
  WGRAD_LOAD(rd, 3);
  // whole rounds of the ring, then the last n % D steps
  int j0 = 0;
  for (; j0 + D <= n; j0 += D) {
    WGRAD_STEP(ra, j0);
    WGRAD_STEP(rb, j0 + 1);
    WGRAD_STEP(rc, j0 + 2);
    WGRAD_STEP(rd, j0 + 3);
  }
  if (j0 < n) WGRAD_STEP(ra, j0);
  if (j0 + 1 < n) WGRAD_STEP(rb, j0 + 1);
  if (j0 + 2 < n) WGRAD_STEP(rc, j0 + 2);
#undef WGRAD_STEP
#undef WGRAD_LOAD
  float *part = g.ws + (int64_t)g.splits * wb_offset(l) + (int64_t)s * n_out * n_in;
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int jn = 0; jn < NI; ++jn) {
      const int col = c0 + wc * (TN / 2) + jn * 16 + (lane & 15);
      const int rbase = r0 + wr * (TM / 2) + i * 16 + (lane >> 4) * 4;
#pragma unroll
      for (int r = 0; r < 4; ++r) part[(int64_t)(rbase + r) * n_in + col] = acc[i][jn][r];
    }
}

__global__ void __launch_bounds__(256) k_wgrad(const WgradArgs g) {
  __shared__ __align__(16) uint16_t stage[2 * 256 * kWgradLd];
  const int s = (int)(blockIdx.x % (unsigned)g.splits);
  int t = (int)(blockIdx.x / (unsigned)g.splits), l = 0;
  while (l + 1 < kLayers && t >= wgrad_tile_offset(l + 1)) ++l;
  t -= wgrad_tile_offset(l);
  if (l == 0)
    wgrad_block<wgrad_tm(0), wgrad_tn(0)>(g, l, t, s, stage);
  else if (l == kLayers - 1)
    wgrad_block<wgrad_tm(kLayers - 1), wgrad_tn(kLayers - 1)>(g, l, t, s, stage);
  else
    wgrad_block<128, 128>(g, l, t, s, stage);
}

constexpr double kDelayFix = 1048576.0;     // 2^20 per ns
constexpr double kLogFix = 4294967296.0;    // 2^32

__device__ __forceinline__ int layer_of(float z, float z_lo, float inv_dz, int n_layers) {
  const float f = floorf((z - z_lo) * inv_dz);
  return f >= 0.0f ? (f >= (float)(n_layers - 1) ? n_layers - 1 : (int)f) : 0;
}

// Features of pair p of the set (source-major: source p / n_doms, module
// p % n_doms) and its diffusion baseline.
__device__ __forceinline__ void pair_features(const FeatureArgs &f, int64_t p, float x[kInReal],
                                              float &mu_base, float &nph, float &R, int &dom) {
  // Divisions by constants are multiplications by their reciprocals, the
  // others hardware reciprocals, and square roots, logarithms and
  // exponentials the hardware's (each within about an ulp of float32): the
  // features are stored as bf16, 2^-8 relative, and the baseline is a smooth
  // physics estimate.
  const int i = (int)(p / f.n_doms), j = (int)(p % f.n_doms);
  const pp::DevSource &S = f.sources[i];
  const float4 m = f.doms[j];
  const float half = 0.5f * S.dir_len.w;
  const float cx = S.pos_t0.x + half * S.dir_len.x, cy = S.pos_t0.y + half * S.dir_len.y;
  const float cz = S.pos_t0.z + half * S.dir_len.z;
  const float dx = m.x - cx, dy = m.y - cy, dz = m.z - cz;
  R = fmaxf(__builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz), 0.5f);
  const float rR = __builtin_amdgcn_rcpf(R);
  const float ux = dx * rR, uy = dy * rR, uz = dz * rR;
  const float cos_eta = ux * S.dir_len.x + uy * S.dir_len.y + uz * S.dir_len.z;
  const pp::DevLayer Ls = f.layers[layer_of(cz, f.z_lo, f.inv_dz, f.n_layers)];
  const pp::DevLayer Ld = f.layers[layer_of(m.z, f.z_lo, f.inv_dz, f.n_layers)];
  // Geometry up to a rotation about the vertical (the ice is layered in
  // depth only): vertical parts, horizontal and vertical offsets, distance,
  // angle to the track and the relative azimuth of the horizontal parts.
  const float h = S.dir_len.x * ux + S.dir_len.y * uy;
  const float hh = __builtin_amdgcn_sqrtf((S.dir_len.x * S.dir_len.x + S.dir_len.y * S.dir_len.y) * (ux * ux + uy * uy));
  x[0] = uz;
  x[1] = __builtin_amdgcn_sqrtf(dx * dx + dy * dy) * 0.01f;
  x[2] = dz * 0.01f;
  x[3] = R * 0.01f;
  x[4] = (__builtin_amdgcn_logf(R) - 3.32192809488736235f) * 0.23104906018664843f;  // ln(R / 10) / 3 via log2
  x[5] = cos_eta;
  x[6] = cos_eta - 0.75470958022277199f;  // cos 41 deg
  x[7] = S.dir_len.z;
  x[8] = h;
  x[9] = hh > 1e-9f ? fminf(fmaxf(h * __builtin_amdgcn_rcpf(hh), -1.0f), 1.0f) : 0.0f;
  x[10] = cz * 0.002f;
  x[11] = m.z * 0.002f;
  x[12] = 100.0f * Ls.coef.x;
  x[13] = 10.0f * Ls.coef.y;
  x[14] = 100.0f * Ld.coef.x;
  x[15] = 10.0f * Ld.coef.y;
  // The segment's extent: impact parameter of the track line, along-track
  // offset of the closest approach from the centre, where on the segment (in
  // lengths, capped to [-1, 2]) direct Cherenkov light at 41 degrees would
  // leave for the module, and the distances to both ends.
  const float L = fmaxf(S.dir_len.w, 1e-3f);
  const float vx = m.x - S.pos_t0.x, vy = m.y - S.pos_t0.y, vz = m.z - S.pos_t0.z;
  const float along = vx * S.dir_len.x + vy * S.dir_len.y + vz * S.dir_len.z;
  const float px = vx - along * S.dir_len.x, py = vy - along * S.dir_len.y, pz = vz - along * S.dir_len.z;
  const float bimp = __builtin_amdgcn_sqrtf(px * px + py * py + pz * pz);
  const float ex = vx - L * S.dir_len.x, ey = vy - L * S.dir_len.y, ez = vz - L * S.dir_len.z;
  x[16] = bimp * 0.01f;
  x[17] = (along - 0.5f * L) * 0.01f;
  x[18] = fminf(fmaxf((along - bimp * (1.0f / kTanCherenkov)) * __builtin_amdgcn_rcpf(L), -1.0f), 2.0f);
  x[19] = __builtin_amdgcn_sqrtf(vx * vx + vy * vy + vz * vz) * 0.01f;
  x[20] = __builtin_amdgcn_sqrtf(ex * ex + ey * ey + ez * ez) * 0.01f;
  // The optics 20 m above and below the segment centre and the module:
  // where the depth profile changes within the range light diffuses over
  // (a dust layer), the two end layers alone do not say so.
  const float zq[4] = {cz + kNeighbourDz, cz - kNeighbourDz, m.z + kNeighbourDz, m.z - kNeighbourDz};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const pp::DevLayer Lq = f.layers[layer_of(zq[q], f.z_lo, f.inv_dz, f.n_layers)];
    x[21 + 2 * q] = 100.0f * Lq.coef.x;
    x[22 + 2 * q] = 10.0f * Lq.coef.y;
  }
  // diffusion baseline with the two layers' mean absorption and
  // effective scattering lengths (lambda_e = (1/b) / (1 - g))
  const float lam_a = 0.5f * (Ls.coef.z + Ld.coef.z);
  const float lam_e = 0.5f * (Ls.coef.w * __builtin_amdgcn_rcpf(Ls.hg.x) + Ld.coef.w * __builtin_amdgcn_rcpf(Ld.hg.x));
  const float D = lam_e * (1.0f / 3.0f);
  const float dl = __builtin_amdgcn_sqrtf(D * lam_a);
  // r^2 exp(-R / dl) / (4 D R), the exponential as 2^(-R log2(e) / dl)
  mu_base = f.radius * f.radius * __builtin_amdgcn_exp2f(-1.44269504088896341f * R * __builtin_amdgcn_rcpf(dl)) *
            __builtin_amdgcn_rcpf(4.0f * D * R);
  nph = f.src_nph[i];
  dom = j;
}

// Feature rows of pairs [first_pair, first_pair + n_pairs); rows past
// n_pairs (padding) are zero.
__global__ void k_features(const FeatureArgs f, int64_t n_rows) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n_rows) return;
  float x[kInReal];
  for (int q = 0; q < kInReal; ++q) x[q] = 0.0f;
  float mu_base = 0.0f, nph = 0.0f, R = 0.0f;
  int dom = 0;
  if (t < f.n_pairs)
    pair_features(f, f.pair_of_row ? f.pair_of_row[f.first_pair + t] : f.first_pair + t, x, mu_base, nph, R, dom);
  uint16_t *row = f.X + t * kInPad;
  for (int q = 0; q < kInPad; ++q) row[q] = q < kInReal ? f2bf(x[q]) : 0;
  if (f.XT)
    for (int q = 0; q < kInPad; ++q) f.XT[(int64_t)q * f.ldxt + t] = q < kInReal ? f2bf(x[q]) : 0;
  if (f.mu_base) f.mu_base[t] = mu_base;
  if (f.nph) f.nph[t] = nph;
  if (f.r_out) f.r_out[t] = R;
}

// Poisson + gamma negative log-likelihood of one row (times its weight)
// and its gradient with respect to the three outputs (log mu / mu_base,
// log kappa, log theta/tau0), scaled by weight / count.
struct RowLoss {
  double part;
  float g0, g1, g2;
};
__device__ __forceinline__ RowLoss row_loss(float y0, float y1_raw, float y2_raw, float mu_base, float nph,
                                            float k, float nt, float s1, float s2, float wt, float inv_norm) {
  RowLoss o{0.0, 0.0f, 0.0f, 0.0f};
  const float y1 = fminf(fmaxf(y1_raw, -8.0f), 8.0f), y2 = fminf(fmaxf(y2_raw, -8.0f), 8.0f);
  const float mu = nph * mu_base * expf(y0);
  const float kappa = expf(y1), theta = kTau0Ns * expf(y2);
  const float log_mu = logf(mu);
  const float pois = mu - (k > 0.0f ? k * log_mu : 0.0f);
  const float gam =
      nt > 0.0f ? nt * (lgammaf(kappa) + kappa * logf(theta)) - (kappa - 1.0f) * s2 + s1 / theta : 0.0f;
  o.part = (double)wt * ((double)pois + (double)kTimeWeight * gam);
  const float scale = wt * inv_norm;
  o.g0 = (mu - k) * scale;
  if (nt > 0.0f) {
    o.g1 = kTimeWeight * kappa * (nt * (digamma(kappa) + logf(theta)) - s2) * scale;
    o.g2 = kTimeWeight * (nt * kappa - s1 / theta) * scale;
    if (y1_raw != y1) o.g1 = 0.0f;  // clamped: no gradient through the clamp
    if (y2_raw != y2) o.g2 = 0.0f;
  }
  return o;
}

// Sum of part[i * stride] over i < n in a fixed order by one wavefront: lane
// l adds parts l, l + 64, l + 128, ... in turn, then the lanes combine by a
// fixed butterfly. The result depends only on the values, not on
// scheduling. Four of a lane's loads are issued before their additions, so
// their latencies overlap.
template <class T>
__device__ __forceinline__ T wave_ordered_sum(const T *part, int n, int64_t stride) {
  const int lane = threadIdx.x & 63;
  T sum = 0;
  int i = lane;
  for (; i + 192 < n; i += 256) {
    const T v0 = part[(int64_t)i * stride], v1 = part[(int64_t)(i + 64) * stride];
    const T v2 = part[(int64_t)(i + 128) * stride], v3 = part[(int64_t)(i + 192) * stride];
    __builtin_amdgcn_sched_barrier(0);  // keep the four loads ahead of the first addition
    sum += v0;
    sum += v1;
    sum += v2;
    sum += v3;
  }
  for (; i < n; i += 64) sum += part[(int64_t)i * stride];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
  return sum;
}

// The Adam step of one parameter (Kingma & Ba, beta1 0.9, beta2 0.999,
// eps 1e-8, bias corrections c1, c2). The two moment updates are written as
// explicit fused multiply-adds, so their rounding does not depend on which
// product the compiler would fuse.
__device__ __forceinline__ void adam_update(const AdamArgs &a, float g, float &th, float &m, float &v) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  m = __builtin_fmaf(b1, m, (1.0f - b1) * g);
  v = __builtin_fmaf(b2, v, (1.0f - b2) * g * g);
  th -= a.lr * (m / a.c1) / (sqrtf(v / a.c2) + eps);
}

constexpr int kWeightBlocks = (int)((wb_count() / 4 + 255) / 256);
constexpr int kBiasBlocks = kBiasCols / 4;
static_assert(wb_count() % 4 == 0 && w_offset(1) % 4 == 0 && wb_offset(1) % 4 == 0,
              "every layer's weights start on a 16-byte boundary");

// Blocks [0, kWeightBlocks): four consecutive weight elements per thread
// (of one row of one layer), their K-slice partials added in slice order,
// then the step and the bf16 copies in both layouts. The next kBiasBlocks:
// one bias element per wavefront, its row-block parts added by
// wave_ordered_sum. The last block: the loss.
__global__ void __launch_bounds__(256) k_reduce_adam(const AdamArgs a) {
  const int bid = blockIdx.x;
  if (bid < kWeightBlocks) {
    const int64_t t = ((int64_t)bid * 256 + threadIdx.x) * 4;
    if (t >= wb_count()) return;
    int l = 0;
    while (l + 1 < kLayers && t >= wb_offset(l + 1)) ++l;
    const int64_t e = t - wb_offset(l);
    const int n_in = in_dim(l), n_out = out_dim(l);
    const int64_t n = (int64_t)n_out * n_in;
    const float4 *p = reinterpret_cast<const float4 *>(a.ws + (int64_t)a.splits * wb_offset(l) + e);
    const int64_t i = w_offset(l) + e;  // a multiple of 4: the four elements are one 16-byte word
    // the parameter and its moments, then every slice's partial, are loaded
    // before the first addition (slices past the count read the last one
    // again and are not added)
    float4 th4 = *reinterpret_cast<const float4 *>(a.theta + i);
    float4 m4 = *reinterpret_cast<const float4 *>(a.m + i), v4 = *reinterpret_cast<const float4 *>(a.v + i);
    float4 v[kWgradSplits];
#pragma unroll
    for (int q = 0; q < kWgradSplits; ++q) v[q] = p[min(q, a.splits - 1) * (n / 4)];
    float4 g = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int q = 0; q < kWgradSplits; ++q)
      if (q < a.splits) g.x += v[q].x, g.y += v[q].y, g.z += v[q].z, g.w += v[q].w;
    *reinterpret_cast<float4 *>(a.grad + i) = g;
    if (a.adam) {
      adam_update(a, g.x, th4.x, m4.x, v4.x);
      adam_update(a, g.y, th4.y, m4.y, v4.y);
      adam_update(a, g.z, th4.z, m4.z, v4.z);
      adam_update(a, g.w, th4.w, m4.w, v4.w);
      *reinterpret_cast<float4 *>(a.m + i) = m4;
      *reinterpret_cast<float4 *>(a.v + i) = v4;
      *reinterpret_cast<float4 *>(a.theta + i) = th4;
      const float th[4] = {th4.x, th4.y, th4.z, th4.w};
      const uint16_t h[4] = {f2bf(th[0]), f2bf(th[1]), f2bf(th[2]), f2bf(th[3])};
      const int o = (int)(e / n_in), c = (int)(e % n_in);  // c % 4 == 0: the four share one lane's 8 columns
      *reinterpret_cast<uint2 *>(a.wb + wb_offset(l) + frag_offset(o, c, n_in)) =
          make_uint2(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16));
#pragma unroll
      for (int k = 0; k < 4; ++k) a.wt[wb_offset(l) + frag_offset(c + k, o, n_out)] = h[k];
    }
  } else if (bid < kWeightBlocks + kBiasBlocks) {
    const int j = (bid - kWeightBlocks) * 4 + (int)(threadIdx.x >> 6);
    const int l = j < 4 * kHidden ? j / kHidden : 4, f = j < 4 * kHidden ? j % kHidden : j - 4 * kHidden;
    const int64_t i = b_offset(l) + f;
    // the parameter and its moments are loaded before the parts, so both
    // wait for one round trip
    float th = a.theta[i], m = a.m[i], v = a.v[i];
    const float g = wave_ordered_sum(a.col_part + (int64_t)j * a.n_blocks, a.n_blocks, 1);
    if ((threadIdx.x & 63) == 0) {
      a.grad[i] = g;
      if (a.adam) {
        adam_update(a, g, th, m, v);
        a.m[i] = m;
        a.v[i] = v;
        a.theta[i] = th;
      }
    }
  } else if (threadIdx.x < 64) {
    const double sum = wave_ordered_sum(a.loss_part, a.n_blocks, 1);
    if (threadIdx.x == 0) {
      *a.loss_sum = sum;
      if (a.loss_epoch) *a.loss_epoch += sum;
    }
  }
}

// bf16 copies of every weight matrix: W (out x in) and W^T (in x out),
// tile-major.
__global__ void k_pack_weights(const float *theta, uint16_t *wb, uint16_t *wt) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= wb_count()) return;
  int l = 0;
  while (l + 1 < kLayers && t >= wb_offset(l + 1)) ++l;
  const int64_t e = t - wb_offset(l);
  const int n_in = in_dim(l), n_out = out_dim(l);
  const int o = (int)(e / n_in), i = (int)(e % n_in);
  const uint16_t h = f2bf(theta[w_offset(l) + e]);
  wb[wb_offset(l) + frag_offset(o, i, n_in)] = h;
  wt[wb_offset(l) + frag_offset(i, o, n_out)] = h;
}

__global__ void k_zero_f32(float *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

__global__ void k_zero_f64(double *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// Training labels from Monte Carlo hits, per (source, module) pair: hit
// count k, and the count, sum and sum of logs of the delays
// t - t0 - max(R - L/2 - r, 0) n_g / c (+ 0.01 ns), R the distance from
// the segment centre to the module centre. The delay is non-negative: no
// photon reaches the module surface sooner. The two sums are accumulated as
// 64-bit fixed point (delays in units of 2^-20 ns, logarithms in units of
// 2^-32), whose additions are exact, so the labels do not depend on the
// order in which the hits arrive.
__global__ void k_labels(const pp::DevHit *hits, const unsigned long long *hit_count, uint64_t cap,
                         const int32_t *event_to_source, uint32_t n_events, const pp::DevSource *sources,
                         const float4 *doms, int n_doms, float radius, float time_per_m,
                         const int32_t *row_of_pair, float *k, float *n_t, unsigned long long *s1q,
                         unsigned long long *s2q) {
  uint64_t n = *hit_count;
  if (n > cap) n = cap;
  for (uint64_t h = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; h < n; h += (uint64_t)gridDim.x * blockDim.x) {
    const pp::DevHit hit = hits[h];
    if (hit.event_id >= n_events || hit.dom_id >= (uint32_t)n_doms) continue;
    const int i = event_to_source[hit.event_id];
    if (i < 0) continue;
    const pp::DevSource &S = sources[i];
    const float4 m = doms[hit.dom_id];
    const float half = 0.5f * S.dir_len.w;
    const float dx = m.x - (S.pos_t0.x + half * S.dir_len.x), dy = m.y - (S.pos_t0.y + half * S.dir_len.y);
    const float dz = m.z - (S.pos_t0.z + half * S.dir_len.z);
    const float R = sqrtf(dx * dx + dy * dy + dz * dz);
    const float delay = fmaxf(hit.time_ns - S.pos_t0.w - fmaxf(R - half - radius, 0.0f) * time_per_m, 0.0f) + 0.01f;
    const int64_t pair = (int64_t)i * n_doms + hit.dom_id;
    const int64_t row = row_of_pair ? (int64_t)row_of_pair[pair] : pair;
    if (row < 0) continue;  // pair not in the training set
    atomicAdd(&k[row], 1.0f);  // whole numbers below 2^24: exact in any order
    atomicAdd(&n_t[row], 1.0f);
    atomicAdd(&s1q[row], (unsigned long long)__double2ll_rn((double)delay * kDelayFix));
    atomicAdd(&s2q[row], (unsigned long long)__double2ll_rn((double)logf(delay) * kLogFix));
  }
}

// Fixed-point label sums to float.
__global__ void k_labels_finish(const unsigned long long *s1q, const unsigned long long *s2q, float *s1, float *s2,
                                int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    s1[i] = (float)((double)(long long)s1q[i] / kDelayFix);
    s2[i] = (float)((double)(long long)s2q[i] / kLogFix);
  }
}

// ---------------------------------------------------------------------------
// Fused inference. A workgroup of four wavefronts owns kFusedRows = 128 pairs:
// it computes their features into LDS, then runs every layer as
// H_out^T = W H_in^T on the matrix cores (W from L2 as the A operand, the
// activations from LDS as the B operand), so a lane's accumulator holds four
// consecutive output features of one pair and is written back to the pair's
// LDS row as one 8-byte store. Wavefront w computes features 64 w .. + 64 of
// all 128 pairs: 4 x 8 tiles of 16 x 16. Layers overwrite their input in
// place, so a barrier separates the reads of a layer from its writes. The
// 68 KB of LDS per workgroup let two workgroups share a CU, so one runs its
// matrix products while the other runs its GELU epilogue. The last layer's
// first output gives the expected hits, which go to the per-module sums with
// one atomic per pair.


__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  const f32x2 v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));  // v_cvt_pk_bf16_f32, round to nearest even
}

template <int K, int LDW>
__device__ __forceinline__ void fused_hidden_layer(uint16_t *lds_h, const uint16_t *__restrict__ w,
                                                   const float *__restrict__ bias, const uint32_t *cdf, int lane,
                                                   int wave) {
  const int fg = wave;
  const int l16 = lane & 15, kq = (lane >> 4) * 8;
  const uint16_t *wfrag = w + lane * 8;  // + 512 (tile index): this lane's 16 bytes of a tile
  const uint16_t *hrow = lds_h + l16 * kFusedLd + kq;
  // the accumulators start at the biases (a lane's four values are features
  // f0 .. f0 + 3 of one pair), which saves the epilogue an addition per value
  f32x4 acc[4][8];
#pragma unroll
  for (int ft = 0; ft < 4; ++ft) {
    const float4 b = *reinterpret_cast<const float4 *>(bias + fg * 64 + ft * 16 + 4 * (lane >> 4));
#pragma unroll
    for (int pt = 0; pt < 8; ++pt) acc[ft][pt] = f32x4{b.x, b.y, b.z, b.w};
  }
#pragma unroll 2  // two K steps in flight fit the 256-register budget of 2 waves per SIMD without spills
  for (int k = 0; k < K; k += 32) {
    bf16x8 wa[4], hb[8];
#pragma unroll
    for (int ft = 0; ft < 4; ++ft) wa[ft] = load8(wfrag + ((fg * 4 + ft) * (LDW / 32) + k / 32) * 512);
#pragma unroll
    for (int pt = 0; pt < 8; ++pt) hb[pt] = lds_load8(hrow + pt * 16 * kFusedLd + k);
#pragma unroll
    for (int ft = 0; ft < 4; ++ft)
#pragma unroll
      for (int pt = 0; pt < 8; ++pt)
        acc[ft][pt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[ft], hb[pt], acc[ft][pt], 0, 0, 0);
  }
  __syncthreads();  // every wavefront has read the layer's input
#pragma unroll
  for (int ft = 0; ft < 4; ++ft) {
    const int f0 = fg * 64 + ft * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int pt = 0; pt < 8; ++pt) {
      const f32x4 v = acc[ft][pt];
      const uint2 h = make_uint2(pack_bf16(gelu_table(v[0], cdf), gelu_table(v[1], cdf)),
                                 pack_bf16(gelu_table(v[2], cdf), gelu_table(v[3], cdf)));
      *reinterpret_cast<uint2 *>(lds_h + (pt * 16 + l16) * kFusedLd + f0) = h;
    }
  }
  __syncthreads();  // the layer's output is complete
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_infer_fused(const FusedArgs a) {
  extern __shared__ __align__(16) uint16_t lds_h[];  // kFusedRows x kFusedLd bf16, then scale and module id
  float *s_scale = reinterpret_cast<float *>(lds_h + kFusedRows * kFusedLd);
  int *s_dom = reinterpret_cast<int *>(s_scale + kFusedRows);
  uint32_t *s_cdf = reinterpret_cast<uint32_t *>(s_dom + kFusedRows);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t q0 = (int64_t)blockIdx.x * kFusedRows;

  // the GELU table, then features: one pair per thread of the first half;
  // input columns kInReal..31 are zero
  for (int i = tid; i <= kCdfN; i += blockDim.x) s_cdf[i] = kCdfTableHalf[i];
  if (tid < kFusedRows) {
    float x[kInReal];
#pragma unroll
    for (int q = 0; q < kInReal; ++q) x[q] = 0.0f;
    float mub = 0.0f, nph = 0.0f, R = 0.0f;
    int dom = -1;
    if (q0 + tid < a.f.n_pairs) pair_features(a.f, a.f.first_pair + q0 + tid, x, mub, nph, R, dom);
    if (R * R > a.cut2) mub = 0.0f;  // beyond the cut: no light, the pair's expectation is 0
    static_assert(kInReal <= 32, "the first layer reads one K step of 32 inputs");
    uint32_t w[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
      w[q] = pack_bf16(2 * q < kInReal ? x[2 * q] : 0.0f, 2 * q + 1 < kInReal ? x[2 * q + 1] : 0.0f);
    uint4 *row = reinterpret_cast<uint4 *>(lds_h + tid * kFusedLd);
#pragma unroll
    for (int q = 0; q < 4; ++q) row[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
    s_scale[tid] = nph * mub;
    s_dom[tid] = dom;
  }
  // A tile with no pair inside the cut skips the network: its pairs expect 0.
  const bool live = tid < kFusedRows && s_scale[tid] > 0.0f;
  if (!__syncthreads_or(live)) {
    if (a.pair_mu && tid < kFusedRows && s_dom[tid] >= 0) a.pair_mu[q0 + tid] = 0.0f;
    return;
  }

  fused_hidden_layer<32, kInPad>(lds_h, a.w[0], a.b[0], s_cdf, lane, wave);  // kInReal real inputs: one K step
  fused_hidden_layer<kHidden, kHidden>(lds_h, a.w[1], a.b[1], s_cdf, lane, wave);
  fused_hidden_layer<kHidden, kHidden>(lds_h, a.w[2], a.b[2], s_cdf, lane, wave);
  fused_hidden_layer<kHidden, kHidden>(lds_h, a.w[3], a.b[3], s_cdf, lane, wave);

  // output layer, first output only: W4 rows 0..15 against pair tiles 2w and 2w + 1
  const int l16 = lane & 15, kq = (lane >> 4) * 8;
  const uint16_t *wfrag = a.w[4] + lane * 8;  // tile 0: rows 0..15
  const uint16_t *h0 = lds_h + (2 * wave * 16 + l16) * kFusedLd + kq;
  const uint16_t *h1 = h0 + 16 * kFusedLd;
  f32x4 o0 = {0, 0, 0, 0}, o1 = o0;
#pragma unroll
  for (int k = 0; k < kHidden; k += 32) {
    const bf16x8 wa = load8(wfrag + (k / 32) * 512);
    o0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, lds_load8(h0 + k), o0, 0, 0, 0);
    o1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, lds_load8(h1 + k), o1, 0, 0, 0);
  }
  if (lane < 16) {  // row 0 of the output tile (feature 0) lives in lanes 0..15, element 0
    const float b = a.b[4][0];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int pr = (2 * wave + j) * 16 + lane;
      const int d = s_dom[pr];
      if (d >= 0) {
        const float sc = s_scale[pr];
        const float mu = sc > 0.0f ? sc * expf((j ? o1[0] : o0[0]) + b) : 0.0f;
        if (a.dom_sums) atomicAdd(&a.dom_sums[d], (double)mu);
        if (a.pair_mu) a.pair_mu[q0 + pr] = mu;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Training, row pass. A workgroup of eight wavefronts owns kTrainRows = 32
// rows of the minibatch and keeps their activations in LDS through the
// forward and the backward pass, computed transposed as in inference
// (wavefront w: features 32 w .. + 32 of all 32 rows, 2 x 2 MFMA tiles; two
// wavefronts per SIMD, so one's memory waits overlap the other's work):
//   forward  H_l^T = GELU(W_l H_{l-1}^T + b_l), GELU and its derivative
//            both from tables in LDS, the derivative kept in LDS as FP16
//            for the backward pass;
//   output   Y (first 16 outputs; three are used), then the loss and dY per
//            row;
//   backward dZ_{l-1}^T = (W_l^T dZ_l^T) * GELU'(Z_{l-1}), from dY down to
//            dZ_0.
// Each layer's weight fragments are loaded into VGPRs two layers ahead
// (two fragment sets alternate), from the tile-major bf16 copies, so a
// wavefront's fragment load reads 1 KB contiguous; the barriers order LDS
// only, so those loads stay in flight across them. Layers alternate between
// two activation buffers (a layer reads one and writes the other), so one
// barrier per layer suffices: the buffer a layer writes was last read two
// layers before, ahead of the previous layer's barrier. After each layer the
// workgroup copies the layer's output from LDS to its block of a
// row-block-major global array, where the weight-gradient pass reads it;
// the copies of dY and dZ_l also sum each column over the 32 rows (the
// bias-gradient parts).
constexpr int kTrainThreads = 512;
constexpr int kWaveFeat = kHidden / (kTrainThreads / 64);  // output features per wavefront
constexpr int kFT = kWaveFeat / 16;                         // 16-feature MFMA tiles per wavefront

__device__ __forceinline__ uint32_t pack_f16(float lo, float hi) {
  typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  const f32x2 v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));  // round to nearest even
}

__device__ __forceinline__ float f16_half(uint32_t u, int hi) {
  const uint16_t h = (uint16_t)(hi ? u >> 16 : u);
  return (float)__builtin_bit_cast(_Float16, h);
}

__device__ __forceinline__ float bf_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// The wavefront's weight fragments of one layer: rows
// kWaveFeat w + 16 ft + lane % 16 of W (LDA elements per row),
// k = 32 s + 8 (lane / 16) .. + 8, s < S.
struct WFrags {
  bf16x8 v[kHidden / 32][kFT];
};

template <int S, int LDA>
__device__ __forceinline__ void load_w(WFrags &w, const uint16_t *__restrict__ W, int lane, int wave) {
  const uint16_t *wfrag = W + lane * 8;  // + 512 (tile index): this lane's 16 bytes of a tile
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int ft = 0; ft < kFT; ++ft) w.v[s][ft] = load8(wfrag + ((wave * kFT + ft) * (LDA / 32) + s) * 512);
}

// acc[ft][pt] = W[kWaveFeat w + 16 ft + .., k] . act[16 pt + .., k] over
// k < 32 S: the wavefront's output features against the workgroup's 32
// rows, the activations from LDS (ld_in elements per row).
template <int S>
__device__ __forceinline__ void rows_mma(f32x4 (&acc)[kFT][2], const WFrags &w, const uint16_t *s_in, int ld_in,
                                         int lane) {
  const uint16_t *hrow = s_in + (lane & 15) * ld_in + (lane >> 4) * 8;
#pragma unroll
  for (int ft = 0; ft < kFT; ++ft) acc[ft][0] = acc[ft][1] = f32x4{0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const bf16x8 h0 = lds_load8(hrow + s * 32), h1 = lds_load8(hrow + 16 * ld_in + s * 32);
#pragma unroll
    for (int ft = 0; ft < kFT; ++ft) {
      acc[ft][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.v[s][ft], h0, acc[ft][0], 0, 0, 0);
      acc[ft][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.v[s][ft], h1, acc[ft][1], 0, 0, 0);
    }
  }
}

// GELU(z) and GELU'(z) from the two tables interleaved in LDS as
// (Phi_i, dPhi_i, G_i, dG_i), float32: the map and interpolation of
// gelu_table().
__device__ __forceinline__ void gelu_and_grad(float z, const float4 *tab, float &h, float &g) {
  const float t = __builtin_amdgcn_fmed3f(__builtin_fmaf(z, kCdfA, kCdfB), 0.0f, (float)kCdfN);
  const float4 e = tab[(uint32_t)t];
  const float f = __builtin_amdgcn_fractf(t);
  h = z * __builtin_fmaf(f, e.y, e.x);
  g = __builtin_fmaf(f, e.w, e.z);
}

// Forward epilogue: z = acc + b (the layer's biases from LDS); GELU(z) as
// bf16 over the layer's input in s_act, GELU'(z) as FP16 into s_gp. A lane
// holds features f0 .. f0 + 3 of one row, written as one 8-byte store each.
__device__ __forceinline__ void fwd_epilogue(const f32x4 (&acc)[kFT][2], const float *s_b, const float4 *tab,
                                             uint16_t *s_act, uint16_t *s_gp, int lane, int wave) {
  const int l16 = lane & 15;
#pragma unroll
  for (int ft = 0; ft < kFT; ++ft) {
    const int f0 = wave * kWaveFeat + ft * 16 + 4 * (lane >> 4);
    const float4 b = *reinterpret_cast<const float4 *>(s_b + f0);
#pragma unroll
    for (int pt = 0; pt < 2; ++pt) {
      const f32x4 v = acc[ft][pt];
      float h[4], g[4];
      gelu_and_grad(v[0] + b.x, tab, h[0], g[0]);
      gelu_and_grad(v[1] + b.y, tab, h[1], g[1]);
      gelu_and_grad(v[2] + b.z, tab, h[2], g[2]);
      gelu_and_grad(v[3] + b.w, tab, h[3], g[3]);
      const int o = (pt * 16 + l16) * kTrainLd + f0;
      *reinterpret_cast<uint2 *>(s_act + o) = make_uint2(pack_bf16(h[0], h[1]), pack_bf16(h[2], h[3]));
      *reinterpret_cast<uint2 *>(s_gp + o) = make_uint2(pack_f16(g[0], g[1]), pack_f16(g[2], g[3]));
    }
  }
}

// Backward epilogue: dZ = acc * GELU'(Z) (from s_gp), as bf16 into s_act.
__device__ __forceinline__ void bwd_epilogue(const f32x4 (&acc)[kFT][2], const uint16_t *s_gp, uint16_t *s_act,
                                             int lane, int wave) {
  const int l16 = lane & 15;
#pragma unroll
  for (int ft = 0; ft < kFT; ++ft) {
    const int f0 = wave * kWaveFeat + ft * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int pt = 0; pt < 2; ++pt) {
      const f32x4 v = acc[ft][pt];
      const int o = (pt * 16 + l16) * kTrainLd + f0;
      const uint2 g = *reinterpret_cast<const uint2 *>(s_gp + o);
      *reinterpret_cast<uint2 *>(s_act + o) =
          make_uint2(pack_bf16(v[0] * f16_half(g.x, 0), v[1] * f16_half(g.x, 1)),
                     pack_bf16(v[2] * f16_half(g.y, 0), v[3] * f16_half(g.y, 1)));
    }
  }
}

// Copies the workgroup's kTrainRows x n_cols bf16 tile in LDS (ld elements
// per row) to its block of the row-block-major dst: column c of row block
// blk at dst + (blk n_cols + c) kTrainRows, the 32 rows contiguous. Four
// consecutive lanes share a pair of adjacent columns, each taking 8 rows:
// eight 4-byte LDS reads (both columns of a row), byte permutes into the
// two columns' 8-row words, and one 16-byte store per column, so a
// wavefront's two stores cover 2 KB contiguous. Lanes of parts 2 and 3 read
// their rows in an order rotated by four, which puts the four parts' reads
// in different LDS banks. If col_sum is not null it also gets each column's
// sum over the rows, column c's at col_sum[c cs_stride]: each lane adds its
// 8 rows in order, then the four lanes combine pairwise.
__device__ __forceinline__ void store_columns(const uint16_t *s, int ld, int n_cols, uint16_t *dst, int blk,
                                              float *col_sum, int cs_stride) {
  static_assert(kTrainRows == 32, "four lanes of 8 rows per column pair");
  const int part = threadIdx.x & 3;
  const int rot = 4 * (part >> 1);  // rows read in a rotated order, so the four parts hit different banks
#pragma unroll
  for (int c0 = 0; c0 < kHidden; c0 += 2 * (kTrainThreads / 4)) {
    const int c = c0 + 2 * (int)(threadIdx.x >> 2);
    if (c0 >= n_cols) break;  // uniform
    const bool live = c < n_cols;
    uint32_t x[8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
      x[r] = live ? *reinterpret_cast<const uint32_t *>(s + (8 * part + ((r + rot) & 7)) * ld + c) : 0u;
    // y[m]: rows (2m + rot) & 7 and the next, low halves (column c) and high halves (column c + 1)
    uint32_t ylo[4], yhi[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      ylo[m] = __builtin_amdgcn_perm(x[2 * m + 1], x[2 * m], 0x05040100u);
      yhi[m] = __builtin_amdgcn_perm(x[2 * m + 1], x[2 * m], 0x07060302u);
    }
    uint32_t wl[4], wh[4];
    // word k (rows 2k, 2k + 1) is y[(k + rot / 2) & 3]
    const bool sw = rot != 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      wl[k] = sw ? ylo[(k + 2) & 3] : ylo[k];
      wh[k] = sw ? yhi[(k + 2) & 3] : yhi[k];
    }
    if (live) {
      *reinterpret_cast<uint4 *>(dst + ((int64_t)blk * n_cols + c) * kTrainRows + 8 * part) =
          make_uint4(wl[0], wl[1], wl[2], wl[3]);
      *reinterpret_cast<uint4 *>(dst + ((int64_t)blk * n_cols + c + 1) * kTrainRows + 8 * part) =
          make_uint4(wh[0], wh[1], wh[2], wh[3]);
    }
    if (col_sum) {
      float sl = 0.0f, sh = 0.0f;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        sl += bf_to_f((uint16_t)wl[k]);
        sl += bf_to_f((uint16_t)(wl[k] >> 16));
        sh += bf_to_f((uint16_t)wh[k]);
        sh += bf_to_f((uint16_t)(wh[k] >> 16));
      }
      sl += __shfl_xor(sl, 1, 64);
      sl += __shfl_xor(sl, 2, 64);
      sh += __shfl_xor(sh, 1, 64);
      sh += __shfl_xor(sh, 2, 64);
      if (live && part == 0) col_sum[(int64_t)c * cs_stride] = sl, col_sum[(int64_t)(c + 1) * cs_stride] = sh;
    }
  }
}

__global__ void __launch_bounds__(kTrainThreads) k_train_rows(const TrainArgs a) {
  extern __shared__ __align__(16) uint16_t lds[];
  float4 *s_tab = reinterpret_cast<float4 *>(lds);                      // kCdfN + 1 table entries
  uint16_t *s_act = lds + (kCdfN + 1) * 8;                               // kTrainRows x kTrainLd bf16
  uint16_t *s_act2 = s_act + kTrainRows * kTrainLd;                      // the other activation buffer
  uint16_t *s_gp = s_act2 + kTrainRows * kTrainLd;                       // 4 layers x kTrainRows x kTrainLd FP16
  uint16_t *s_dy = s_gp + 4 * kTrainRows * kTrainLd;                     // kTrainRows x kDyLd bf16
  float *s_lab = reinterpret_cast<float *>(s_dy + kTrainRows * kDyLd);   // kTrainRows x 8
  double *s_loss = reinterpret_cast<double *>(s_lab + kTrainRows * 8);  // kTrainRows
  float *s_bias = reinterpret_cast<float *>(s_loss + kTrainRows);        // 4 x kHidden hidden biases, kOutPad output
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int blk = blockIdx.x;
  const int64_t i0 = (int64_t)blk * kTrainRows;
  const int nb = a.M / kTrainRows;           // row blocks: the bias parts of column c are col_part[c nb ..]
  float *col_part = a.col_part + blk;
  constexpr int kLayerLds = kTrainRows * kTrainLd;
  constexpr int kS = kHidden / 32, kS0 = kInPad / 32, kSOut = kOutPad / 32;
  static_assert(kS0 <= kS && kSOut <= kS, "weight fragments fit the hidden layers' buffer");

  // Loads in the order they are needed: the rows and labels, the tables and
  // biases (then copied to LDS), and last the first two layers' weights, so
  // that waiting for the rows does not wait for the weights as well (loads
  // complete in issue order).
  uint4 xrow = make_uint4(0, 0, 0, 0);
  float lab = 0.0f;
  const int gr = tid >> 3, gc = tid & 7;  // gather: row, 16-byte chunk of its 64 features (and label gc)
  if (tid < kTrainRows * 8 && i0 + gr < a.count) {
    const uint64_t p = (a.mul * (uint64_t)(a.first + i0 + gr) + a.add) % a.P;
    xrow = *reinterpret_cast<const uint4 *>(a.X + p * kInPad + gc * 8);
    switch (gc) {
      case 0: lab = a.mu_base[p]; break;
      case 1: lab = a.nph[p]; break;
      case 2: lab = a.k[p]; break;
      case 3: lab = a.n_t[p]; break;
      case 4: lab = a.s1[p]; break;
      case 5: lab = a.s2[p]; break;
      case 6: lab = a.w ? a.w[p] : 1.0f; break;
      default: break;
    }
  }
  float2 cdf[3], grad[3];
  float bias[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int q = tid + k * kTrainThreads;
    if (q <= kCdfN) cdf[k] = kCdfTable[q], grad[k] = kGeluGradTable[q];
    if (q < 4 * kHidden + kOutPad) bias[k] = q < 4 * kHidden ? a.b[q / kHidden][q % kHidden] : a.b[4][q - 4 * kHidden];
  }
  // two fragment sets: each layer's weights are loaded two layers ahead
  WFrags fa, fb;
  load_w<kS0, kInPad>(fa, a.wb[0], lane, wave);
  load_w<kS, kHidden>(fb, a.wb[1], lane, wave);
  if (tid < kTrainRows * 8) {
    *reinterpret_cast<uint4 *>(s_act + gr * kTrainLd + gc * 8) = xrow;
    s_lab[gr * 8 + gc] = lab;
  }
  for (int q = tid; q < kTrainRows * kDyLd / 8; q += kTrainThreads)
    reinterpret_cast<uint4 *>(s_dy)[q] = make_uint4(0, 0, 0, 0);
  // the biases live in LDS: a global load in an epilogue would make its
  // wait cover the weight loads issued before it as well
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int q = tid + k * kTrainThreads;
    if (q <= kCdfN) s_tab[q] = make_float4(cdf[k].x, cdf[k].y, grad[k].x, grad[k].y);
    if (q < 4 * kHidden + kOutPad) s_bias[q] = bias[k];
  }
  static_assert(3 * kTrainThreads > kCdfN && 3 * kTrainThreads >= 4 * kHidden + kOutPad, "three rounds cover both");
  lds_barrier();
  store_columns(s_act, kTrainLd, kInPad, a.XT, blk, nullptr, 0);

  // forward
  f32x4 acc[kFT][2];
  rows_mma<kS0>(acc, fa, s_act, kTrainLd, lane);
  load_w<kS, kHidden>(fa, a.wb[2], lane, wave);
  fwd_epilogue(acc, s_bias, s_tab, s_act2, s_gp, lane, wave);
  lds_barrier();  // the layer's output is complete
  store_columns(s_act2, kTrainLd, kHidden, a.HT[0], blk, nullptr, 0);
  rows_mma<kS>(acc, fb, s_act2, kTrainLd, lane);
  load_w<kS, kHidden>(fb, a.wb[3], lane, wave);
  fwd_epilogue(acc, s_bias + kHidden, s_tab, s_act, s_gp + kLayerLds, lane, wave);
  lds_barrier();
  store_columns(s_act, kTrainLd, kHidden, a.HT[1], blk, nullptr, 0);
  rows_mma<kS>(acc, fa, s_act, kTrainLd, lane);
  load_w<kSOut, kOutPad>(fa, a.wt[4], lane, wave);  // the first backward product
  if (wave < 2) {  // and the output layer's (W4 rows 0..15, tile 0) in the set's free slots
    static_assert(kSOut <= 2 && kFT == 2 && kS == 8, "eight output fragments fit slots 2..7 x 2");
#pragma unroll
    for (int s = 0; s < kS; ++s) fa.v[2 + s / 2][s % 2] = load8(a.wb[4] + lane * 8 + s * 512);
  }
  fwd_epilogue(acc, s_bias + 2 * kHidden, s_tab, s_act2, s_gp + 2 * kLayerLds, lane, wave);
  lds_barrier();
  store_columns(s_act2, kTrainLd, kHidden, a.HT[2], blk, nullptr, 0);
  rows_mma<kS>(acc, fb, s_act2, kTrainLd, lane);
  load_w<kS, kHidden>(fb, a.wt[3], lane, wave);
  fwd_epilogue(acc, s_bias + 3 * kHidden, s_tab, s_act, s_gp + 3 * kLayerLds, lane, wave);
  lds_barrier();
  store_columns(s_act, kTrainLd, kHidden, a.HT[3], blk, nullptr, 0);

  // output layer (outputs 0..15 of W4) for rows 16 w .. + 16, w = 0, 1; lane
  // l < 16 then holds outputs 0..3 of row 16 w + l and takes its loss
  if (wave < 2) {
    const int l16 = lane & 15, kq = (lane >> 4) * 8;
    const uint16_t *hrow = s_act + (wave * 16 + l16) * kTrainLd + kq;
    f32x4 o = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < kS; ++s)
      o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa.v[2 + s / 2][s % 2], lds_load8(hrow + s * 32), o, 0, 0, 0);
    if (lane < 16) {
      const int r = wave * 16 + lane;
      const float *L = s_lab + r * 8;
      RowLoss q{0.0, 0.0f, 0.0f, 0.0f};
      if (i0 + r < a.count)
        q = row_loss(o[0] + s_bias[4 * kHidden], o[1] + s_bias[4 * kHidden + 1], o[2] + s_bias[4 * kHidden + 2],
                     L[0], L[1], L[2], L[3], L[4], L[5], L[6], a.inv_norm);
      s_loss[r] = q.part;
      *reinterpret_cast<uint2 *>(s_dy + r * kDyLd) = make_uint2(pack_bf16(q.g0, q.g1), pack_bf16(q.g2, 0.0f));
    }
  }
  lds_barrier();
  if (wave == 0) {  // the rows' losses summed by a fixed butterfly over lanes 0..31
    static_assert(kTrainRows == 32, "one loss per lane of half a wavefront");
    double sum = lane < kTrainRows ? s_loss[lane] : 0.0;
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    if (lane == 0) a.loss_part[blk] = sum;
  }
  store_columns(s_dy, kDyLd, kOutPad, a.dYT, blk, col_part + (int64_t)4 * kHidden * nb, nb);

  // backward; every read of H_2 in s_act2 happened before the last forward barrier
  rows_mma<kSOut>(acc, fa, s_dy, kDyLd, lane);  // dH_3^T = W_4^T dY^T
  load_w<kS, kHidden>(fa, a.wt[2], lane, wave);
  bwd_epilogue(acc, s_gp + 3 * kLayerLds, s_act2, lane, wave);
  lds_barrier();
  store_columns(s_act2, kTrainLd, kHidden, a.dZT[3], blk, col_part + (int64_t)3 * kHidden * nb, nb);
  rows_mma<kS>(acc, fb, s_act2, kTrainLd, lane);  // dH_2^T = W_3^T dZ_3^T
  load_w<kS, kHidden>(fb, a.wt[1], lane, wave);
  bwd_epilogue(acc, s_gp + 2 * kLayerLds, s_act, lane, wave);
  lds_barrier();
  store_columns(s_act, kTrainLd, kHidden, a.dZT[2], blk, col_part + (int64_t)2 * kHidden * nb, nb);
  rows_mma<kS>(acc, fa, s_act, kTrainLd, lane);  // dH_1^T = W_2^T dZ_2^T
  bwd_epilogue(acc, s_gp + kLayerLds, s_act2, lane, wave);
  lds_barrier();
  store_columns(s_act2, kTrainLd, kHidden, a.dZT[1], blk, col_part + (int64_t)kHidden * nb, nb);
  rows_mma<kS>(acc, fb, s_act2, kTrainLd, lane);  // dH_0^T = W_1^T dZ_1^T
  bwd_epilogue(acc, s_gp, s_act, lane, wave);
  lds_barrier();
  store_columns(s_act, kTrainLd, kHidden, a.dZT[0], blk, col_part, nb);
}

__global__ void k_zero_u64(unsigned long long *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

int blocks_for(int64_t n, int threads) { return (int)((n + threads - 1) / threads); }

}  // namespace

size_t train_lds_bytes() {
  return sizeof(float4) * (kCdfN + 1) + sizeof(uint16_t) * (6 * kTrainRows * kTrainLd + kTrainRows * kDyLd) +
         sizeof(float) * kTrainRows * 8 + sizeof(double) * kTrainRows + sizeof(float) * (4 * kHidden + kOutPad);
}

hipError_t launch_train_rows(const TrainArgs &a, hipStream_t s) {
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_train_rows),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     static_cast<int>(train_lds_bytes()));
  if (attr != hipSuccess) return attr;
  if (a.M <= 0 || a.M % 64 != 0 || a.count > a.M) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_train_rows, dim3((unsigned)(a.M / kTrainRows)), dim3(kTrainThreads), train_lds_bytes(), s, a);
  return hipGetLastError();
}

hipError_t launch_wgrad(const WgradArgs &g, hipStream_t s) {
  if (g.M <= 0 || g.M % kTrainRows != 0 || g.splits <= 0 || g.splits > g.M / kTrainRows) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_wgrad, dim3((unsigned)(wgrad_tile_offset(kLayers) * g.splits)), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_reduce_adam(const AdamArgs &a, hipStream_t s) {
  // the kernel reads slices 0 .. splits - 1 and holds at most kWgradSplits of them
  if (a.splits <= 0 || a.splits > kWgradSplits || a.n_blocks <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce_adam, dim3(kWeightBlocks + kBiasBlocks + 1), dim3(256), 0, s, a);
  return hipGetLastError();
}

size_t fused_lds_bytes() {
  return sizeof(uint16_t) * kFusedRows * kFusedLd + 2 * sizeof(float) * kFusedRows + sizeof(uint32_t) * (kCdfN + 1);
}

hipError_t launch_infer_fused(const FusedArgs &a, hipStream_t s) {
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_infer_fused),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     static_cast<int>(fused_lds_bytes()));
  if (attr != hipSuccess) return attr;
  if (a.f.n_pairs <= 0) return hipSuccess;
  const int64_t blocks = (a.f.n_pairs + kFusedRows - 1) / kFusedRows;
  hipLaunchKernelGGL(k_infer_fused, dim3(static_cast<uint32_t>(blocks)), dim3(256), fused_lds_bytes(), s, a);
  return hipGetLastError();
}

hipError_t launch_features(const FeatureArgs &f, hipStream_t s) {
  const int64_t rows = (f.n_pairs + kTile - 1) / kTile * kTile;
  hipLaunchKernelGGL(k_features, dim3(blocks_for(rows, 256)), dim3(256), 0, s, f, rows);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u64, dim3(min(blocks_for(n, 256), 4096)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_pack_weights(const float *theta, uint16_t *w_bf16, uint16_t *wt_bf16, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_weights, dim3(blocks_for(wb_count(), 256)), dim3(256), 0, s, theta, w_bf16, wt_bf16);
  return hipGetLastError();
}

hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_f32, dim3(min(blocks_for(n, 256), 4096)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_f64, dim3(min(blocks_for(n, 256), 4096)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_labels(const pp::DevHit *hits, const unsigned long long *hit_count, uint64_t hit_cap,
                         const int32_t *event_to_source, uint32_t n_events, const pp::DevSource *sources,
                         const float4 *doms, int n_doms, float radius, float time_per_m,
                         const int32_t *row_of_pair, float *k, float *n_t, unsigned long long *s1q,
                         unsigned long long *s2q, float *s1, float *s2, int64_t n_rows, hipStream_t s) {
  hipError_t e = launch_zero_u64(s1q, n_rows, s);
  if (e == hipSuccess) e = launch_zero_u64(s2q, n_rows, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_labels, dim3(1024), dim3(256), 0, s, hits, hit_count, hit_cap, event_to_source, n_events,
                     sources, doms, n_doms, radius, time_per_m, row_of_pair, k, n_t, s1q, s2q);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_labels_finish, dim3(min(blocks_for(n_rows, 256), 4096)), dim3(256), 0, s, s1q, s2q, s1, s2,
                     n_rows);
  return hipGetLastError();
}

// Training-pair selection, one workgroup of 256 per source. The counting
// pass writes the number of kept pairs of the source; the scatter pass
// writes them in module order from the source's first row on, using the
// wavefront ballot for the order within a wavefront and LDS for the order
// between wavefronts, so the row order does not depend on scheduling.
template <bool kScatter>
__global__ void __launch_bounds__(256) k_select(const SelectArgs a) {
  const int i = blockIdx.x;
  if (i >= a.n_sources) return;
  const pp::DevSource &S = a.sources[i];
  // explicit fmaf: both passes must take the same decision for every pair,
  // whatever the compiler would contract in either instantiation
  const float half = 0.5f * S.dir_len.w;
  const float cx = fmaf(half, S.dir_len.x, S.pos_t0.x), cy = fmaf(half, S.dir_len.y, S.pos_t0.y);
  const float cz = fmaf(half, S.dir_len.z, S.pos_t0.z);
  __shared__ uint32_t wave_kept[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t next_row = kScatter ? a.row_offset[i] : 0;
  uint32_t kept_total = 0;
  for (int j0 = 0; j0 < a.n_doms; j0 += 256) {
    const int j = j0 + (int)threadIdx.x;
    bool keep = false, near = false;
    if (j < a.n_doms) {
      const float4 m = a.doms[j];
      const float dx = m.x - cx, dy = m.y - cy, dz = m.z - cz;
      near = fmaf(dx, dx, fmaf(dy, dy, __fmul_rn(dz, dz))) <= a.near2;
      keep = near || ((uint32_t)j + (uint32_t)i) % a.far_stride == 0u;
    }
    const uint64_t ballot = __ballot(keep);
    if (lane == 0) wave_kept[wave] = (uint32_t)__popcll(ballot);
    __syncthreads();
    uint32_t before = 0, chunk = 0;
    for (int q = 0; q < 4; ++q) {
      before += q < wave ? wave_kept[q] : 0u;
      chunk += wave_kept[q];
    }
    if (kScatter && j < a.n_doms) {
      const int64_t pair = (int64_t)i * a.n_doms + j;
      const int64_t row = next_row + before + (uint32_t)__popcll(ballot & ((1ull << lane) - 1ull));
      if (keep && row < a.n_rows) {
        a.pair_of_row[row] = pair;
        a.w[row] = near ? 1.0f : (float)a.far_stride;
        a.row_of_pair[pair] = (int32_t)row;
      } else {
        a.row_of_pair[pair] = -1;
      }
    }
    next_row += chunk;
    kept_total += chunk;
    __syncthreads();  // wave_kept is rewritten by the next chunk
  }
  if (!kScatter && threadIdx.x == 0) a.count[i] = kept_total;
}

hipError_t launch_select(const SelectArgs &a, bool scatter, hipStream_t s) {
  if (a.n_sources <= 0) return hipSuccess;
  if (scatter)
    hipLaunchKernelGGL(k_select<true>, dim3(a.n_sources), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_select<false>, dim3(a.n_sources), dim3(256), 0, s, a);
  return hipGetLastError();
}


}  // namespace sur

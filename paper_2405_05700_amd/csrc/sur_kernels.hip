// gfx950 kernels of the learned surrogate: a five-layer GELU perceptron in
// BF16 with FP32 accumulation on the matrix cores, its backward pass, loss,
// Adam, and the features / labels / reductions around it.
//
// GEMM: C[M x N] = A[M x K] * B[N x K]^T with both operands K-contiguous
// bf16. A workgroup of four wavefronts computes a 64 x 64 tile; each
// wavefront a 32 x 32 quarter as 2 x 2 v_mfma_f32_16x16x32_bf16 tiles. The
// weights (at most 128 KB per layer) stay in L2, so operand fragments are
// loaded straight into VGPRs, 16 bytes per lane per fragment. Epilogues fuse
// the bias, GELU and its derivative, the transposed copies the next GEMM
// needs, and split-K partials. Every sum that gradients or labels depend on
// is formed in a fixed order (partials reduced in order, or exact
// fixed-point atomics), so training is bit-reproducible.

#include "sur_device.h"
#include "gelu_cdf_table.h"

namespace sur {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 load8(const uint16_t *p) {
  const uint4 v = *reinterpret_cast<const uint4 *>(p);
  return __builtin_bit_cast(bf16x8, v);
}

// Standard normal CDF Phi(z) = erfc(-z / sqrt 2) / 2 from the rational
// approximation of Abramowitz & Stegun 7.1.26: for x >= 0,
// erfc(x) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2),
// t = 1 / (1 + p x), absolute error <= 1.5e-7 (far below the bf16 rounding
// of every stored activation). Also returns e = exp(-z^2 / 2), which the
// GELU derivative reuses.
__device__ __forceinline__ float norm_cdf(float z, float &e) {
  const float x = fabsf(z) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.3275911f, x, 1.0f));
  float q = __builtin_fmaf(t, 1.061405429f, -1.453152027f);
  q = __builtin_fmaf(t, q, 1.421413741f);
  q = __builtin_fmaf(t, q, -0.284496736f);
  q = __builtin_fmaf(t, q, 0.254829592f);
  e = __builtin_amdgcn_exp2f(z * z * -0.72134752044448170f);  // exp(-z^2 / 2) = 2^(-z^2 log2(e) / 2)
  const float lower = 0.5f * t * q * e;                       // Phi(-|z|)
  return z >= 0.0f ? 1.0f - lower : lower;
}

// GELU(z) = z Phi(z) = z / 2 + H(z^2) / 2 with H(u) = sqrt(u) erf(sqrt(u / 2)),
// an entire function of u: H / 2 is a degree-12 polynomial in
// x = min(u / 12.5 - 1, 1), which covers |z| <= 5; beyond, erf(|z| / sqrt 2)
// = 1 - O(6e-7) and H grows as |z|, added as max(|z| - 5, 0) / 2. The
// coefficients and the FP32 error bound (|error| <= 3.4e-6 for all z) come
// from gelu_poly.py beside this file. No transcendental and no branch:
// 19 full-rate operations, where the rational form of erfc needs a
// reciprocal and an exponential.
__device__ __forceinline__ float gelu(float z) {
  const float x = fminf(__builtin_fmaf(z * z, 0.08f, -1.0f), 1.0f);
  float h = -0.012713938f;
  h = __builtin_fmaf(h, x, 0.026097981f);
  h = __builtin_fmaf(h, x, -0.011562989f);
  h = __builtin_fmaf(h, x, 0.015651802f);
  h = __builtin_fmaf(h, x, -0.05995361f);
  h = __builtin_fmaf(h, x, 0.08401806f);
  h = __builtin_fmaf(h, x, -0.08555572f);
  h = __builtin_fmaf(h, x, 0.096760295f);
  h = __builtin_fmaf(h, x, -0.112569965f);
  h = __builtin_fmaf(h, x, 0.13914998f);
  h = __builtin_fmaf(h, x, -0.23469144f);
  h = __builtin_fmaf(h, x, 0.8883197f);
  h = __builtin_fmaf(h, x, 1.7670473f);
  h = __builtin_fmaf(0.5f, fmaxf(fabsf(z) - 5.0f, 0.0f), h);
  return __builtin_fmaf(0.5f, z, h);
}

// GELU for the fused inference kernel: z Phi(z) with Phi linear between the
// 1025 nodes of a table in LDS (gelu_table.py beside this file derives it
// and bounds the error: |error| <= 5.3e-6 for all z, 2^-12 relative where
// |GELU| > 0.01). Eight full-rate operations and one 8-byte LDS read, where
// the polynomial takes nineteen; t = N (z >= 6) lands on the last node,
// whose difference is 0, and a NaN converts to index 0.
__device__ __forceinline__ float gelu_table(float z, const float2 *cdf) {
  const float t = __builtin_amdgcn_fmed3f(__builtin_fmaf(z, kCdfA, kCdfB), 0.0f, (float)kCdfN);
  const float2 e = cdf[(uint32_t)t];
  return z * __builtin_fmaf(__builtin_amdgcn_fractf(t), e.y, e.x);
}

// Its derivative Phi(z) + z phi(z), from the rational form above.
__device__ __forceinline__ float gelu_grad(float z) {
  float e;
  const float cdf = norm_cdf(z, e);
  return __builtin_fmaf(z * e, 0.39894228040143268f, cdf);
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

template <int EPI>
__global__ void __launch_bounds__(256) k_gemm(const GemmArgs g) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = blockIdx.y * kTile + (wave >> 1) * 32;
  const int col0 = blockIdx.x * kTile + (wave & 1) * 32;
  const int kbeg = blockIdx.z * g.k_chunk;
  const int kend = min(g.K, kbeg + g.k_chunk);
  const int lr = lane & 15, lk = (lane >> 4) * 8;
  f32x4 acc00 = {0, 0, 0, 0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
  const uint16_t *a0 = g.A + (int64_t)(row0 + lr) * g.lda + lk;
  const uint16_t *a1 = a0 + 16 * g.lda;
  const uint16_t *b0 = g.B + (int64_t)(col0 + lr) * g.ldb + lk;
  const uint16_t *b1 = b0 + 16 * g.ldb;
  // The operands of step k + 32 are loaded before the products of step k,
  // so one step of loads is always in flight (the last step reloads its own
  // operands, which stay in bounds).
  bf16x8 va0 = load8(a0 + kbeg), va1 = load8(a1 + kbeg);
  bf16x8 vb0 = load8(b0 + kbeg), vb1 = load8(b1 + kbeg);
  for (int k = kbeg; k < kend; k += 32) {
    const int kn = k + 32 < kend ? k + 32 : k;
    const bf16x8 na0 = load8(a0 + kn), na1 = load8(a1 + kn);
    const bf16x8 nb0 = load8(b0 + kn), nb1 = load8(b1 + kn);
    acc00 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va0, vb0, acc00, 0, 0, 0);
    acc01 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va0, vb1, acc01, 0, 0, 0);
    acc10 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va1, vb0, acc10, 0, 0, 0);
    acc11 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va1, vb1, acc11, 0, 0, 0);
    va0 = na0, va1 = na1, vb0 = nb0, vb1 = nb1;
  }
  // Output layout of a 16 x 16 tile: lane holds rows 4 (lane / 16) + r,
  // r = 0..3, of column lane % 16.
  const f32x4 accs[4] = {acc00, acc01, acc10, acc11};
  float csum[2] = {0.0f, 0.0f};  // kEpiGeluBwd: this lane's part of the column sums of the wave's 32 rows
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int i = t >> 1, j = t & 1;
    const int col = col0 + j * 16 + lr;
    const int rbase = row0 + i * 16 + (lane >> 4) * 4;
    const f32x4 v = accs[t];
    if (EPI == kEpiGelu) {
      const float b = g.bias[col];
      uint16_t h[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float z = v[r] + b;
        const int64_t idx = (int64_t)(rbase + r) * g.N + col;
        if (g.Z) g.Z[idx] = z;
        h[r] = f2bf(gelu(z));
        g.H[idx] = h[r];
      }
      if (g.HT) {
        const uint2 packed = make_uint2(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16));
        *reinterpret_cast<uint2 *>(g.HT + (int64_t)col * g.ldt + rbase) = packed;
      }
    } else if (EPI == kEpiGeluBwd) {
      uint16_t h[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t idx = (int64_t)(rbase + r) * g.N + col;
        h[r] = f2bf(v[r] * gelu_grad(g.Zin[idx]));
        g.H[idx] = h[r];
        csum[j] += __uint_as_float((uint32_t)h[r] << 16);
      }
      const uint2 packed = make_uint2(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16));
      *reinterpret_cast<uint2 *>(g.HT + (int64_t)col * g.ldt + rbase) = packed;
    } else if (EPI == kEpiSplitK) {
      // this K slice's partial product; a reduction in slice order follows
      float *part = g.ws + (int64_t)blockIdx.z * g.M * g.N;
#pragma unroll
      for (int r = 0; r < 4; ++r) part[(int64_t)(rbase + r) * g.N + col] = v[r];
    } else if (EPI == kEpiLinear) {
      const float b = g.bias[col];
#pragma unroll
      for (int r = 0; r < 4; ++r) g.out[(int64_t)(rbase + r) * g.N + col] = v[r] + b;
    }
  }
  if (EPI == kEpiGeluBwd && g.col_part) {
    // lanes l, l + 16, l + 32, l + 48 hold the same column: sum them into
    // the column sum of the wave's 32 rows, stored for the block of rows
    // (a reduction over the row blocks in order follows)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      float cs = csum[j];
      cs += __shfl_xor(cs, 16, 64);
      cs += __shfl_xor(cs, 32, 64);
      if (lane < 16) g.col_part[(int64_t)(row0 / 32) * g.N + col0 + j * 16 + lane] = cs;
    }
  }
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
  const int i = (int)(p / f.n_doms), j = (int)(p % f.n_doms);
  const pp::DevSource &S = f.sources[i];
  const float4 m = f.doms[j];
  const float half = 0.5f * S.dir_len.w;
  const float cx = S.pos_t0.x + half * S.dir_len.x, cy = S.pos_t0.y + half * S.dir_len.y;
  const float cz = S.pos_t0.z + half * S.dir_len.z;
  const float dx = m.x - cx, dy = m.y - cy, dz = m.z - cz;
  R = fmaxf(sqrtf(dx * dx + dy * dy + dz * dz), 0.5f);
  const float ux = dx / R, uy = dy / R, uz = dz / R;
  const float cos_eta = ux * S.dir_len.x + uy * S.dir_len.y + uz * S.dir_len.z;
  const pp::DevLayer Ls = f.layers[layer_of(cz, f.z_lo, f.inv_dz, f.n_layers)];
  const pp::DevLayer Ld = f.layers[layer_of(m.z, f.z_lo, f.inv_dz, f.n_layers)];
  // Geometry up to a rotation about the vertical (the ice is layered in
  // depth only): vertical parts, horizontal and vertical offsets, distance,
  // angle to the track and the relative azimuth of the horizontal parts.
  const float h = S.dir_len.x * ux + S.dir_len.y * uy;
  const float hh = sqrtf((S.dir_len.x * S.dir_len.x + S.dir_len.y * S.dir_len.y) * (ux * ux + uy * uy));
  x[0] = uz;
  x[1] = sqrtf(dx * dx + dy * dy) / 100.0f;
  x[2] = dz / 100.0f;
  x[3] = R / 100.0f;
  x[4] = logf(R / 10.0f) / 3.0f;
  x[5] = cos_eta;
  x[6] = cos_eta - 0.75470958022277199f;  // cos 41 deg
  x[7] = S.dir_len.z;
  x[8] = h;
  x[9] = hh > 1e-9f ? fminf(fmaxf(h / hh, -1.0f), 1.0f) : 0.0f;
  x[10] = cz / 500.0f;
  x[11] = m.z / 500.0f;
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
  const float bimp = sqrtf(px * px + py * py + pz * pz);
  const float ex = vx - L * S.dir_len.x, ey = vy - L * S.dir_len.y, ez = vz - L * S.dir_len.z;
  x[16] = bimp / 100.0f;
  x[17] = (along - 0.5f * L) / 100.0f;
  x[18] = fminf(fmaxf((along - bimp / kTanCherenkov) / L, -1.0f), 2.0f);
  x[19] = sqrtf(vx * vx + vy * vy + vz * vz) / 100.0f;
  x[20] = sqrtf(ex * ex + ey * ey + ez * ez) / 100.0f;
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
  const float lam_e = 0.5f * (Ls.coef.w / Ls.hg.x + Ld.coef.w / Ld.hg.x);
  const float D = lam_e / 3.0f;
  const float dl = sqrtf(D * lam_a);
  mu_base = f.radius * f.radius * expf(-R / dl) / (4.0f * D * R);
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

// Poisson + gamma negative log-likelihood per row and its gradient with
// respect to the three outputs (log mu / mu_base, log kappa, log theta/tau0).
__global__ void __launch_bounds__(256) k_loss(const LossArgs l) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  double part = 0.0;
  float bsum[3] = {0.0f, 0.0f, 0.0f};
  if (m < l.M_pad) {
    float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
    if (m < l.M_real) {
      const float *y = l.Y + (int64_t)m * kOutPad;
      const float y1 = fminf(fmaxf(y[1], -8.0f), 8.0f), y2 = fminf(fmaxf(y[2], -8.0f), 8.0f);
      const float mu = l.nph[m] * l.mu_base[m] * expf(y[0]);
      const float kappa = expf(y1), theta = kTau0Ns * expf(y2);
      const float k = l.k[m], nt = l.n_t[m], s1 = l.s1[m], s2 = l.s2[m];
      const float log_mu = logf(mu);
      const float pois = mu - (k > 0.0f ? k * log_mu : 0.0f);
      const float gam = nt > 0.0f ? nt * (lgammaf(kappa) + kappa * logf(theta)) - (kappa - 1.0f) * s2 + s1 / theta
                                  : 0.0f;
      const float wt = l.w ? l.w[m] : 1.0f;
      part = (double)wt * ((double)pois + (double)kTimeWeight * gam);
      const float scale = wt * l.inv_norm;
      g0 = (mu - k) * scale;
      if (nt > 0.0f) {
        g1 = kTimeWeight * kappa * (nt * (digamma(kappa) + logf(theta)) - s2) * scale;
        g2 = kTimeWeight * (nt * kappa - s1 / theta) * scale;
        if (y[1] != y1) g1 = 0.0f;  // clamped: no gradient through the clamp
        if (y[2] != y2) g2 = 0.0f;
      }
    }
    uint16_t *row = l.dY + (int64_t)m * kOutPad;
    row[0] = f2bf(g0);
    row[1] = f2bf(g1);
    row[2] = f2bf(g2);
    for (int q = kOutReal; q < kOutPad; ++q) row[q] = 0;
    l.dYT[m] = f2bf(g0);
    l.dYT[(int64_t)l.M_pad + m] = f2bf(g1);
    l.dYT[2 * (int64_t)l.M_pad + m] = f2bf(g2);
    for (int q = kOutReal; q < kOutPad; ++q) l.dYT[(int64_t)q * l.M_pad + m] = 0;
    bsum[0] = __uint_as_float((uint32_t)row[0] << 16);
    bsum[1] = __uint_as_float((uint32_t)row[1] << 16);
    bsum[2] = __uint_as_float((uint32_t)row[2] << 16);
  }
  __shared__ double red[256];
  __shared__ float bred[3][256];
  red[threadIdx.x] = part;
  for (int q = 0; q < 3; ++q) bred[q][threadIdx.x] = bsum[q];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[threadIdx.x] += red[threadIdx.x + o];
      for (int q = 0; q < 3; ++q) bred[q][threadIdx.x] += bred[q][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    l.loss_part[blockIdx.x] = red[0];
    for (int q = 0; q < 3; ++q) l.bias_part[3 * blockIdx.x + q] = bred[q][0];
  }
}

// Sum of part[i * stride] over i < n in a fixed order by one wavefront: lane
// l adds parts l, l + 64, l + 128, ... in turn, then the lanes combine by a
// fixed butterfly. The result depends only on the values, not on
// scheduling, and the wave's loads are independent.
template <class T>
__device__ __forceinline__ T wave_ordered_sum(const T *part, int n, int64_t stride) {
  const int lane = threadIdx.x & 63;
  T sum = 0;
  for (int i = lane; i < n; i += 64) sum += part[(int64_t)i * stride];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
  return sum;
}

// The workgroups' loss and output-bias-gradient partials, summed in a fixed
// order: wavefront 0 the loss, wavefronts 1..3 the three bias entries.
__global__ void __launch_bounds__(256) k_loss_reduce(const LossArgs l, int n_blocks) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (wave == 0) {
    const double sum = wave_ordered_sum(l.loss_part, n_blocks, 1);
    if (lane == 0) {
      *l.loss_sum = sum;
      if (l.loss_epoch) *l.loss_epoch += sum;
    }
  } else if (l.out_bias_grad) {
    const float sum = wave_ordered_sum(l.bias_part + wave - 1, n_blocks, 3);
    if (lane == 0) l.out_bias_grad[wave - 1] = sum;
  }
}

// out[j] = sum over i < n_parts of part[i * stride + j], in order of i: one
// thread per element (few parts, many elements: the split-K slices).
__global__ void k_sum_parts(float *out, const float *part, int64_t n, int n_parts, int64_t stride) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    float sum = 0.0f;
#pragma unroll 8
    for (int i = 0; i < n_parts; ++i) sum += part[i * stride + j];
    out[j] = sum;
  }
}

// The same with one wavefront per element (many parts, few elements: the
// per-32-row column sums of a bias gradient).
__global__ void __launch_bounds__(256) k_sum_parts_wave(float *out, const float *part, int64_t n, int n_parts,
                                                        int64_t stride) {
  const int64_t j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  const float sum = wave_ordered_sum(part + j, n_parts, stride);
  if ((threadIdx.x & 63) == 0) out[j] = sum;
}

// Adam (Kingma & Ba) with bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void k_adam(float *theta, const float *grad, float *m, float *v, int64_t n, float lr, float c1,
                       float c2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// bf16 copies of every weight matrix: W (out x in) and W^T (in x out).
__global__ void k_pack_weights(const float *theta, uint16_t *wb, uint16_t *wt) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= wb_count()) return;
  int l = 0;
  while (l + 1 < kLayers && t >= wb_offset(l + 1)) ++l;
  const int64_t e = t - wb_offset(l);
  const int n_in = in_dim(l), n_out = out_dim(l);
  const int o = (int)(e / n_in), i = (int)(e % n_in);
  const uint16_t h = f2bf(theta[w_offset(l) + e]);
  wb[t] = h;
  wt[wb_offset(l) + (int64_t)i * n_out + o] = h;
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

__device__ __forceinline__ bf16x8 lds_load8(const uint16_t *p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(p));
}

__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  const f32x2 v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));  // v_cvt_pk_bf16_f32, round to nearest even
}

template <int K, int LDW>
__device__ __forceinline__ void fused_hidden_layer(uint16_t *lds_h, const uint16_t *__restrict__ w,
                                                   const float *__restrict__ bias, const float2 *cdf, int lane,
                                                   int wave) {
  const int fg = wave;
  const int l16 = lane & 15, kq = (lane >> 4) * 8;
  const uint16_t *wrow = w + (int64_t)(fg * 64 + l16) * LDW + kq;
  const uint16_t *hrow = lds_h + l16 * kFusedLd + kq;
  f32x4 acc[4][8];
#pragma unroll
  for (int ft = 0; ft < 4; ++ft)
#pragma unroll
    for (int pt = 0; pt < 8; ++pt) acc[ft][pt] = f32x4{0, 0, 0, 0};
#pragma unroll 2  // two K steps in flight fit the 256-register budget of 2 waves per SIMD without spills
  for (int k = 0; k < K; k += 32) {
    bf16x8 wa[4], hb[8];
#pragma unroll
    for (int ft = 0; ft < 4; ++ft) wa[ft] = load8(wrow + ft * 16 * LDW + k);
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
    const float b0 = bias[f0], b1 = bias[f0 + 1], b2 = bias[f0 + 2], b3 = bias[f0 + 3];
#pragma unroll
    for (int pt = 0; pt < 8; ++pt) {
      const f32x4 v = acc[ft][pt];
      const uint2 h = make_uint2(pack_bf16(gelu_table(v[0] + b0, cdf), gelu_table(v[1] + b1, cdf)),
                                 pack_bf16(gelu_table(v[2] + b2, cdf), gelu_table(v[3] + b3, cdf)));
      *reinterpret_cast<uint2 *>(lds_h + (pt * 16 + l16) * kFusedLd + f0) = h;
    }
  }
  __syncthreads();  // the layer's output is complete
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_infer_fused(const FusedArgs a) {
  extern __shared__ __align__(16) uint16_t lds_h[];  // kFusedRows x kFusedLd bf16, then scale and module id
  float *s_scale = reinterpret_cast<float *>(lds_h + kFusedRows * kFusedLd);
  int *s_dom = reinterpret_cast<int *>(s_scale + kFusedRows);
  float2 *s_cdf = reinterpret_cast<float2 *>(s_dom + kFusedRows);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t q0 = (int64_t)blockIdx.x * kFusedRows;

  // the GELU table, then features: one pair per thread of the first half;
  // input columns kInReal..31 are zero
  for (int i = tid; i <= kCdfN; i += blockDim.x) s_cdf[i] = kCdfTable[i];
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
  const uint16_t *wrow = a.w[4] + (int64_t)l16 * kHidden + kq;
  const uint16_t *h0 = lds_h + (2 * wave * 16 + l16) * kFusedLd + kq;
  const uint16_t *h1 = h0 + 16 * kFusedLd;
  f32x4 o0 = {0, 0, 0, 0}, o1 = o0;
#pragma unroll
  for (int k = 0; k < kHidden; k += 32) {
    const bf16x8 wa = load8(wrow + k);
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

__global__ void k_zero_u64(unsigned long long *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

int blocks_for(int64_t n, int threads) { return (int)((n + threads - 1) / threads); }

}  // namespace

hipError_t launch_sum_parts(float *out, const float *part, int64_t n, int n_parts, int64_t stride, hipStream_t s) {
  if (n_parts > 32 && n <= 65536)
    hipLaunchKernelGGL(k_sum_parts_wave, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, out, part, n, n_parts, stride);
  else
    hipLaunchKernelGGL(k_sum_parts, dim3(min(blocks_for(n, 256), 2048)), dim3(256), 0, s, out, part, n, n_parts,
                       stride);
  return hipGetLastError();
}

hipError_t launch_gemm(int epi, const GemmArgs &g, int splits, hipStream_t s) {
  const dim3 grid(g.N / kTile, g.M / kTile, splits);
  switch (epi) {
    case kEpiGelu: hipLaunchKernelGGL(k_gemm<kEpiGelu>, grid, dim3(256), 0, s, g); break;
    case kEpiGeluBwd: hipLaunchKernelGGL(k_gemm<kEpiGeluBwd>, grid, dim3(256), 0, s, g); break;
    case kEpiSplitK: hipLaunchKernelGGL(k_gemm<kEpiSplitK>, grid, dim3(256), 0, s, g); break;
    case kEpiLinear: hipLaunchKernelGGL(k_gemm<kEpiLinear>, grid, dim3(256), 0, s, g); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (epi == kEpiSplitK)
    return launch_sum_parts(g.out, g.ws, (int64_t)g.M * g.N, splits, (int64_t)g.M * g.N, s);
  if (epi == kEpiGeluBwd && g.col_part)
    return launch_sum_parts(g.col_sums, g.col_part, g.N, g.M / 32, g.N, s);
  return hipSuccess;
}

size_t fused_lds_bytes() {
  return sizeof(uint16_t) * kFusedRows * kFusedLd + 2 * sizeof(float) * kFusedRows + sizeof(float2) * (kCdfN + 1);
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

int loss_blocks(int M_pad) { return blocks_for(M_pad, 256); }

hipError_t launch_loss(const LossArgs &l, hipStream_t s) {
  const int blocks = loss_blocks(l.M_pad);
  hipLaunchKernelGGL(k_loss, dim3(blocks), dim3(256), 0, s, l);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(256), 0, s, l, blocks);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u64, dim3(min(blocks_for(n, 256), 4096)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// One thread per (batch row, feature column); columns 64..69 carry the labels.
__global__ void __launch_bounds__(256) k_gather(const GatherArgs g) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t i = t / 72, c = t % 72;
  if (i >= g.M) return;
  const bool real = i < g.count;
  const uint64_t r = (uint64_t)(g.first + i);
  const uint64_t p = real ? (g.mul * r + g.add) % g.P : 0;
  if (c < kInPad) {
    const uint16_t v = real ? g.X[p * kInPad + c] : (uint16_t)0;
    g.gX[i * kInPad + c] = v;
    g.gXT[c * (int64_t)g.M + i] = v;
    return;
  }
  const float *src;
  float *dst;
  switch (c - kInPad) {
    case 0: src = g.mu_base, dst = g.g_mu_base; break;
    case 1: src = g.nph, dst = g.g_nph; break;
    case 2: src = g.k, dst = g.g_k; break;
    case 3: src = g.n_t, dst = g.g_n_t; break;
    case 4: src = g.s1, dst = g.g_s1; break;
    case 5: src = g.s2, dst = g.g_s2; break;
    case 6:
      if (!g.w) return;
      src = g.w, dst = g.g_w;
      break;
    default: return;
  }
  dst[i] = real ? src[p] : 0.0f;
}

hipError_t launch_gather(const GatherArgs &g, hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(blocks_for((int64_t)g.M * 72, 256)), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_adam(float *theta, const float *grad, float *m, float *v, int64_t n, float lr, float c1,
                       float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(min(blocks_for(n, 256), 1024)), dim3(256), 0, s, theta, grad, m, v, n, lr, c1, c2);
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

// gfx950 kernels of the photon-propagation library.
//
// k_propagate is the hot path: Monte Carlo propagation of optical photons
// through layered ice to optical-module hits (Meagher & van Santen, Sec. 2,
// photon-propagation paragraph: draw the distance to the next scatter, pick
// a new direction from the scattering physics, repeat until the photon hits
// a module or is absorbed; the work is embarrassingly parallel over photons).
//
// Design for CDNA4 (wave64, 4 SIMD per CU, 160 KB LDS per CU):
//   * one photon per lane; the kernel is persistent and each wavefront takes
//     chunks of photon ids from a global queue with one atomic per chunk;
//     lanes whose photon ended are refilled from the chunk in the same pass
//     (ballot + mbcnt rank), so lanes stay busy despite the long,
//     geometric tail of steps per photon;
//   * emission shares the pass with propagation: a new lane draws Philox
//     block 0 where a running lane draws block 2 + j, and both go through
//     the same rotation code (emission is a rotation of the source axis);
//   * the layer table, the string table and the horizontal search grid are
//     staged in LDS once per workgroup; module coordinates stay in global
//     memory (read only when a photon passes within reach of a string);
//   * hits are compacted per wavefront (ballot, popcount, one atomic, mbcnt
//     slot), so the hit buffer is dense;
//   * all state lives in VGPRs; the Philox key is wave-uniform (SGPRs).
// The arithmetic is FP32 with hardware transcendentals; every step follows
// the FP64 definition (same random words, same tie rules), so each photon
// reproduces the FP64 result up to rounding.

#include "pp_device.h"

namespace pp {
namespace {

constexpr uint32_t kNoDom = 0xFFFFFFFFu;
constexpr uint32_t kLive = 0xFFu;
constexpr uint32_t kFateAbsorbed = 0, kFateHit = 1, kFateCapped = 2, kFateEscaped = 3;
constexpr float kNsPerMetreLight = 3.3356409519815204f;  // 1 / c, c = 0.299792458 m/ns
constexpr float kLn2 = 0.69314718055994531f;

__device__ __forceinline__ float inf_f() { return __builtin_huge_valf(); }

// Philox4x32-10 (Salmon et al., SC'11). The key schedule is wave-uniform, so
// the compiler keeps it in SGPRs; each round costs two 32x32->64 multiplies
// per lane.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t w[4]) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const unsigned long long p0 = (unsigned long long)0xD2511F53u * c0;
    const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  w[0] = c0;
  w[1] = c1;
  w[2] = c2;
  w[3] = c3;
}

// (2 (w >> 9) + 1) 2^-24: exact in FP32 (the conversion of a 23-bit integer
// and the fused multiply-add both round nothing).
__device__ __forceinline__ float u01(uint32_t w) {
  return __builtin_fmaf((float)(w >> 9), 0x1p-23f, 0x1p-24f);
}

__device__ __forceinline__ uint32_t lane_rank(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ unsigned long long first_lane_u64(unsigned long long v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

struct Segment {
  float px, py, pz, vx, vy, vz, len;
};

// Ray-sphere test of one module against the segment; keeps the nearest
// entry point, ties to the lower module id. A sphere containing the start
// point is ignored.
__device__ __forceinline__ void test_module(const float4 m, const Segment &s, float r2,
                                            float &best_t, uint32_t &best_id) {
  const float dx = s.px - m.x, dy = s.py - m.y, dz = s.pz - m.z;
  const float b = dx * s.vx + dy * s.vy + dz * s.vz;
  const float hx = dx - b * s.vx, hy = dy - b * s.vy, hz = dz - b * s.vz;
  const float disc = r2 - (hx * hx + hy * hy + hz * hz);
  if (disc >= 0.0f && dx * dx + dy * dy + dz * dz >= r2) {
    const float t = -b - __builtin_sqrtf(disc);
    const uint32_t id = __float_as_uint(m.w);
    if (t >= 0.0f && t <= s.len && (t < best_t || (t == best_t && id < best_id))) {
      best_t = t;
      best_id = id;
    }
  }
}

// Tests the modules of one string that the segment can reach: first a
// horizontal reach check against the string centre, then the slots whose z
// range overlaps the segment's (arithmetic for evenly spaced strings).
__device__ __forceinline__ void test_string(const DevString &st, const float4 *__restrict__ doms,
                                            const Segment &s, float radius, float r2,
                                            float &best_t, uint32_t &best_id, uint32_t &tests) {
  const float dx = st.xy_reach_z0.x - s.px, dy = st.xy_reach_z0.y - s.py;
  const float lim = __builtin_fmaf(s.len, 1.00001f, st.xy_reach_z0.z + 0.01f);
  if (dx * dx + dy * dy > lim * lim) return;
  const float zend = __builtin_fmaf(s.len, s.vz, s.pz);
  const float zmin = fminf(s.pz, zend) - radius;  // fminf drops a NaN end (infinite flat step)
  const float zmax = fmaxf(s.pz, zend) + radius;
  const float nf = (float)st.n;
  float flo = (zmin - st.xy_reach_z0.w) * st.inv_dz - st.kpad;
  float fhi = (zmax - st.xy_reach_z0.w) * st.inv_dz + st.kpad;
  flo = fminf(fmaxf(flo, -1.0f), nf);  // NaN -> -1: whole string
  fhi = fmaxf(fminf(fhi, nf), -1.0f);  // NaN -> n
  const int klo = max((int)floorf(flo), 0);
  const int khi = min((int)ceilf(fhi), st.n - 1);
  for (int k = klo; k <= khi; ++k) {
    ++tests;
    test_module(doms[st.first + k], s, r2, best_t, best_id);
  }
}

// Orthonormal basis of the unit vector r (Duff et al., JCGT 2017) and the
// direction at polar cosine 1 - om and azimuth phi (in turns) about r.
__device__ __forceinline__ void rotate(float rx, float ry, float rz, float om, float phi_turns,
                                       float &vx, float &vy, float &vz) {
  const float sign = copysignf(1.0f, rz);
  const float a = -__builtin_amdgcn_rcpf(sign + rz);
  const float b = rx * ry * a;
  const float e1x = __builtin_fmaf(sign * rx * rx, a, 1.0f), e1y = sign * b, e1z = -sign * rx;
  const float e2x = b, e2y = __builtin_fmaf(ry * ry, a, sign), e2z = -ry;
  const float mu = 1.0f - om;
  const float st = __builtin_sqrtf(om * (2.0f - om));
  const float c = __builtin_amdgcn_cosf(phi_turns);  // hardware cos/sin take turns
  const float s = __builtin_amdgcn_sinf(phi_turns);
  const float sc = st * c, ss = st * s;
  float x = mu * rx + sc * e1x + ss * e2x;
  float y = mu * ry + sc * e1y + ss * e2y;
  float z = mu * rz + sc * e1z + ss * e2z;
  const float inv = __builtin_amdgcn_rsqf(x * x + y * y + z * z);
  vx = x * inv;
  vy = y * inv;
  vz = z * inv;
}

__global__ void __launch_bounds__(1024) k_propagate(const PropagateArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  DevLayer *s_layers = reinterpret_cast<DevLayer *>(lds_raw);
  DevString *s_strings = reinterpret_cast<DevString *>(s_layers + a.n_layers);
  uint32_t *s_cells = reinterpret_cast<uint32_t *>(s_strings + a.n_strings);
  for (int i = threadIdx.x; i < a.n_layers; i += blockDim.x) s_layers[i] = a.layers[i];
  for (int i = threadIdx.x; i < a.n_strings; i += blockDim.x) s_strings[i] = a.strings[i];
  for (int i = threadIdx.x; i < a.nx * a.ny; i += blockDim.x) s_cells[i] = a.cells[i];
  __syncthreads();

  const uint32_t lane = __lane_id();
  const float r2 = a.radius2;

  // wave-uniform queue state
  uint32_t ch_src = 0, ch_left = 0;
  unsigned long long ch_local = 0;
  bool more = true;

  // lane state
  bool alive = false, fresh = false;
  uint32_t src = 0, event = 0, iter = 0, ncross = 0;
  unsigned long long local = 0, pidx = 0, seq = 0;
  float px = 0, py = 0, pz = 0, vx = 0, vy = 0, vz = 1, t = 0, tau_a = 0, lambda = 0;
  int layer = 0;

  uint32_t st_photons = 0, st_iter = 0, st_cross = 0, st_tests = 0;
  uint32_t st_hits = 0, st_abs = 0, st_cap = 0, st_esc = 0;

  for (;;) {
    // Refill lanes whose photon ended from the wavefront's chunk; grab a new
    // chunk when it runs out.
    if (more) {
      unsigned long long dead = __ballot(!alive);
      while (dead != 0 && more) {
        if (ch_left == 0) {
          unsigned long long c = 0;
          if (lane == 0) c = atomicAdd(&a.counters[kChunkNext], 1ull);
          c = first_lane_u64(c);
          if (c >= a.n_chunks) {
            more = false;
            break;
          }
          const DevChunk e = a.chunks[c];
          ch_src = e.src;
          ch_left = e.count;
          ch_local = e.local;
        }
        const uint32_t take = min((uint32_t)__popcll(dead), ch_left);
        const uint32_t rank = lane_rank(dead);
        if (!alive && rank < take) {
          alive = true;
          fresh = true;
          src = ch_src;
          local = ch_local + rank;
        }
        ch_left -= take;
        ch_local += take;
        dead = __ballot(!alive);
      }
    }
    if (__ballot(alive) == 0) break;

    uint32_t fate = kLive, hit_dom = kNoDom;
    if (alive) {
      // Source data for new photons.
      float4 sp = make_float4(0, 0, 0, 0), sd = sp, se = sp;
      uint32_t stype = 0;
      if (fresh) {
        const DevSource &S = a.sources[src];
        sp = S.pos_t0;
        sd = S.dir_len;
        se = S.emit;
        stype = S.ids.x;
        event = S.ids.y;
        pidx = S.first_index + local;
        seq = S.seq_base + local;
      }
      uint32_t w[4];
      philox4x32_10(fresh ? 0u : 2u + iter, event, (uint32_t)pidx, (uint32_t)(pidx >> 32),
                    a.seed_lo, a.seed_hi, w);
      const float u0 = u01(w[0]), u1 = u01(w[1]), u2 = u01(w[2]);
      // one logarithm: the absorption budget at emission, the scattering
      // optical depth of the step otherwise
      const float neg_log = -kLn2 * __builtin_amdgcn_logf(fresh ? u2 : u0);

      float rx = 0, ry = 0, rz = 1, om = 0, phi = 0;
      bool turn = false;
      if (fresh) {
        // Emission: a point source rotates +z by cos(theta) = 2 u0 - 1; a
        // Cherenkov segment emits from u0 * length along the track, on the
        // cone about the track axis. Azimuth u1 in both cases.
        const bool point = stype == 0;
        const float sdist = point ? 0.0f : u0 * sd.w;
        px = __builtin_fmaf(sdist, sd.x, sp.x);
        py = __builtin_fmaf(sdist, sd.y, sp.y);
        pz = __builtin_fmaf(sdist, sd.z, sp.z);
        t = __builtin_fmaf(sdist, kNsPerMetreLight, sp.w);
        rx = sd.x;
        ry = sd.y;
        rz = sd.z;
        om = point ? 2.0f * (1.0f - u0) : se.x;
        phi = u1;
        turn = true;
        tau_a = neg_log;
        lambda = se.y != 0.0f ? se.y : __builtin_amdgcn_rcpf(__builtin_fmaf(-u01(w[3]), se.w, se.z));
        const float lf = floorf((pz - a.z_lo) / a.dz);
        layer = lf >= 0.0f ? (lf >= (float)(a.n_layers - 1) ? a.n_layers - 1 : (int)lf) : 0;
        iter = 0;
        ncross = 0;
        fresh = false;
        ++st_photons;
      } else {
        ++iter;
        ++st_iter;
        float tau_s = neg_log;
        // Layer walk: consume both optical-depth budgets layer by layer
        // until one runs out (ties: absorb <= scatter <= boundary).
        const int dir = vz > 0.0f ? 1 : (vz < 0.0f ? -1 : 0);
        const float rvz = __builtin_amdgcn_rcpf(vz);
        float len = 0.0f, zc = pz;
        int i = layer;
        uint32_t end;  // 0 absorb, 1 scatter, 2 escape
        for (;;) {
          const float4 c = s_layers[i].coef;
          const float d_abs = c.x > 0.0f ? tau_a * c.z : inf_f();
          const float d_sca = c.y > 0.0f ? tau_s * c.w : inf_f();
          const int nb = dir > 0 ? i + 1 : i;
          const bool bounded = (dir > 0 && i < a.n_layers - 1) || (dir < 0 && i > 0);
          const float zb = __builtin_fmaf((float)nb, a.dz, a.z_lo);
          const float d_bnd = bounded ? fmaxf(0.0f, (zb - zc) * rvz) : inf_f();
          if (d_abs == inf_f() && d_sca == inf_f() && d_bnd == inf_f()) {
            len = inf_f();
            end = 2;
            break;
          }
          if (d_abs <= d_sca && d_abs <= d_bnd) {
            len += d_abs;
            tau_a = 0.0f;
            end = 0;
            break;
          }
          if (d_sca <= d_bnd) {
            len += d_sca;
            tau_a = fmaxf(0.0f, tau_a - c.x * d_sca);
            end = 1;
            break;
          }
          len += d_bnd;
          tau_a = fmaxf(0.0f, tau_a - c.x * d_bnd);
          tau_s = fmaxf(0.0f, tau_s - c.y * d_bnd);
          zc = zb;
          i += dir;
          ++ncross;
          ++st_cross;
        }
        layer = i;

        // Nearest module on the segment: the string listed for the grid
        // cell of the start point, and every other string only when the step
        // is longer than the cell's clearance to them.
        Segment seg{px, py, pz, vx, vy, vz, len};
        float best_t = inf_f();
        uint32_t best_id = kNoDom;
        {
          const float fx = fminf(fmaxf((px - a.gx0) * a.inv_cell, 0.0f), (float)(a.nx - 1));
          const float fy = fminf(fmaxf((py - a.gy0) * a.inv_cell, 0.0f), (float)(a.ny - 1));
          const uint32_t word = s_cells[(int)fy * a.nx + (int)fx];
          const uint32_t s1 = word & 0xFFFFu, q = word >> 16;
          const float clearance = q == 0xFFFFu ? inf_f() : (float)q * 0.0625f;
          if (s1 != 0xFFFFu)
            test_string(s_strings[s1], a.doms, seg, a.radius, r2, best_t, best_id, st_tests);
          if (len >= clearance) {
            for (int s = 0; s < a.n_strings; ++s)
              if ((uint32_t)s != s1)
                test_string(s_strings[s], a.doms, seg, a.radius, r2, best_t, best_id, st_tests);
          }
        }

        if (best_id != kNoDom) {
          px = __builtin_fmaf(best_t, vx, px);
          py = __builtin_fmaf(best_t, vy, py);
          pz = __builtin_fmaf(best_t, vz, pz);
          t = __builtin_fmaf(best_t, a.time_per_m, t);
          fate = kFateHit;
          hit_dom = best_id;
        } else if (end == 2) {
          fate = kFateEscaped;
        } else {
          px = __builtin_fmaf(len, vx, px);
          py = __builtin_fmaf(len, vy, py);
          pz = __builtin_fmaf(len, vz, pz);
          t = __builtin_fmaf(len, a.time_per_m, t);
          if (end == 0) {
            fate = kFateAbsorbed;
          } else {
            // Henyey-Greenstein polar angle in the cancellation-free form
            // 1 - mu = (1 - g)(1 - u)(s + 1 - g)/w, w = 1 - g + 2 g u,
            // s = (1 - g^2)/w; azimuth u2.
            const float4 hg = s_layers[layer].hg;
            const float wv = __builtin_fmaf(hg.z, u1, hg.x);
            const float rw = __builtin_amdgcn_rcpf(wv);
            const float sv = hg.y * rw;
            om = hg.x * (1.0f - u1) * (sv + hg.x) * rw;
            phi = u2;
            rx = vx;
            ry = vy;
            rz = vz;
            turn = true;
          }
        }
      }
      if (turn) {
        rotate(rx, ry, rz, om, phi, vx, vy, vz);
        if (iter >= a.step_cap) fate = kFateCapped;
      }
    }

    // Wave-compacted hit output: one atomic per wavefront.
    const bool is_hit = fate == kFateHit;
    const unsigned long long hmask = __ballot(is_hit);
    if (hmask != 0) {
      unsigned long long base = 0;
      if (lane == 0) base = atomicAdd(&a.counters[kHitCount], (unsigned long long)__popcll(hmask));
      base = first_lane_u64(base);
      if (is_hit) {
        const unsigned long long slot = base + lane_rank(hmask);
        if (slot < a.hit_capacity) {
          uint4 *out = reinterpret_cast<uint4 *>(a.hits + slot);
          const uint32_t particle = a.sources[src].ids.z;
          out[0] = make_uint4((uint32_t)pidx, (uint32_t)(pidx >> 32), event, particle);
          out[1] = make_uint4(hit_dom, __float_as_uint(t), __float_as_uint(1.0f), 0u);
        }
      }
    }
    if (fate != kLive) {
      st_hits += fate == kFateHit;
      st_abs += fate == kFateAbsorbed;
      st_cap += fate == kFateCapped;
      st_esc += fate == kFateEscaped;
      if (a.rec.fate != nullptr) {
        a.rec.fate[seq] = fate;
        a.rec.dom[seq] = hit_dom;
        a.rec.n_iter[seq] = iter;
        a.rec.n_cross[seq] = ncross;
        a.rec.t[seq] = t;
        a.rec.x[seq] = px;
        a.rec.y[seq] = py;
        a.rec.z[seq] = pz;
        a.rec.vx[seq] = vx;
        a.rec.vy[seq] = vy;
        a.rec.vz[seq] = vz;
        a.rec.wavelength[seq] = lambda;
      }
      alive = false;
    }
  }

  // Per-wavefront reduction of the counters, then one atomic each.
  const uint32_t sums[8] = {wave_sum(st_photons), wave_sum(st_iter), wave_sum(st_cross),
                            wave_sum(st_tests),   wave_sum(st_hits), wave_sum(st_abs),
                            wave_sum(st_cap),     wave_sum(st_esc)};
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (sums[k] != 0) atomicAdd(&a.counters[kStatPhotons + k], (unsigned long long)sums[k]);
  }
}

__global__ void k_reset(unsigned long long *counters, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) counters[i] = 0;
}

__global__ void k_zero_u32(uint32_t *p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = 0;
}

// Per-module hit histogram: an LDS histogram per workgroup over a slice of
// the hit buffer, then one global atomic per non-empty bin.
__global__ void __launch_bounds__(256) k_dom_histogram(const DevHit *__restrict__ hits,
                                                       const unsigned long long *hit_count,
                                                       unsigned long long cap, uint32_t *counts,
                                                       uint32_t n_doms) {
  extern __shared__ uint32_t hist[];
  for (uint32_t i = threadIdx.x; i < n_doms; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  unsigned long long n = *hit_count;
  if (n > cap) n = cap;
  for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    const uint32_t d = hits[i].dom_id;
    if (d < n_doms) atomicAdd(&hist[d], 1u);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n_doms; i += blockDim.x)
    if (hist[i] != 0) atomicAdd(&counts[i], hist[i]);
}

__global__ void k_dom_histogram_global(const DevHit *__restrict__ hits,
                                       const unsigned long long *hit_count, unsigned long long cap,
                                       uint32_t *counts, uint32_t n_doms) {
  unsigned long long n = *hit_count;
  if (n > cap) n = cap;
  for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    const uint32_t d = hits[i].dom_id;
    if (d < n_doms) atomicAdd(&counts[d], 1u);
  }
}

}  // namespace

size_t propagate_lds_bytes(int n_layers, int n_strings, int n_cells) {
  return sizeof(DevLayer) * n_layers + sizeof(DevString) * n_strings + 4u * n_cells;
}

hipError_t launch_reset(unsigned long long *counters, int n, hipStream_t stream) {
  hipLaunchKernelGGL(k_reset, dim3((n + 63) / 64), dim3(64), 0, stream, counters, n);
  return hipGetLastError();
}

hipError_t launch_propagate(const PropagateArgs &args, int grid, int block, hipStream_t stream) {
  const size_t lds = propagate_lds_bytes(args.n_layers, args.n_strings, args.nx * args.ny);
  hipLaunchKernelGGL(k_propagate, dim3(grid), dim3(block), lds, stream, args);
  return hipGetLastError();
}

hipError_t propagate_occupancy(int block, size_t lds_bytes, int *blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_propagate, block, lds_bytes);
}

hipError_t launch_dom_histogram(const DevHit *hits, const unsigned long long *hit_count,
                                unsigned long long hit_capacity, uint32_t *counts, uint32_t n_doms,
                                hipStream_t stream) {
  if (n_doms == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3(min((n_doms + 255u) / 256u, 1024u)), dim3(256), 0, stream,
                     counts, n_doms);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (n_doms <= 16384) {
    hipLaunchKernelGGL(k_dom_histogram, dim3(256), dim3(256), n_doms * sizeof(uint32_t), stream,
                       hits, hit_count, hit_capacity, counts, n_doms);
  } else {
    hipLaunchKernelGGL(k_dom_histogram_global, dim3(256), dim3(256), 0, stream, hits, hit_count,
                       hit_capacity, counts, n_doms);
  }
  return hipGetLastError();
}

}  // namespace pp

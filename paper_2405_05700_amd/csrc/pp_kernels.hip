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
//   * emission shares the pass with propagation: a refilled lane draws
//     Philox block 0 where a running lane draws block 2 + j, and both share
//     the generator, the logarithm and the rotation (emission is a rotation
//     of the source axis), so the refill itself is only bookkeeping and can
//     run every few passes;
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
constexpr uint32_t kLive = 0xFFu;  // fate of a photon still propagating
constexpr uint32_t kFateAbsorbed = 0, kFateHit = 1, kFateCapped = 2, kFateEscaped = 3;
constexpr float kNsPerMetreLight = 3.3356409519815204f;  // 1 / c, c = 0.299792458 m/ns
constexpr float kLn2 = 0.69314718055994531f;

__device__ __forceinline__ float inf_f() { return __builtin_huge_valf(); }

// a ^ b ^ c in one gfx950 instruction (v_bitop3_b32, truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon et al., SC'11). The key schedule is wave-uniform, so
// the compiler keeps it in SGPRs; each round costs two 32x32->64 multiplies
// and two three-input xors per lane.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t w[4]) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const unsigned long long p0 = (unsigned long long)0xD2511F53u * c0;
    const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c2;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
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

__device__ __forceinline__ float first_lane_f32(float v) {
  return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v)));
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
    const float t = -b - __builtin_amdgcn_sqrtf(disc);
    const uint32_t id = __float_as_uint(m.w);
    if (t >= 0.0f && t <= s.len && (t < best_t || (t == best_t && id < best_id))) {
      best_t = t;
      best_id = id;
    }
  }
}

// Tests the modules of one string that the segment can reach. First the
// horizontal filter: the segment's projection on the horizontal plane must
// pass within the string's reach (largest module offset from the axis + r +
// margin) of the string's axis, a necessary condition for meeting any of its
// spheres; then the slots whose z range overlaps the segment's (arithmetic
// for evenly spaced strings). A module is read from the global table (x, y,
// z, id), or, for a vertical string, rebuilt from the string centre and its
// (z, id) pair in LDS.
template <bool kLds>
__device__ __forceinline__ void test_string(const DevString &st, const float4 *__restrict__ doms,
                                            const float2 *zid, const Segment &s, float radius, float r2,
                                            float &best_t, uint32_t &best_id, uint32_t &tests) {
  const float dx = st.xy_reach_z0.x - s.px, dy = st.xy_reach_z0.y - s.py;
  // No point of the step is within reach if its start is farther than
  // len + reach from the axis (with a margin far above rounding, so this
  // never drops a step the test below would keep).
  const float rr = __builtin_fmaf(s.len + st.xy_reach_z0.z, 1.0f / 1024.0f, s.len + st.xy_reach_z0.z) + 1e-3f;
  if (dx * dx + dy * dy > rr * rr) return;
  // closest approach of the projected segment to the axis: t in [0, len]
  // along v (a vertical segment stays at its start point)
  const float hh = s.vx * s.vx + s.vy * s.vy;
  const float proj = dx * s.vx + dy * s.vy;
  const float tq = hh > 0.0f ? fminf(fmaxf(proj * __builtin_amdgcn_rcpf(hh), 0.0f), s.len) : 0.0f;
  const float qx = __builtin_fmaf(-tq, s.vx, dx), qy = __builtin_fmaf(-tq, s.vy, dy);
  const float reach = st.xy_reach_z0.z;
  if (qx * qx + qy * qy > reach * reach) return;
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
    if (kLds) {
      const float2 e = zid[st.first + k];
      test_module(make_float4(st.xy_reach_z0.x, st.xy_reach_z0.y, e.x, e.y), s, r2, best_t, best_id);
    } else {
      test_module(doms[st.first + k], s, r2, best_t, best_id);
    }
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
  const float st = __builtin_amdgcn_sqrtf(om * (2.0f - om));  // v_sqrt_f32 (1 ulp)
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

// Weight of a hit (the chance that it makes a photoelectron): acceptance
// table at the wavelength, linear between points and held beyond the ends,
// times the angular polynomial in the cosine of incidence c = -v . n, n the
// outward surface normal where the photon meets the module.
__device__ __forceinline__ float hit_weight(const PropagateArgs &a, uint32_t dom, float px, float py, float pz,
                                         float vx, float vy, float vz, float lambda) {
  float A = a.acc[0];
  if (a.n_acc > 1) {
    const float x = fminf(fmaxf((lambda - a.acc_l0) * a.inv_acc_dl, 0.0f), (float)(a.n_acc - 1));
    const uint32_t k = min((uint32_t)x, a.n_acc - 2);
    const float f = x - (float)k;
    A = __builtin_fmaf(a.acc[k + 1] - a.acc[k], f, a.acc[k]);
  }
  const float4 m = a.doms_by_id[dom];
  const float c = -((px - m.x) * vx + (py - m.y) * vy + (pz - m.z) * vz) * a.inv_radius;
  const float cc = fminf(fmaxf(c, 0.0f), 1.0f);
  float P = 0.0f;
  for (int k = (int)a.n_poly - 1; k >= 0; --k) P = __builtin_fmaf(P, cc, a.poly[k]);
  return A * P;
}

// kWave: the photon's wavelength matters (wavelength-dependent optics, hit
// acceptance, or debug records that ask for it). Without it the kernel draws
// no wavelength and scales nothing, and every hit weighs 1; its photons take
// the same paths, since the wavelength has a Philox word of its own.
// kRecords: per-photon terminal records (parity checks only).
// kLdsDoms: every string is vertical, so a module is its string's centre
// and a (z, id) pair, and the pairs of all modules are staged in LDS (8
// bytes each): the ray-sphere tests of the few lanes near a string then read
// LDS instead of stalling the whole wavefront on global memory.
template <bool kRecords, bool kWave, bool kLdsDoms>
__global__ void __launch_bounds__(1024)
k_propagate(const PropagateArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  DevLayer *s_layers = reinterpret_cast<DevLayer *>(lds_raw);
  DevString *s_strings = reinterpret_cast<DevString *>(s_layers + a.n_layers);
  uint32_t *s_cells = reinterpret_cast<uint32_t *>(s_strings + a.n_strings);
  float *s_bounds = reinterpret_cast<float *>(s_cells + a.nx * a.ny);
  for (int i = threadIdx.x; i < a.n_layers; i += blockDim.x) s_layers[i] = a.layers[i];
  for (int i = threadIdx.x; i < a.n_strings; i += blockDim.x) s_strings[i] = a.strings[i];
  for (int i = threadIdx.x; i < a.nx * a.ny; i += blockDim.x) s_cells[i] = a.cells[i];
  for (int i = threadIdx.x; i <= a.n_layers; i += blockDim.x) s_bounds[i] = a.bounds[i];
  float2 *s_zid = nullptr;
  if (kLdsDoms) {
    const size_t off = (static_cast<size_t>(reinterpret_cast<unsigned char *>(s_bounds + a.n_layers + 1) - lds_raw) +
                        7) & ~static_cast<size_t>(7);
    s_zid = reinterpret_cast<float2 *>(lds_raw + off);
    for (int i = threadIdx.x; i < a.n_doms; i += blockDim.x) {
      const float4 m = a.doms[i];
      s_zid[i] = make_float2(m.z, m.w);
    }
  }
  __syncthreads();

  const uint32_t lane = __lane_id();
  const float r2 = a.radius2;

  // wave-uniform queue state and counters; the chunk's source record is
  // read once per chunk into wave-uniform registers, so handing photons to
  // free lanes reads no memory
  uint32_t ch_src = 0, ch_left = 0, countdown = 0;
  unsigned long long ch_local = 0;
  unsigned long long cs_first = 0, cs_seq = 0;
  uint32_t cs_event = 0, cs_particle = 0;
  float cs_px = 0, cs_py = 0, cs_pz = 0, cs_t = 0, cs_vx = 0, cs_vy = 0, cs_vz = 1, cs_elen = 0, cs_eom = -1;
  bool more = true;
  uint32_t n_photons = 0, n_hits = 0, n_abs = 0, n_cap = 0, n_esc = 0;

  // Lane state. A lane is free, emitting (photon assigned: position and
  // direction hold the source's start point and axis), live (propagating)
  // or ended (stopped, output not yet written).
  constexpr uint32_t kFree = 0, kEmit = 1, kRun = 2, kEnded = 3;
  uint32_t phase = kFree;
  uint32_t event = 0, particle = 0, iter = 0, ncross = 0, fate = 0, hit_dom = kNoDom, src = 0;
  unsigned long long pidx = 0, seq = 0;
  float px = 0, py = 0, pz = 0, vx = 0, vy = 0, vz = 1, t = 0, tau_a = 0, lambda = 0;
  float elen = 0, eom = 0;  // emission: track length (0: point) and 1 - cos(cone), < 0 for a point source
  float inv_sb = 1.0f;      // 1 / scattering-coefficient scale at the photon's wavelength
  int layer = 0;
  uint32_t st_iter = 0, st_cross = 0, st_tests = 0;

  for (;;) {
    // Every refill_interval passes (or when no lane is emitting or live):
    // write out the lanes that ended, then hand free lanes the next photon
    // ids of the wavefront's chunk.
    if (countdown == 0 || __ballot(phase == kEmit || phase == kRun) == 0) {
      countdown = a.refill_interval;
      const bool ended = phase == kEnded;
      const unsigned long long hmask = __ballot(ended && fate == kFateHit);
      if (hmask != 0) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&a.counters[kHitCount], (unsigned long long)__popcll(hmask));
        base = first_lane_u64(base);
        if (ended && fate == kFateHit) {
          const unsigned long long slot = base + lane_rank(hmask);
          if (slot < a.hit_capacity) {
            const float weight =
                kWave && a.n_acc ? hit_weight(a, hit_dom, px, py, pz, vx, vy, vz, lambda) : 1.0f;
            uint4 *out = reinterpret_cast<uint4 *>(a.hits + slot);
            out[0] = make_uint4((uint32_t)pidx, (uint32_t)(pidx >> 32), event, particle);
            out[1] = make_uint4(hit_dom, __float_as_uint(t), __float_as_uint(weight), 0u);
          }
        }
      }
      n_hits += __popcll(hmask);
      n_abs += __popcll(__ballot(ended && fate == kFateAbsorbed));
      n_cap += __popcll(__ballot(ended && fate == kFateCapped));
      n_esc += __popcll(__ballot(ended && fate == kFateEscaped));
      if (kRecords && ended) {
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
        a.rec.wavelength[seq] = kWave ? lambda : 0.0f;  // a variant without kWave draws none
      }
      if (ended) phase = kFree;

      unsigned long long free_mask = __ballot(phase == kFree);
      while (free_mask != 0 && more) {
        if (ch_left == 0) {
          unsigned long long c = 0;
          if (lane == 0) c = atomicAdd(&a.counters[kChunkNext], 1ull);
          c = first_lane_u64(c);
          if (c >= a.n_chunks) {
            more = false;
            break;
          }
          const DevChunk e = a.chunks[c];
          ch_src = __builtin_amdgcn_readfirstlane(e.src);
          ch_left = __builtin_amdgcn_readfirstlane(e.count);
          ch_local = first_lane_u64(e.local);
          // The lanes start at the source's reference point on its axis; the
          // emission pass moves them along the track and turns them onto the
          // emission cone (or the sphere, for a point source).
          const DevSource &S = a.sources[ch_src];
          const bool point = __builtin_amdgcn_readfirstlane(S.ids.x) == 0;
          cs_first = first_lane_u64(S.first_index);
          if (kRecords) cs_seq = first_lane_u64(S.seq_base);
          cs_event = __builtin_amdgcn_readfirstlane(S.ids.y);
          cs_particle = __builtin_amdgcn_readfirstlane(S.ids.z);
          cs_px = first_lane_f32(S.pos_t0.x);
          cs_py = first_lane_f32(S.pos_t0.y);
          cs_pz = first_lane_f32(S.pos_t0.z);
          cs_t = first_lane_f32(S.pos_t0.w);
          cs_vx = first_lane_f32(S.dir_len.x);
          cs_vy = first_lane_f32(S.dir_len.y);
          cs_vz = first_lane_f32(S.dir_len.z);
          cs_elen = point ? 0.0f : first_lane_f32(S.dir_len.w);
          cs_eom = point ? -1.0f : first_lane_f32(S.emit.x);
        }
        const uint32_t take = min((uint32_t)__popcll(free_mask), ch_left);
        const uint32_t rank = lane_rank(free_mask);
        if (((free_mask >> lane) & 1ull) && rank < take) {
          const unsigned long long local = ch_local + rank;
          pidx = cs_first + local;
          if (kWave) src = ch_src;
          if (kRecords) seq = cs_seq + local;
          event = cs_event;
          particle = cs_particle;
          px = cs_px;
          py = cs_py;
          pz = cs_pz;
          t = cs_t;
          vx = cs_vx;
          vy = cs_vy;
          vz = cs_vz;
          elen = cs_elen;
          eom = cs_eom;
          iter = 0;
          ncross = 0;
          fate = kFateCapped;
          hit_dom = kNoDom;
          phase = kEmit;
        }
        n_photons += take;
        ch_left -= take;
        ch_local += take;
        free_mask = __ballot(phase == kFree);
      }
      if (!more && __ballot(phase != kFree) == 0) break;
    }
    --countdown;

    if (phase == kEmit || phase == kRun) {
      const bool emit = phase == kEmit;
      // The round keys are recomputed with scalar adds each pass rather than
      // held in 20 SGPRs across the loop (which would cap occupancy).
      uint32_t k0 = a.seed_lo, k1 = a.seed_hi;
      asm volatile("" : "+s"(k0), "+s"(k1));
      uint32_t w[4];
      philox4x32_10(emit ? 0u : 2u + iter, event, (uint32_t)pidx, (uint32_t)(pidx >> 32), k0, k1, w);
      // One logarithm per pass: the absorption budget -ln u2 at emission,
      // the scattering budget -ln u0 on a step.
      const float budget = -kLn2 * __builtin_amdgcn_logf(u01(emit ? w[2] : w[0]));
      float om, phi;
      uint32_t f;
      bool turn;  // take the rotated direction: emission, or a scatter (also the one that reaches the cap)
      if (emit) {
        // Emission (block 0): u0 places a Cherenkov photon along the track
        // (a point source: cos(theta) = 2 u0 - 1 about +z), u1 is the
        // azimuth, u2 the absorption budget.
        const float u0 = u01(w[0]);
        const float sdist = u0 * elen;
        px = __builtin_fmaf(sdist, vx, px);
        py = __builtin_fmaf(sdist, vy, py);
        pz = __builtin_fmaf(sdist, vz, pz);
        t = __builtin_fmaf(sdist, kNsPerMetreLight, t);
        om = eom < 0.0f ? 2.0f * (1.0f - u0) : eom;
        phi = u01(w[1]);
        tau_a = budget;
        if (kWave) {
          // wavelength: fixed, or u3 through the inverse CDF of a 1/l^2 density
          const float4 em = a.sources[src].emit;
          lambda = em.y != 0.0f ? em.y : __builtin_amdgcn_rcpf(__builtin_fmaf(-u01(w[3]), em.w, em.z));
          // Coefficients scaled by s = (l / l_ref)^-kappa are the same as the
          // table's coefficients with every optical-depth budget divided by
          // s: the absorption budget once here, the scattering budget each
          // step. Exponents 0 give factors of exactly 1.
          const float lr = __builtin_amdgcn_logf(lambda * a.inv_lambda_ref);
          tau_a = budget * __builtin_amdgcn_exp2f(a.kappa_abs * lr);
          inv_sb = __builtin_amdgcn_exp2f(a.kappa_scat * lr);
        }
        const float lf = floorf((pz - a.z_lo) * a.inv_dz);
        layer = lf >= 0.0f ? (lf >= (float)(a.n_layers - 1) ? a.n_layers - 1 : (int)lf) : 0;
        f = a.step_cap != 0 ? kLive : kFateCapped;
        turn = true;
      } else {
        ++iter;
        ++st_iter;
        float tau_s = kWave ? budget * inv_sb : budget;

        // Layer walk: consume both optical-depth budgets layer by layer
        // until one runs out (ties: absorb <= scatter <= boundary). A zero
        // coefficient has an infinite reciprocal; fminf turns the 0 * inf of
        // an exhausted budget there into +inf (an infinite distance), so no
        // distance is NaN and a crossing always has a finite boundary
        // distance (the edge layers' boundaries are at infinity).
        const bool up = vz > 0.0f;
        const bool flat = vz == 0.0f;
        const float rvz = __builtin_amdgcn_rcpf(vz);
        const int di = up ? 1 : -1, bofs = up ? 1 : 0;
        float len = 0.0f, zc = pz, cx, d_abs, d_sca;
        int i = layer;
        for (;;) {
          const float4 c = s_layers[i].coef;
          cx = c.x;
          d_abs = fminf(tau_a * c.z, inf_f());
          d_sca = fminf(tau_s * c.w, inf_f());
          const float zb = s_bounds[i + bofs];
          const float d_bnd = flat ? inf_f() : fmaxf(0.0f, (zb - zc) * rvz);
          if (!(d_bnd < fminf(d_abs, d_sca))) break;
          len += d_bnd;
          tau_a = fmaxf(0.0f, tau_a - c.x * d_bnd);
          tau_s = fmaxf(0.0f, tau_s - c.y * d_bnd);
          zc = zb;
          i += di;
        }
        const uint32_t crossed = (uint32_t)abs(i - layer);
        ncross += crossed;
        st_cross += crossed;
        int end;  // 0 absorb, 1 scatter, 2 escape (all three distances infinite)
        if (d_abs == inf_f() && d_sca == inf_f()) {
          len = inf_f();
          end = 2;
        } else if (d_abs <= d_sca) {
          len += d_abs;
          end = 0;
        } else {
          len += d_sca;
          tau_a = fmaxf(0.0f, tau_a - cx * d_sca);
          end = 1;
        }

        // Nearest module on the segment: the string listed for the grid cell
        // of the start point, and every other string only when the step is
        // at least the cell's clearance to them.
        const Segment seg{px, py, pz, vx, vy, vz, len};
        float best_t = inf_f();
        uint32_t best_id = kNoDom;
        {
          const float fx = __builtin_amdgcn_fmed3f((px - a.gx0) * a.inv_cell, 0.0f, a.nx_max);
          const float fy = __builtin_amdgcn_fmed3f((py - a.gy0) * a.inv_cell, 0.0f, a.ny_max);
          const uint32_t word = s_cells[__umul24((uint32_t)fy, (uint32_t)a.nx) + (uint32_t)fx];
          const uint32_t s1 = word & 0xFFFFu;
          const float clearance = __uint_as_float(word & 0xFFFF0000u);
          if (s1 != 0xFFFFu)
            test_string<kLdsDoms>(s_strings[s1], a.doms, s_zid, seg, a.radius, r2, best_t, best_id, st_tests);
          if (len >= clearance) {
            for (int s = 0; s < a.n_strings; ++s)
              if ((uint32_t)s != s1)
                test_string<kLdsDoms>(s_strings[s], a.doms, s_zid, seg, a.radius, r2, best_t, best_id, st_tests);
          }
        }

        const bool hit = best_id != kNoDom;
        const float dmove = hit ? best_t : (end == 2 ? 0.0f : len);
        px = __builtin_fmaf(dmove, vx, px);
        py = __builtin_fmaf(dmove, vy, py);
        pz = __builtin_fmaf(dmove, vz, pz);
        t = __builtin_fmaf(dmove, a.time_per_m, t);
        layer = i;
        hit_dom = best_id;
        f = hit ? kFateHit : (end == 2 ? kFateEscaped : (end == 0 ? kFateAbsorbed : kLive));
        turn = f == kLive;
        if (turn && iter >= a.step_cap) f = kFateCapped;

        // Henyey-Greenstein polar angle in the cancellation-free form
        // 1 - mu = (1 - g)(1 - u)(s + 1 - g)/w, w = 1 - g + 2 g u,
        // s = (1 - g^2)/w, with u = u1, and azimuth u2.
        const float4 hg = s_layers[i].hg;
        const float u1 = u01(w[1]);
        const float rw = __builtin_amdgcn_rcpf(__builtin_fmaf(hg.z, u1, hg.x));
        om = hg.x * (1.0f - u1) * __builtin_fmaf(hg.y, rw, hg.x) * rw;
        phi = u01(w[2]);
      }
      // One rotation serves both: the emission cone about the source axis
      // and the scattering angle about the current direction.
      float nx, ny, nz;
      rotate(vx, vy, vz, om, phi, nx, ny, nz);
      if (turn) {
        vx = nx;
        vy = ny;
        vz = nz;
      }
      if (f == kLive) {
        phase = kRun;
      } else {
        phase = kEnded;
        fate = f;
      }
    }
  }

  // Per-wavefront reduction of the counters, then one atomic each.
  const uint32_t it = wave_sum(st_iter), cr = wave_sum(st_cross), te = wave_sum(st_tests);
  if (lane == 0) {
    const uint32_t v[8] = {n_photons, it, cr, te, n_hits, n_abs, n_cap, n_esc};
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (v[k] != 0) atomicAdd(&a.counters[kStatPhotons + k], (unsigned long long)v[k]);
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

// Per-module sums of hit weights (double): a histogram per workgroup in
// LDS, then one global atomic per non-empty bin; used when n_doms x 8 B fits
// the LDS budget, else straight global atomics.
template <bool kLds>
__global__ void __launch_bounds__(256) k_dom_weights(const DevHit *__restrict__ hits,
                                                     const unsigned long long *hit_count, unsigned long long cap,
                                                     double *sums, uint32_t n_doms) {
  extern __shared__ double wsum[];
  if (kLds) {
    for (uint32_t i = threadIdx.x; i < n_doms; i += blockDim.x) wsum[i] = 0.0;
    __syncthreads();
  }
  unsigned long long n = *hit_count;
  if (n > cap) n = cap;
  for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    const uint32_t d = hits[i].dom_id;
    if (d < n_doms) atomicAdd(kLds ? &wsum[d] : &sums[d], (double)hits[i].weight);
  }
  if (kLds) {
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n_doms; i += blockDim.x)
      if (wsum[i] != 0.0) atomicAdd(&sums[i], wsum[i]);
  }
}

}  // namespace

size_t propagate_lds_bytes(int n_layers, int n_strings, int n_cells, int n_lds_doms) {
  const size_t tables = sizeof(DevLayer) * n_layers + sizeof(DevString) * n_strings + 4u * n_cells +
                        4u * (n_layers + 1);
  return n_lds_doms > 0 ? ((tables + 7) & ~static_cast<size_t>(7)) + sizeof(float2) * n_lds_doms : tables;
}

hipError_t launch_reset(unsigned long long *counters, int n, hipStream_t stream) {
  hipLaunchKernelGGL(k_reset, dim3((n + 63) / 64), dim3(64), 0, stream, counters, n);
  return hipGetLastError();
}

bool needs_wave(const PropagateArgs &a) { return a.kappa_abs != 0.0f || a.kappa_scat != 0.0f || a.n_acc != 0; }

// Launches / sizes one kernel variant; its dynamic-LDS limit is raised once
// to kMaxPropagateLds.
template <bool R, bool Wv, bool L>
hipError_t allow_lds() {
  static const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_propagate<R, Wv, L>),
                                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  static_cast<int>(kMaxPropagateLds));
  return e;
}

template <bool R, bool Wv, bool L>
hipError_t launch_variant(const PropagateArgs &a, int grid, int block, size_t lds, hipStream_t stream) {
  const hipError_t e = allow_lds<R, Wv, L>();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_propagate<R, Wv, L>), dim3(grid), dim3(block), lds, stream, a);
  return hipGetLastError();
}

template <bool R, bool Wv, bool L>
hipError_t occupancy_variant(int block, size_t lds, int *per_cu) {
  const hipError_t e = allow_lds<R, Wv, L>();
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_propagate<R, Wv, L>, block, lds);
}

hipError_t launch_propagate(const PropagateArgs &args, int grid, int block, hipStream_t stream) {
  const bool L = args.lds_doms != 0;
  const size_t lds = propagate_lds_bytes(args.n_layers, args.n_strings, args.nx * args.ny, L ? args.n_doms : 0);
  if (args.rec.fate != nullptr) {
    if (needs_wave(args) || args.records_wavelength)
      return L ? launch_variant<true, true, true>(args, grid, block, lds, stream)
               : launch_variant<true, true, false>(args, grid, block, lds, stream);
    return L ? launch_variant<true, false, true>(args, grid, block, lds, stream)
             : launch_variant<true, false, false>(args, grid, block, lds, stream);
  }
  if (needs_wave(args))
    return L ? launch_variant<false, true, true>(args, grid, block, lds, stream)
             : launch_variant<false, true, false>(args, grid, block, lds, stream);
  return L ? launch_variant<false, false, true>(args, grid, block, lds, stream)
           : launch_variant<false, false, false>(args, grid, block, lds, stream);
}

hipError_t propagate_occupancy(bool records, bool wave, bool lds_doms, int block, size_t lds_bytes,
                               int *blocks_per_cu) {
  if (records && wave)
    return lds_doms ? occupancy_variant<true, true, true>(block, lds_bytes, blocks_per_cu)
                    : occupancy_variant<true, true, false>(block, lds_bytes, blocks_per_cu);
  if (records)
    return lds_doms ? occupancy_variant<true, false, true>(block, lds_bytes, blocks_per_cu)
                    : occupancy_variant<true, false, false>(block, lds_bytes, blocks_per_cu);
  if (wave)
    return lds_doms ? occupancy_variant<false, true, true>(block, lds_bytes, blocks_per_cu)
                    : occupancy_variant<false, true, false>(block, lds_bytes, blocks_per_cu);
  return lds_doms ? occupancy_variant<false, false, true>(block, lds_bytes, blocks_per_cu)
                  : occupancy_variant<false, false, false>(block, lds_bytes, blocks_per_cu);
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

hipError_t launch_dom_weights(const DevHit *hits, const unsigned long long *hit_count,
                              unsigned long long hit_capacity, double *sums, uint32_t n_doms, hipStream_t stream) {
  if (n_doms == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3(min((2u * n_doms + 255u) / 256u, 1024u)), dim3(256), 0, stream,
                     reinterpret_cast<uint32_t *>(sums), 2u * n_doms);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (n_doms <= 8192) {
    hipLaunchKernelGGL(k_dom_weights<true>, dim3(256), dim3(256), n_doms * sizeof(double), stream, hits,
                       hit_count, hit_capacity, sums, n_doms);
  } else {
    hipLaunchKernelGGL(k_dom_weights<false>, dim3(256), dim3(256), 0, stream, hits, hit_count, hit_capacity,
                       sums, n_doms);
  }
  return hipGetLastError();
}

}  // namespace pp

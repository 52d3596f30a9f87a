// Internal interface between the host library (pp_api.cpp) and the gfx950
// kernels (pp_kernels.hip): device-side table layouts and kernel arguments.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pp {

// Per-layer coefficients, staged into LDS: {a = 1/lambda_a, b = 1/lambda_s,
// 1/a, 1/b} (a reciprocal is +inf where the coefficient is 0) and the
// Henyey-Greenstein constants {1 - g, 1 - g^2, 2 g, 0}.
struct DevLayer {
  float4 coef;
  float4 hg;
};

// Per-string search data, staged into LDS. Modules of string s sit at
// positions first .. first + n - 1 of the sorted module array, ordered by
// z. If the string is evenly spaced (spacing 1/inv_dz within a tolerance)
// the modules a segment can reach are found arithmetically, widened by
// kpad slots; otherwise inv_dz = 0 and kpad = n cover the whole string.
struct DevString {
  float4 xy_reach_z0;  // centre x, centre y, reach + 0.01 m margin, z of slot 0
  float inv_dz, kpad;
  int first, n;
};

// Light source as the kernel reads it (one record per submitted source).
struct DevSource {
  float4 pos_t0;      // start point, emission time
  float4 dir_len;     // unit direction (+z for point sources), segment length (0 for points)
  float4 emit;        // 1 - cos(cone angle) (0 for points), fixed wavelength (0 if spread),
                      // 1/lambda_min, 1/lambda_min - 1/lambda_max
  uint4 ids;          // type, event id, particle id, 0
  unsigned long long first_index;  // photon index of local photon 0
  unsigned long long seq_base;     // submission-order number of local photon 0
};

// Work queue entry: photons [local, local + count) of source src.
struct DevChunk {
  uint32_t src, count;
  unsigned long long local;
};

// Device hit record, bit-compatible with pp_hit.
struct DevHit {
  unsigned long long photon_index;
  uint32_t event_id, particle_id, dom_id;
  float time_ns, weight;
  uint32_t reserved;
};

// Counters, zeroed before each propagation.
enum Counter {
  kChunkNext = 0,
  kHitCount,
  kStatPhotons,
  kStatIterations,
  kStatCrossings,
  kStatDomTests,
  kStatHits,
  kStatAbsorbed,
  kStatCapped,
  kStatEscaped,
  kNumCounters
};

struct Records {  // terminal records, structure of arrays (null if off)
  uint32_t *fate, *dom, *n_iter, *n_cross;
  float *t, *x, *y, *z, *vx, *vy, *vz, *wavelength;
};

constexpr int kMaxPoly = 8;          // coefficients of the angular acceptance polynomial
constexpr int kMaxAcceptance = 256;  // points of the wavelength acceptance table

struct PropagateArgs {
  // ice: layer table and the n_layers + 1 boundary heights (first -inf,
  // last +inf, so the edge layers extend to infinity)
  const DevLayer *layers;
  const float *bounds;
  int n_layers;
  float z_lo, inv_dz;
  float time_per_m;  // n_group / c
  // geometry: grid cell word = nearest string (low 16 bits, 0xFFFF none) |
  // upper half of the float clearance to every other string (rounded down)
  const DevString *strings;
  int n_strings;
  const uint32_t *cells;
  int nx, ny;
  float gx0, gy0, inv_cell, nx_max, ny_max;  // nx_max = nx - 1 as float
  const float4 *doms;  // sorted by string then z: x, y, z, module id (as bits)
  int n_doms;
  int lds_doms;        // 1: every string is vertical; the kernel stages each module's (z, id) in LDS
  float radius, radius2;
  // work
  const DevSource *sources;
  const DevChunk *chunks;
  uint32_t n_chunks;
  uint32_t seed_lo, seed_hi;
  uint32_t step_cap;
  uint32_t refill_interval;
  // wavelength dependence: a photon of wavelength l sees the layer
  // coefficients scaled by (l * inv_lambda_ref)^-kappa (kappas 0: none)
  float inv_lambda_ref, kappa_abs, kappa_scat;
  // hit acceptance (n_acc 0: weight 1): table at acc_l0 + k / inv_acc_dl,
  // linear between points, times sum_k poly[k] c^k, c = cosine of incidence
  const float *acc;
  uint32_t n_acc, n_poly;
  float acc_l0, inv_acc_dl;
  float poly[kMaxPoly];
  const float4 *doms_by_id;  // module centres by module id
  float inv_radius;
  // debug records draw each photon's wavelength even when nothing else
  // needs it (0: records come from the variant that runs without them)
  int records_wavelength;
  // outputs
  unsigned long long *counters;
  DevHit *hits;
  unsigned long long hit_capacity;
  Records rec;
};

// Dynamic LDS bytes the propagation kernel needs for these tables, plus
// n_lds_doms staged (z, id) module records (8 bytes each, 8-byte aligned).
size_t propagate_lds_bytes(int n_layers, int n_strings, int n_cells, int n_lds_doms);
// Largest dynamic LDS a propagation launch may use (modules are staged in
// LDS only if everything fits).
constexpr size_t kMaxPropagateLds = 152 * 1024;

hipError_t launch_reset(unsigned long long *counters, int n, hipStream_t stream);
hipError_t launch_propagate(const PropagateArgs &args, int grid, int block, hipStream_t stream);
// records: debug records on; wave: the kernel variant that draws
// wavelengths (wavelength-dependent optics, hit acceptance, or records that
// ask for the wavelength).
hipError_t propagate_occupancy(bool records, bool wave, bool lds_doms, int block, size_t lds_bytes,
                               int *blocks_per_cu);
hipError_t launch_dom_histogram(const DevHit *hits, const unsigned long long *hit_count,
                                unsigned long long hit_capacity, uint32_t *counts, uint32_t n_doms,
                                hipStream_t stream);
hipError_t launch_dom_weights(const DevHit *hits, const unsigned long long *hit_count,
                              unsigned long long hit_capacity, double *sums, uint32_t n_doms, hipStream_t stream);

}  // namespace pp

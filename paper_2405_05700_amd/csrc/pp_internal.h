// Internal definitions shared by the host-side translation units of libpp
// (pp_api.cpp and sur_api.cpp): the context, its batches, and helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/pp.h"
#include "pp_device.h"

struct pp_surrogate;

namespace ppi {

constexpr uint32_t kMaxLayers = 1024;
constexpr uint32_t kMaxStrings = 512;
constexpr uint32_t kGridSide = 64;  // at most 64 x 64 cells
constexpr double kGridMargin = 1.0;
constexpr double kClearanceMargin = 0.02;
constexpr uint64_t kDefaultStepCap = 100000;

struct Batch {
  std::vector<pp::DevSource> src;
  uint64_t n_photons = 0;
  pp::DevSource *d_src = nullptr;
  pp::DevChunk *d_chunks = nullptr;
  uint32_t n_chunks = 0, chunk_size = 0;
  unsigned long long *d_counters = nullptr;
  pp::DevHit *d_hits = nullptr;
  uint64_t hit_cap = 0;
  void *d_rec = nullptr;
  pp::Records rec{};
  bool propagated = false, rec_valid = false, rec_wavelength = false;
  bool hits_complete = false;  // hit count checked against the buffer since the last propagation
  // results generation of the context in which a propagation's hits were
  // found to fit the buffer (0: never). Hits depend only on the sources and
  // on that state, so a later propagation in the same generation fits too.
  uint64_t fits_gen = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t ev_use = nullptr;  // after the last other enqueued work that reads the batch's buffers
  pp_launch_config used{};
  hipGraphExec_t graph = nullptr;  // captured reset + propagation, if any
  pp_launch_config graph_cfg{};
  bool graph_records = false, graph_rec_wavelength = false;
};

}  // namespace ppi

struct pp_context {
  int device = -1;
  uint64_t seed = 0;
  std::string err;
  pp_launch_config cfg{};
  uint64_t step_cap = ppi::kDefaultStepCap;
  // bumped by every call that can change what a propagation produces (ice,
  // geometry, step cap, optics, acceptance)
  uint64_t results_gen = 1;
  bool records = false;
  bool records_wavelength = false;  // records from the wavelength-drawing kernel variant
  int n_cu = 0;
  // ice
  bool ice_loaded = false;
  pp_ice_header ice{};
  std::vector<pp::DevLayer> layers;
  std::vector<float> bounds;
  pp::DevLayer *d_layers = nullptr;
  float *d_bounds = nullptr;
  // geometry
  bool geo_loaded = false;
  uint32_t n_doms = 0;
  float radius = 0;
  std::vector<pp::DevString> strings;
  std::vector<uint32_t> cells;
  std::vector<float4> doms_sorted;
  pp_geometry_info geo{};
  pp::DevString *d_strings = nullptr;
  uint32_t *d_cells = nullptr;
  float4 *d_doms = nullptr;
  float4 *d_doms_by_id = nullptr;  // module centres in module-id order
  bool vertical_strings = false;   // every module sits exactly at its string's (x, y) centre
  // wavelength dependence and hit acceptance
  pp_chromatic chroma{};           // lambda_ref_nm 0: none
  std::vector<float> acc_table, acc_poly;
  float acc_l0 = 0, acc_dl = 1;
  float *d_acc = nullptr;
  // caching allocator of batch buffers: blocks up to kPoolMaxBlock bytes in
  // power-of-two size classes, reused instead of freed (hipFree waits for
  // the whole device), up to kPoolCacheBytes cached
  std::map<size_t, std::vector<void *>> pool_free;
  std::map<void *, size_t> pool_live;
  size_t pool_cached = 0;
  // batches
  std::map<uint64_t, ppi::Batch> batches;
  uint64_t next_batch = 1;
};


namespace ppi {
// Default device hit-buffer size (hits) for a batch of n photons.
inline uint64_t default_hit_capacity(uint64_t n_photons) {
  return n_photons / 64 > 65536 ? n_photons / 64 : 65536;
}
// Upper bound on the device bytes a batch allocates (records off): source
// records, work-queue chunks of at least `chunk` ids, counters, hit buffer.
inline uint64_t batch_device_bytes(uint64_t n_sources, uint64_t n_photons, uint64_t chunk,
                                   uint64_t hit_capacity) {
  return 80 * n_sources + 16 * (n_sources + n_photons / chunk + 1) + 8 * 16 + 32 * hit_capacity;
}
// Launch shape of one propagation: workgroup size, workgroups (before the
// clamp to the number of work chunks), photon ids per chunk, and whether the
// modules' (z, id) pairs are staged in LDS.
struct LaunchShape {
  uint32_t block, grid, chunk;
  bool lds_doms;
};
// Shape for n_photons photons under the context's launch configuration.
pp_status launch_shape(pp_context *ctx, uint64_t n_photons, bool records, LaunchShape *out);
uint32_t clamp_grid(uint32_t grid, uint32_t block, uint64_t n_chunks);
// Kernel arguments that come from the context (ice, geometry, optics, seed,
// step cap); work, counters and outputs are left for the caller.
void fill_args(const pp_context *ctx, const LaunchShape &shape, pp::PropagateArgs *out);
// Work-queue entries of at most chunk photon ids, source by source.
void split_chunks(const std::vector<pp::DevSource> &src, uint64_t n_photons, uint32_t chunk,
                  std::vector<pp::DevChunk> *out);
bool wants_wavelength(const pp_context *ctx);
// Looks up the device address of pp_propagate_static's scratch array on the
// current device (once per device).
hipError_t static_scratch_setup(int device);
// Expected hits of every (source, module) pair of a batch that need not be
// registered with the context (host records b.src, device records b.d_src),
// source-major into host memory out (b.src.size() x n_doms floats).
pp_status sur_predict_batch(pp_surrogate *s, Batch &b, float *out);
pp_status fail(pp_context *ctx, pp_status st, const char *fmt, ...);
pp_status need_device(pp_context *ctx);
pp_status find_batch(pp_context *ctx, uint64_t id, Batch **out);
pp_status complete_hits(pp_context *ctx, Batch &b, uint64_t *n_total);
pp_status build_sources(const pp_source *src, uint32_t n, std::vector<pp::DevSource> *out, uint64_t *total,
                        std::string *err);
bool finite(float v);
}  // namespace ppi

#define PP_HIP(ctx, expr)                                                                   \
  do {                                                                                      \
    const hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                                   \
      return fail((ctx), e_ == hipErrorOutOfMemory ? PP_ENOMEM : PP_EDEVICE, "%s: %s", #expr, \
                  hipGetErrorString(e_));                                                   \
  } while (0)

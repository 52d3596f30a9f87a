// pp_propagate_static: one propagation that allocates no device memory.
//
// The call's sources, its work queue and its counters live in `scratch`, a
// file-scope device array of fixed size (each GPU the library runs on holds
// its own copy until the process ends); the caller brings the hit buffer.
// The array's device address is looked up once per device, in pp_create with
// that device current, and only that address is used from host code: the
// array's name in host code is a host-side stand-in, not a device address.
// The propagation itself is the same kernel pp_propagate launches, so the
// hits are the same.

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/pp.h"
#include "pp_device.h"
#include "pp_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;
constexpr size_t kCounterOff = 0;
constexpr size_t kSourceOff = 256;
constexpr size_t kChunkOff = kSourceOff + sizeof(pp::DevSource) * PP_STATIC_MAX_SOURCES;
constexpr uint64_t kMaxChunks = (kScratchBytes - kChunkOff) / sizeof(pp::DevChunk);
static_assert(sizeof(unsigned long long) * pp::kNumCounters <= kSourceOff, "counters overlap the sources");
static_assert(kChunkOff % 256 == 0 && kChunkOff < kScratchBytes, "scratch layout");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_scratch[kMaxDevices];  // device address of `scratch` on each device; null until looked up

}  // namespace

namespace ppi {

// Looks up this device's address of the scratch array (the device must be
// current). Called by pp_create; later calls on the same device return at once.
hipError_t static_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (g_scratch[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[device] = p;
  return hipSuccess;
}

static unsigned char *static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mutex);
  return static_cast<unsigned char *>(g_scratch[device]);
}

}  // namespace ppi

using namespace ppi;

extern "C" pp_status pp_propagate_static(pp_context *ctx, const pp_source *sources, uint32_t n_sources,
                                         pp_hit *dev_hits, uint64_t hit_cap, uint64_t *n_total, pp_stats *stats,
                                         void *hip_stream) {
  if (!ctx) return PP_EINVAL;
  if (!n_total || (n_sources > 0 && !sources) || (hit_cap > 0 && !dev_hits))
    return fail(ctx, PP_EINVAL, "null argument");
  *n_total = 0;
  if (!ctx->ice_loaded || !ctx->geo_loaded) return fail(ctx, PP_ESTATE, "load ice and geometry first");
  if (ctx->records)
    return fail(ctx, PP_ESTATE, "debug records need per-photon device memory; turn them off for this call");
  if (n_sources > PP_STATIC_MAX_SOURCES)
    return fail(ctx, PP_EINVAL, "%u sources: this call takes at most %u", n_sources, PP_STATIC_MAX_SOURCES);
  pp_status st = need_device(ctx);
  if (st != PP_OK) return st;
  unsigned char *base = static_scratch(ctx->device);
  if (!base) return fail(ctx, PP_EDEVICE, "no scratch address for device %d", ctx->device);

  // Host staging, reused by the calling thread.
  thread_local std::vector<pp::DevSource> src;
  thread_local std::vector<pp::DevChunk> chunks;
  uint64_t total = 0;
  std::string err;
  if (build_sources(sources, n_sources, &src, &total, &err) != PP_OK) return fail(ctx, PP_EINVAL, "%s", err.c_str());
  LaunchShape shape;
  if ((st = launch_shape(ctx, total, false, &shape)) != PP_OK) return st;
  // Larger chunks until the queue fits the scratch (at most n_sources +
  // total / chunk entries).
  uint64_t chunk = shape.chunk;
  while (n_sources + total / chunk + 1 > kMaxChunks) chunk *= 2;
  if (chunk > 0x80000000ull) return fail(ctx, PP_EINVAL, "photon count too large for the static work queue");
  shape.chunk = static_cast<uint32_t>(chunk);
  split_chunks(src, total, shape.chunk, &chunks);
  const uint32_t grid = clamp_grid(shape.grid, shape.block, chunks.size());

  pp::PropagateArgs a;
  fill_args(ctx, shape, &a);
  a.sources = reinterpret_cast<const pp::DevSource *>(base + kSourceOff);
  a.chunks = reinterpret_cast<const pp::DevChunk *>(base + kChunkOff);
  a.n_chunks = static_cast<uint32_t>(chunks.size());
  a.counters = reinterpret_cast<unsigned long long *>(base + kCounterOff);
  a.hits = reinterpret_cast<pp::DevHit *>(dev_hits);
  a.hit_capacity = hit_cap;

  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  if (!src.empty())
    PP_HIP(ctx, hipMemcpyAsync(base + kSourceOff, src.data(), sizeof(pp::DevSource) * src.size(),
                               hipMemcpyHostToDevice, stream));
  if (!chunks.empty())
    PP_HIP(ctx, hipMemcpyAsync(base + kChunkOff, chunks.data(), sizeof(pp::DevChunk) * chunks.size(),
                               hipMemcpyHostToDevice, stream));
  PP_HIP(ctx, pp::launch_reset(a.counters, pp::kNumCounters, stream));
  if (a.n_chunks > 0) PP_HIP(ctx, pp::launch_propagate(a, static_cast<int>(grid), static_cast<int>(shape.block), stream));
  unsigned long long c[pp::kNumCounters];
  PP_HIP(ctx, hipMemcpyAsync(c, a.counters, sizeof c, hipMemcpyDeviceToHost, stream));
  PP_HIP(ctx, hipStreamSynchronize(stream));

  *n_total = c[pp::kHitCount];
  if (stats) {
    *stats = pp_stats{};
    stats->photons = c[pp::kStatPhotons];
    stats->iterations = c[pp::kStatIterations];
    stats->layer_crossings = c[pp::kStatCrossings];
    stats->dom_tests = c[pp::kStatDomTests];
    stats->hits = c[pp::kStatHits];
    stats->absorbed = c[pp::kStatAbsorbed];
    stats->capped = c[pp::kStatCapped];
    stats->escaped = c[pp::kStatEscaped];
    stats->kernel_ms = 0.0f;
    stats->block_size = shape.block;
    stats->grid_blocks = grid;
    stats->chunk_size = shape.chunk;
    stats->refill_interval = a.refill_interval;
  }
  if (*n_total > hit_cap)
    return fail(ctx, PP_ETRUNC, "%llu hits, buffer holds %llu", static_cast<unsigned long long>(*n_total),
                static_cast<unsigned long long>(hit_cap));
  return PP_OK;
}

// Host side of the C ABI declared in include/pp.h: validation, geometry
// indexing (string table and horizontal search grid), device memory, the
// photon work queue and kernel launches.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/pp.h"
#include "pp_device.h"
#include "pp_internal.h"

std::string g_create_error;

namespace ppi {

pp_status fail(pp_context *ctx, pp_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  ctx->err = buf;
  return st;
}


bool finite(float v) { return std::isfinite(v); }

pp_status need_device(pp_context *ctx) {
  if (ctx->device < 0) return fail(ctx, PP_EDEVICE, "host-only context has no device");
  PP_HIP(ctx, hipSetDevice(ctx->device));
  return PP_OK;
}

template <class T>
pp_status upload(pp_context *ctx, T **dptr, const std::vector<T> &host) {
  if (*dptr) {
    (void)hipFree(*dptr);
    *dptr = nullptr;
  }
  if (host.empty()) return PP_OK;
  PP_HIP(ctx, hipMalloc(reinterpret_cast<void **>(dptr), sizeof(T) * host.size()));
  PP_HIP(ctx, hipMemcpy(*dptr, host.data(), sizeof(T) * host.size(), hipMemcpyHostToDevice));
  return PP_OK;
}

constexpr size_t kPoolMinBlock = 4096;
constexpr size_t kPoolMaxBlock = size_t(256) << 20;
constexpr size_t kPoolCacheBytes = size_t(8) << 30;

// Device memory for a batch buffer: a cached block of the request's
// power-of-two size class if one is free, else a new one. Requests above
// kPoolMaxBlock get their own allocation.
pp_status pool_alloc(pp_context *ctx, void **out, size_t bytes) {
  bytes = std::max<size_t>(bytes, 1);
  size_t cls = bytes;
  if (bytes <= kPoolMaxBlock) {
    cls = kPoolMinBlock;
    while (cls < bytes) cls <<= 1;
    auto it = ctx->pool_free.find(cls);
    if (it != ctx->pool_free.end() && !it->second.empty()) {
      *out = it->second.back();
      it->second.pop_back();
      ctx->pool_cached -= cls;
      ctx->pool_live[*out] = cls;
      return PP_OK;
    }
  }
  hipError_t e = hipMalloc(out, cls);
  if (e != hipSuccess && ctx->pool_cached > 0) {  // give the cache back and try once more
    for (auto &kv : ctx->pool_free)
      for (void *p : kv.second) (void)hipFree(p);
    ctx->pool_free.clear();
    ctx->pool_cached = 0;
    e = hipMalloc(out, cls);
  }
  if (e != hipSuccess) {
    *out = nullptr;
    return fail(ctx, PP_ENOMEM, "device allocation of %zu bytes: %s", cls, hipGetErrorString(e));
  }
  ctx->pool_live[*out] = cls;
  return PP_OK;
}

// Returns a block to the cache (or frees it). The caller guarantees that no
// enqueued work still uses it.
void pool_free(pp_context *ctx, void *p) {
  if (!p) return;
  auto it = ctx->pool_live.find(p);
  if (it == ctx->pool_live.end()) {
    (void)hipFree(p);
    return;
  }
  const size_t cls = it->second;
  ctx->pool_live.erase(it);
  if (cls > kPoolMaxBlock || ctx->pool_cached + cls > kPoolCacheBytes) {
    (void)hipFree(p);
    return;
  }
  ctx->pool_free[cls].push_back(p);
  ctx->pool_cached += cls;
}

template <class T>
pp_status pool_upload(pp_context *ctx, T **dptr, const std::vector<T> &host) {
  pool_free(ctx, *dptr);
  *dptr = nullptr;
  if (host.empty()) return PP_OK;
  void *p = nullptr;
  pp_status st = pool_alloc(ctx, &p, sizeof(T) * host.size());
  if (st != PP_OK) return st;
  *dptr = static_cast<T *>(p);
  PP_HIP(ctx, hipMemcpy(*dptr, host.data(), sizeof(T) * host.size(), hipMemcpyHostToDevice));
  return PP_OK;
}

// Records that work enqueued on stream reads the batch's buffers, so that
// releasing the batch waits for it.
pp_status note_use(pp_context *ctx, Batch &b, hipStream_t stream) {
  if (!b.ev_use) PP_HIP(ctx, hipEventCreateWithFlags(&b.ev_use, hipEventDisableTiming));
  PP_HIP(ctx, hipEventRecord(b.ev_use, stream));
  return PP_OK;
}

void drop_graph(Batch &b) {
  if (b.graph) (void)hipGraphExecDestroy(b.graph);
  b.graph = nullptr;
}

void free_batch(pp_context *ctx, Batch &b) {
  if (b.ev1) (void)hipEventSynchronize(b.ev1);
  if (b.ev_use) (void)hipEventSynchronize(b.ev_use);
  drop_graph(b);
  pool_free(ctx, b.d_src);
  pool_free(ctx, b.d_chunks);
  pool_free(ctx, b.d_counters);
  pool_free(ctx, b.d_hits);
  pool_free(ctx, b.d_rec);
  if (b.ev0) (void)hipEventDestroy(b.ev0);
  if (b.ev1) (void)hipEventDestroy(b.ev1);
  if (b.ev_use) (void)hipEventDestroy(b.ev_use);
  b = Batch{};
}

pp_status find_batch(pp_context *ctx, uint64_t id, Batch **out) {
  auto it = ctx->batches.find(id);
  if (it == ctx->batches.end()) return fail(ctx, PP_EINVAL, "unknown batch %llu", (unsigned long long)id);
  *out = &it->second;
  return PP_OK;
}

uint32_t default_block() { return 256; }
uint32_t default_chunk() { return 256; }
uint32_t default_refill_interval() { return 4; }

// Horizontal distance from the rectangle [x0,x1] x [y0,y1] to the point.
double rect_point_distance(double x0, double x1, double y0, double y1, double px, double py) {
  const double dx = px < x0 ? x0 - px : (px > x1 ? px - x1 : 0.0);
  const double dy = py < y0 ? y0 - py : (py > y1 ? py - y1 : 0.0);
  return std::hypot(dx, dy);
}

// Builds the string table, the z-sorted module array and the search grid.
// Grid cell word: low 16 bits = the string nearest to the cell (tested for
// every photon starting there), high 16 bits = floor(16 * (clearance -
// margin)), where clearance is a lower bound on the horizontal distance
// from any point of the cell to the reach cylinder of any other string
// (0xFFFF = no other string).
void build_geometry(pp_context *ctx, const pp_dom *doms, uint32_t n, float radius,
                    const std::vector<uint32_t> &string_keys) {
  ctx->strings.clear();
  ctx->cells.clear();
  ctx->doms_sorted.clear();
  ctx->vertical_strings = true;
  std::map<uint32_t, std::vector<uint32_t>> by_string;
  for (uint32_t k = 0; k < n; ++k) by_string[doms[k].string_id].push_back(k);
  std::vector<double> cx, cy, reach;
  for (auto &kv : by_string) {
    std::vector<uint32_t> &ids = kv.second;
    std::sort(ids.begin(), ids.end(), [&](uint32_t a, uint32_t b) {
      return doms[a].z < doms[b].z || (doms[a].z == doms[b].z && a < b);
    });
    double sx = 0, sy = 0;
    for (uint32_t k : ids) sx += doms[k].x, sy += doms[k].y;
    sx /= ids.size();
    sy /= ids.size();
    double rmax = 0;
    for (uint32_t k : ids) rmax = std::max(rmax, std::hypot(doms[k].x - sx, doms[k].y - sy));
    const double rch = rmax + radius;
    pp::DevString st{};
    const int m = static_cast<int>(ids.size());
    const double z0 = doms[ids[0]].z;
    st.first = static_cast<int>(ctx->doms_sorted.size());
    st.n = m;
    st.inv_dz = 0.0f;
    st.kpad = static_cast<float>(m);
    if (m >= 2) {
      const double dz = (static_cast<double>(doms[ids[m - 1]].z) - z0) / (m - 1);
      double tol = 0;
      for (int k = 0; k < m; ++k)
        tol = std::max(tol, std::fabs(doms[ids[k]].z - (z0 + k * dz)));
      if (dz > 0 && tol <= 0.25 * dz) {
        st.inv_dz = static_cast<float>(1.0 / dz);
        st.kpad = static_cast<float>(tol / dz + 1.0);
      }
    }
    // the kernel's horizontal reach test carries a 0.01 m margin for FP32
    // rounding of positions up to a few km
    st.xy_reach_z0 = make_float4(static_cast<float>(sx), static_cast<float>(sy),
                                 static_cast<float>(rch + 0.01), static_cast<float>(z0));
    for (uint32_t k : ids)
      if (doms[k].x != st.xy_reach_z0.x || doms[k].y != st.xy_reach_z0.y) ctx->vertical_strings = false;
    for (uint32_t k : ids) {
      uint32_t bits = k;
      float fid;
      std::memcpy(&fid, &bits, 4);
      ctx->doms_sorted.push_back(make_float4(doms[k].x, doms[k].y, doms[k].z, fid));
    }
    ctx->strings.push_back(st);
    cx.push_back(sx);
    cy.push_back(sy);
    reach.push_back(rch);
  }
  (void)string_keys;
  const size_t S = ctx->strings.size();
  pp_geometry_info &gi = ctx->geo;
  gi = pp_geometry_info{};
  gi.n_doms = n;
  gi.n_strings = static_cast<uint32_t>(S);
  double max_reach = 0;
  for (double r : reach) max_reach = std::max(max_reach, r);
  gi.max_reach_m = static_cast<float>(max_reach);
  if (S == 0) {
    gi.grid_nx = gi.grid_ny = 1;
    gi.cell_m = 1.0f;
    ctx->cells.push_back(0x7F80FFFFu);  // no string, infinite clearance
    return;
  }
  double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
  for (size_t s = 0; s < S; ++s) {
    x0 = std::min(x0, cx[s] - reach[s]);
    x1 = std::max(x1, cx[s] + reach[s]);
    y0 = std::min(y0, cy[s] - reach[s]);
    y1 = std::max(y1, cy[s] + reach[s]);
  }
  x0 -= kGridMargin, x1 += kGridMargin, y0 -= kGridMargin, y1 += kGridMargin;
  const double cell = std::max(std::max(x1 - x0, y1 - y0) / kGridSide, 1.0);
  const uint32_t nx = std::min<uint32_t>(kGridSide, static_cast<uint32_t>(std::ceil((x1 - x0) / cell)));
  const uint32_t ny = std::min<uint32_t>(kGridSide, static_cast<uint32_t>(std::ceil((y1 - y0) / cell)));
  // The grid origin and cell are rounded to float first so that the host
  // cell rectangles are the ones the kernel indexes.
  const float fx0 = static_cast<float>(x0), fy0 = static_cast<float>(y0);
  const float fcell = static_cast<float>(cell);
  gi.grid_nx = nx;
  gi.grid_ny = ny;
  gi.grid_x0_m = fx0;
  gi.grid_y0_m = fy0;
  gi.cell_m = fcell;
  ctx->cells.assign(static_cast<size_t>(nx) * ny, 0);
  for (uint32_t iy = 0; iy < ny; ++iy) {
    for (uint32_t ix = 0; ix < nx; ++ix) {
      const double rx0 = fx0 + static_cast<double>(fcell) * ix, rx1 = rx0 + fcell;
      const double ry0 = fy0 + static_cast<double>(fcell) * iy, ry1 = ry0 + fcell;
      double best = std::numeric_limits<double>::infinity(), second = best;
      uint32_t s1 = 0;
      for (size_t s = 0; s < S; ++s) {
        const double d = std::max(0.0, rect_point_distance(rx0, rx1, ry0, ry1, cx[s], cy[s]) - reach[s]);
        if (d < best) {
          second = best;
          best = d;
          s1 = static_cast<uint32_t>(s);
        } else if (d < second) {
          second = d;
        }
      }
      // clearance stored as the upper half of its float (truncation rounds
      // a positive value down, so the bound stays conservative)
      const float clr = std::isfinite(second)
                            ? static_cast<float>(std::max(0.0, second - kClearanceMargin))
                            : std::numeric_limits<float>::infinity();
      uint32_t bits;
      std::memcpy(&bits, &clr, 4);
      ctx->cells[static_cast<size_t>(iy) * nx + ix] = (bits & 0xFFFF0000u) | s1;
    }
  }
}

pp_status build_chunks(pp_context *ctx, Batch &b, uint32_t chunk) {
  if (b.d_chunks && b.chunk_size == chunk) return PP_OK;
  std::vector<pp::DevChunk> ch;
  split_chunks(b.src, b.n_photons, chunk, &ch);
  if (ch.size() >= 0xFFFFFFFFull) return fail(ctx, PP_EINVAL, "too many work chunks; raise chunk_size");
  drop_graph(b);
  pp_status st = pool_upload(ctx, &b.d_chunks, ch);
  if (st != PP_OK) return st;
  b.n_chunks = static_cast<uint32_t>(ch.size());
  b.chunk_size = chunk;
  return PP_OK;
}

pp_status alloc_hits(pp_context *ctx, Batch &b, uint64_t cap) {
  drop_graph(b);
  pool_free(ctx, b.d_hits);
  b.d_hits = nullptr;
  b.hit_cap = 0;
  void *p = nullptr;
  pp_status st = pool_alloc(ctx, &p, sizeof(pp::DevHit) * std::max<uint64_t>(cap, 1));
  if (st != PP_OK) return st;
  b.d_hits = static_cast<pp::DevHit *>(p);
  b.hit_cap = cap;
  return PP_OK;
}

pp_status alloc_records(pp_context *ctx, Batch &b) {
  if (b.d_rec) return PP_OK;
  const uint64_t n = std::max<uint64_t>(b.n_photons, 1);
  pp_status st = pool_alloc(ctx, &b.d_rec, 48 * n);
  if (st != PP_OK) return st;
  char *base = static_cast<char *>(b.d_rec);
  uint32_t **u[] = {&b.rec.fate, &b.rec.dom, &b.rec.n_iter, &b.rec.n_cross};
  float **f[] = {&b.rec.t, &b.rec.x, &b.rec.y, &b.rec.z, &b.rec.vx, &b.rec.vy, &b.rec.vz, &b.rec.wavelength};
  for (int i = 0; i < 4; ++i) *u[i] = reinterpret_cast<uint32_t *>(base + 4 * n * i);
  for (int i = 0; i < 8; ++i) *f[i] = reinterpret_cast<float *>(base + 4 * n * (4 + i));
  return PP_OK;
}

struct Prepared {
  pp::PropagateArgs args;
  uint32_t grid, block;
  pp_launch_config used;
};

bool wants_wavelength(const pp_context *ctx) {
  return (ctx->chroma.lambda_ref_nm > 0 && (ctx->chroma.kappa_abs != 0.0f || ctx->chroma.kappa_scat != 0.0f)) ||
         !ctx->acc_table.empty();
}

pp_status launch_shape(pp_context *ctx, uint64_t n_photons, bool records, LaunchShape *out) {
  const pp_launch_config &c = ctx->cfg;
  // With vertical strings each module's (z, id) joins the LDS tables when
  // everything fits; a CU then holds fewer workgroups, so the default
  // workgroup grows to keep 24 wavefronts per CU.
  const int n_layers = static_cast<int>(ctx->ice.n_layers), n_strings = static_cast<int>(ctx->strings.size());
  const int n_cells = static_cast<int>(ctx->geo.grid_nx * ctx->geo.grid_ny);
  const size_t with_doms = pp::propagate_lds_bytes(n_layers, n_strings, n_cells, static_cast<int>(ctx->n_doms));
  const bool lds_doms = ctx->n_doms > 0 && ctx->vertical_strings && with_doms <= pp::kMaxPropagateLds;
  const size_t lds = lds_doms ? with_doms : pp::propagate_lds_bytes(n_layers, n_strings, n_cells, 0);
  uint32_t block = c.block_size;
  if (block == 0) {
    const size_t per_cu = std::max<size_t>(1, (160 * 1024) / std::max<size_t>(lds, 1));
    const size_t waves = (24 + per_cu - 1) / per_cu;
    block = static_cast<uint32_t>(std::min<size_t>(1024, std::max<size_t>(default_block(), 64 * waves)));
  }
  uint32_t grid = c.grid_blocks;
  if (grid == 0) {
    int per_cu = 0;
    const bool wave = wants_wavelength(ctx) || (records && ctx->records_wavelength);
    PP_HIP(ctx, pp::propagate_occupancy(records, wave, lds_doms, static_cast<int>(block), lds, &per_cu));
    grid = static_cast<uint32_t>(std::max(per_cu, 1) * std::max(ctx->n_cu, 1));
  }
  // Default chunk: 256 ids (measured best on the full detector), smaller
  // for small batches so that every resident wavefront gets several chunks.
  uint32_t chunk = c.chunk_size;
  if (chunk == 0) {
    const uint64_t waves = static_cast<uint64_t>(grid) * (block / 64);
    chunk = static_cast<uint32_t>(std::min<uint64_t>(default_chunk(),
                                                     std::max<uint64_t>(64, n_photons / (waves * 8) + 1)));
  }
  out->block = block;
  out->grid = grid;
  out->chunk = chunk;
  out->lds_doms = lds_doms;
  return PP_OK;
}

uint32_t clamp_grid(uint32_t grid, uint32_t block, uint64_t n_chunks) {
  // no more workgroups than there are chunks to share among their wavefronts
  return static_cast<uint32_t>(
      std::min<uint64_t>(grid, std::max<uint64_t>(1, (n_chunks * 64 + block - 1) / block)));
}

void fill_args(const pp_context *ctx, const LaunchShape &shape, pp::PropagateArgs *out) {
  const pp_launch_config &c = ctx->cfg;
  pp::PropagateArgs a{};
  a.layers = ctx->d_layers;
  a.bounds = ctx->d_bounds;
  a.n_layers = static_cast<int>(ctx->ice.n_layers);
  a.z_lo = ctx->ice.z_lo_m;
  a.inv_dz = static_cast<float>(1.0 / ctx->ice.dz_m);
  a.time_per_m = static_cast<float>(static_cast<double>(ctx->ice.n_group) / 0.299792458);
  a.strings = ctx->d_strings;
  a.n_strings = static_cast<int>(ctx->strings.size());
  a.cells = ctx->d_cells;
  a.nx = static_cast<int>(ctx->geo.grid_nx);
  a.ny = static_cast<int>(ctx->geo.grid_ny);
  a.gx0 = ctx->geo.grid_x0_m;
  a.gy0 = ctx->geo.grid_y0_m;
  a.inv_cell = 1.0f / ctx->geo.cell_m;
  a.nx_max = static_cast<float>(a.nx - 1);
  a.ny_max = static_cast<float>(a.ny - 1);
  a.doms = ctx->d_doms;
  a.n_doms = static_cast<int>(ctx->n_doms);
  a.lds_doms = shape.lds_doms ? 1 : 0;
  a.radius = ctx->radius;
  a.radius2 = ctx->radius * ctx->radius;
  a.seed_lo = static_cast<uint32_t>(ctx->seed);
  a.seed_hi = static_cast<uint32_t>(ctx->seed >> 32);
  a.step_cap = static_cast<uint32_t>(ctx->step_cap);
  a.refill_interval = c.refill_interval ? c.refill_interval : default_refill_interval();
  const bool chroma = ctx->chroma.lambda_ref_nm > 0;
  a.inv_lambda_ref = chroma ? 1.0f / ctx->chroma.lambda_ref_nm : 1.0f;
  a.kappa_abs = chroma ? ctx->chroma.kappa_abs : 0.0f;
  a.kappa_scat = chroma ? ctx->chroma.kappa_scat : 0.0f;
  a.n_acc = static_cast<uint32_t>(ctx->acc_table.size());
  a.acc = ctx->d_acc;
  a.acc_l0 = ctx->acc_l0;
  a.inv_acc_dl = 1.0f / ctx->acc_dl;
  a.n_poly = static_cast<uint32_t>(ctx->acc_poly.size());
  for (uint32_t k = 0; k < a.n_poly; ++k) a.poly[k] = ctx->acc_poly[k];
  a.doms_by_id = ctx->d_doms_by_id;
  a.inv_radius = 1.0f / ctx->radius;
  *out = a;
}

void split_chunks(const std::vector<pp::DevSource> &src, uint64_t n_photons, uint32_t chunk,
                  std::vector<pp::DevChunk> *out) {
  out->clear();
  for (uint32_t s = 0; s < src.size(); ++s) {
    const uint64_t begin = src[s].seq_base;
    const uint64_t total = (s + 1 < src.size() ? src[s + 1].seq_base : n_photons) - begin;
    for (uint64_t l = 0; l < total; l += chunk) {
      pp::DevChunk c{};
      c.src = s;
      c.count = static_cast<uint32_t>(std::min<uint64_t>(chunk, total - l));
      c.local = l;
      out->push_back(c);
    }
  }
}

// Allocates what the batch needs for the context's launch configuration and
// fills the kernel arguments. No work is enqueued.
pp_status prepare(pp_context *ctx, Batch &b, Prepared *out) {
  const pp_launch_config &c = ctx->cfg;
  LaunchShape shape;
  pp_status st = launch_shape(ctx, b.n_photons, ctx->records, &shape);
  if (st != PP_OK) return st;
  if ((st = build_chunks(ctx, b, shape.chunk)) != PP_OK) return st;
  const uint32_t grid = clamp_grid(shape.grid, shape.block, b.n_chunks);
  if (!b.d_counters) {
    void *p = nullptr;
    if ((st = pool_alloc(ctx, &p, sizeof(unsigned long long) * pp::kNumCounters)) != PP_OK) return st;
    b.d_counters = static_cast<unsigned long long *>(p);
  }
  if (!b.d_hits) {
    const uint64_t cap = c.hit_capacity ? c.hit_capacity : default_hit_capacity(b.n_photons);
    st = alloc_hits(ctx, b, cap);
    if (st != PP_OK) return st;
  }
  if (ctx->records) {
    st = alloc_records(ctx, b);
    if (st != PP_OK) return st;
  }
  if (!b.ev0) PP_HIP(ctx, hipEventCreate(&b.ev0));
  if (!b.ev1) PP_HIP(ctx, hipEventCreate(&b.ev1));

  pp::PropagateArgs a;
  fill_args(ctx, shape, &a);
  a.sources = b.d_src;
  a.chunks = b.d_chunks;
  a.n_chunks = b.n_chunks;
  a.counters = b.d_counters;
  a.hits = b.d_hits;
  a.hit_capacity = b.hit_cap;
  if (ctx->records) {
    a.rec = b.rec;
    a.records_wavelength = ctx->records_wavelength ? 1 : 0;
  }

  out->args = a;
  out->grid = grid;
  out->block = shape.block;
  out->used = c;
  out->used.block_size = shape.block;
  out->used.chunk_size = shape.chunk;
  out->used.grid_blocks = grid;
  out->used.refill_interval = a.refill_interval;
  out->used.hit_capacity = b.hit_cap;
  return PP_OK;
}

// Counter reset and the propagation kernel on the stream (what a graph
// captures).
pp_status enqueue(pp_context *ctx, Batch &b, const Prepared &p, hipStream_t stream) {
  PP_HIP(ctx, pp::launch_reset(b.d_counters, pp::kNumCounters, stream));
  if (b.n_chunks > 0)
    PP_HIP(ctx, pp::launch_propagate(p.args, static_cast<int>(p.grid), static_cast<int>(p.block), stream));
  return PP_OK;
}

void mark_propagated(Batch &b, const pp_launch_config &used, bool records, bool rec_wavelength,
                     hipStream_t stream) {
  b.stream = stream;
  b.propagated = true;
  b.rec_valid = records;
  b.rec_wavelength = records && rec_wavelength;
  b.hits_complete = false;
  b.used = used;
}

pp_status launch(pp_context *ctx, Batch &b, hipStream_t stream) {
  Prepared p;
  pp_status st = prepare(ctx, b, &p);
  if (st != PP_OK) return st;
  PP_HIP(ctx, hipEventRecord(b.ev0, stream));
  if ((st = enqueue(ctx, b, p, stream)) != PP_OK) return st;
  PP_HIP(ctx, hipEventRecord(b.ev1, stream));
  mark_propagated(b, p.used, ctx->records, ctx->records_wavelength, stream);
  return PP_OK;
}

pp_status sync_counters(pp_context *ctx, Batch &b, unsigned long long *host) {
  if (!b.propagated) return fail(ctx, PP_ESTATE, "batch not propagated");
  PP_HIP(ctx, hipEventSynchronize(b.ev1));
  PP_HIP(ctx, hipMemcpy(host, b.d_counters, sizeof(unsigned long long) * pp::kNumCounters,
                        hipMemcpyDeviceToHost));
  return PP_OK;
}

// Makes sure the device hit buffer holds every hit of the batch (rerunning
// with a larger buffer if it overflowed) and returns the hit count.
pp_status complete_hits(pp_context *ctx, Batch &b, uint64_t *n_total) {
  unsigned long long cnt[pp::kNumCounters];
  pp_status st = sync_counters(ctx, b, cnt);
  if (st != PP_OK) return st;
  if (cnt[pp::kHitCount] > b.hit_cap) {
    const uint64_t need = cnt[pp::kHitCount];
    st = alloc_hits(ctx, b, need + need / 8 + 1024);
    if (st != PP_OK) return st;
    const pp_launch_config saved = ctx->cfg;
    const bool saved_rec = ctx->records, saved_wave = ctx->records_wavelength;
    ctx->cfg = b.used;
    ctx->cfg.hit_capacity = 0;
    ctx->records = b.rec_valid;
    ctx->records_wavelength = b.rec_wavelength;
    st = launch(ctx, b, b.stream);
    ctx->cfg = saved;
    ctx->records = saved_rec;
    ctx->records_wavelength = saved_wave;
    if (st != PP_OK) return st;
    st = sync_counters(ctx, b, cnt);
    if (st != PP_OK) return st;
    if (cnt[pp::kHitCount] != need)
      return fail(ctx, PP_EDEVICE, "rerun after hit-buffer overflow gave %llu hits, expected %llu",
                  cnt[pp::kHitCount], (unsigned long long)need);
  }
  *n_total = cnt[pp::kHitCount];
  b.hits_complete = true;
  b.fits_gen = ctx->results_gen;
  return PP_OK;
}

// Makes the batch's complete hit buffer visible to work enqueued next on
// stream: if the buffer could have overflowed and no propagation of the
// batch under the same results-affecting state has been checked to fit it,
// checks the count (synchronising the batch's stream and rerunning on
// overflow); then orders stream after the propagation.
pp_status hits_ready_on(pp_context *ctx, Batch &b, hipStream_t stream) {
  if (!b.propagated) return fail(ctx, PP_ESTATE, "batch not propagated");
  if (!b.hits_complete && b.hit_cap < b.n_photons && b.fits_gen != ctx->results_gen) {
    uint64_t n = 0;
    pp_status st = complete_hits(ctx, b, &n);
    if (st != PP_OK) return st;
  }
  PP_HIP(ctx, hipStreamWaitEvent(stream, b.ev1, 0));
  return PP_OK;
}

}  // namespace ppi

namespace ppi {

// Validates submitted sources and converts them to device records. Pure
// (touches no context), so the server's client threads can call it.
pp_status build_sources(const pp_source *src, uint32_t n, std::vector<pp::DevSource> *out, uint64_t *total_out,
                        std::string *err) {
  char buf[256];
  auto bad = [&](const char *fmt, uint32_t i, uint32_t v = 0) {
    std::snprintf(buf, sizeof buf, fmt, i, v);
    *err = buf;
    return PP_EINVAL;
  };
  out->assign(n, pp::DevSource{});
  uint64_t total = 0;
  std::vector<std::pair<std::pair<uint32_t, uint64_t>, uint64_t>> ranges;
  for (uint32_t i = 0; i < n; ++i) {
    const pp_source &s = src[i];
    if (s.type != PP_SOURCE_POINT && s.type != PP_SOURCE_CHERENKOV)
      return bad("source %u: unknown type %u", i, s.type);
    if (!finite(s.x) || !finite(s.y) || !finite(s.z) || !finite(s.t0_ns))
      return bad("source %u: non-finite position or time", i);
    if (!finite(s.lambda_min_nm) || !finite(s.lambda_max_nm) || !(s.lambda_min_nm > 0) ||
        s.lambda_min_nm > s.lambda_max_nm)
      return bad("source %u: need 0 < lambda_min <= lambda_max", i);
    if (s.first_photon_index + s.n_photons < s.first_photon_index)
      return bad("source %u: photon index range overflows", i);
    if (total + s.n_photons < total) return bad("source %u: photon count overflows", i);
    pp::DevSource &d = (*out)[i];
    double dx = 0, dy = 0, dz = 1, len = 0, om = 0;
    if (s.type == PP_SOURCE_CHERENKOV) {
      if (!finite(s.dx) || !finite(s.dy) || !finite(s.dz) || !finite(s.length_m) || !(s.length_m >= 0) ||
          !finite(s.cherenkov_deg) || !(s.cherenkov_deg > 0 && s.cherenkov_deg < 180))
        return bad("source %u: bad direction, length or Cherenkov angle", i);
      const double nrm = std::sqrt(static_cast<double>(s.dx) * s.dx + static_cast<double>(s.dy) * s.dy +
                                   static_cast<double>(s.dz) * s.dz);
      if (!(std::fabs(nrm - 1.0) <= 1e-3)) return bad("source %u: |direction| not within 1e-3 of 1", i);
      dx = s.dx / nrm, dy = s.dy / nrm, dz = s.dz / nrm;
      len = s.length_m;
      const double half = 0.5 * s.cherenkov_deg * M_PI / 180.0;
      om = 2.0 * std::sin(half) * std::sin(half);  // 1 - cos(angle) without cancellation
    }
    d.pos_t0 = make_float4(s.x, s.y, s.z, s.t0_ns);
    d.dir_len = make_float4(static_cast<float>(dx), static_cast<float>(dy), static_cast<float>(dz),
                            static_cast<float>(len));
    const double inv_min = 1.0 / s.lambda_min_nm, inv_max = 1.0 / s.lambda_max_nm;
    const bool fixed = s.lambda_min_nm == s.lambda_max_nm;
    d.emit = make_float4(static_cast<float>(om), fixed ? s.lambda_min_nm : 0.0f,
                         static_cast<float>(inv_min), fixed ? 0.0f : static_cast<float>(inv_min - inv_max));
    d.ids = make_uint4(s.type, s.event_id, s.particle_id, 0u);
    d.first_index = s.first_photon_index;
    d.seq_base = total;
    total += s.n_photons;
    if (s.n_photons > 0) ranges.push_back({{s.event_id, s.first_photon_index}, s.n_photons});
  }
  std::sort(ranges.begin(), ranges.end());
  for (size_t i = 1; i < ranges.size(); ++i) {
    const auto &p = ranges[i - 1], &q = ranges[i];
    if (p.first.first == q.first.first && q.first.second < p.first.second + p.second)
      return bad("overlapping photon-index ranges in event %u", q.first.first);
  }
  *total_out = total;
  return PP_OK;
}

}  // namespace ppi

using namespace ppi;

extern "C" {

pp_status pp_create(int hip_device, uint64_t seed, pp_context **out) {
  if (!out) return PP_EINVAL;
  *out = nullptr;
  if (hip_device < -1) {
    g_create_error = "hip_device must be >= -1";
    return PP_EINVAL;
  }
  pp_context *ctx = new (std::nothrow) pp_context;
  if (!ctx) return PP_ENOMEM;
  ctx->device = hip_device;
  ctx->seed = seed;
  if (hip_device >= 0) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || hip_device >= count) {
      g_create_error = std::string("no HIP device ") + std::to_string(hip_device) + ": " +
                       (e != hipSuccess ? hipGetErrorString(e) : "index out of range");
      delete ctx;
      return PP_EDEVICE;
    }
    hipDeviceProp_t prop;
    e = hipSetDevice(hip_device);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, hip_device);
    if (e != hipSuccess) {
      g_create_error = hipGetErrorString(e);
      delete ctx;
      return PP_EDEVICE;
    }
    ctx->n_cu = prop.multiProcessorCount;
    e = static_scratch_setup(hip_device);
    if (e != hipSuccess) {
      g_create_error = std::string("scratch of pp_propagate_static: ") + hipGetErrorString(e);
      delete ctx;
      return PP_EDEVICE;
    }
  }
  *out = ctx;
  return PP_OK;
}

void pp_destroy(pp_context *ctx) {
  if (!ctx) return;
  if (ctx->device >= 0) {
    (void)hipSetDevice(ctx->device);
    for (auto &kv : ctx->batches) free_batch(ctx, kv.second);
    for (auto &kv : ctx->pool_free)
      for (void *p : kv.second) (void)hipFree(p);
    (void)hipFree(ctx->d_layers);
    (void)hipFree(ctx->d_bounds);
    (void)hipFree(ctx->d_strings);
    (void)hipFree(ctx->d_cells);
    (void)hipFree(ctx->d_doms);
    (void)hipFree(ctx->d_doms_by_id);
    (void)hipFree(ctx->d_acc);
  }
  delete ctx;
}

const char *pp_last_error(const pp_context *ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

pp_status pp_set_launch_config(pp_context *ctx, const pp_launch_config *cfg) {
  if (!ctx || !cfg) return PP_EINVAL;
  if (cfg->block_size != 0 && (cfg->block_size % 64 != 0 || cfg->block_size > 1024))
    return fail(ctx, PP_EINVAL, "block_size must be a multiple of 64 in 64..1024");
  ctx->cfg = *cfg;
  return PP_OK;
}

pp_status pp_get_launch_config(const pp_context *ctx, pp_launch_config *cfg) {
  if (!ctx || !cfg) return PP_EINVAL;
  *cfg = ctx->cfg;
  if (!cfg->block_size) cfg->block_size = default_block();
  if (!cfg->chunk_size) cfg->chunk_size = default_chunk();
  if (!cfg->refill_interval) cfg->refill_interval = default_refill_interval();
  return PP_OK;
}

pp_status pp_set_step_cap(pp_context *ctx, uint64_t step_cap) {
  if (!ctx) return PP_EINVAL;
  if (step_cap > (1ull << 31)) return fail(ctx, PP_EINVAL, "step_cap above 2^31");
  ctx->step_cap = step_cap;
  ++ctx->results_gen;
  return PP_OK;
}

pp_status pp_set_chromatic(pp_context *ctx, const pp_chromatic *c) {
  if (!ctx) return PP_EINVAL;
  ++ctx->results_gen;
  if (!c) {
    ctx->chroma = pp_chromatic{};
    return PP_OK;
  }
  if (!finite(c->lambda_ref_nm) || !(c->lambda_ref_nm > 0) || !finite(c->kappa_abs) || !finite(c->kappa_scat) ||
      std::fabs(c->kappa_abs) > 10.0f || std::fabs(c->kappa_scat) > 10.0f)
    return fail(ctx, PP_EINVAL, "lambda_ref_nm must be finite and > 0, exponents finite with |kappa| <= 10");
  ctx->chroma = *c;
  return PP_OK;
}

pp_status pp_set_acceptance(pp_context *ctx, const pp_acceptance *acc) {
  if (!ctx) return PP_EINVAL;
  ++ctx->results_gen;
  if (!acc) {
    ctx->acc_table.clear();
    ctx->acc_poly.clear();
    return PP_OK;
  }
  if (acc->n_table < 1 || acc->n_table > static_cast<uint32_t>(pp::kMaxAcceptance) || !acc->table)
    return fail(ctx, PP_EINVAL, "n_table must be 1..%d with a table", pp::kMaxAcceptance);
  if (acc->n_poly < 1 || acc->n_poly > static_cast<uint32_t>(pp::kMaxPoly) || !acc->poly)
    return fail(ctx, PP_EINVAL, "n_poly must be 1..%d with coefficients", pp::kMaxPoly);
  if (!finite(acc->lambda0_nm) || !finite(acc->dlambda_nm) || (acc->n_table > 1 && !(acc->dlambda_nm > 0)))
    return fail(ctx, PP_EINVAL, "lambda0_nm must be finite and dlambda_nm finite and > 0");
  for (uint32_t k = 0; k < acc->n_table; ++k)
    if (!finite(acc->table[k]) || acc->table[k] < 0)
      return fail(ctx, PP_EINVAL, "acceptance %u must be finite and >= 0", k);
  for (uint32_t k = 0; k < acc->n_poly; ++k)
    if (!finite(acc->poly[k])) return fail(ctx, PP_EINVAL, "coefficient %u is not finite", k);
  std::vector<float> table(acc->table, acc->table + acc->n_table);
  if (ctx->device >= 0) {
    pp_status st = need_device(ctx);
    if (st != PP_OK) return st;
    if ((st = upload(ctx, &ctx->d_acc, table)) != PP_OK) return st;
  }
  ctx->acc_table = std::move(table);
  ctx->acc_poly.assign(acc->poly, acc->poly + acc->n_poly);
  ctx->acc_l0 = acc->lambda0_nm;
  ctx->acc_dl = acc->n_table > 1 ? acc->dlambda_nm : 1.0f;
  return PP_OK;
}

pp_status pp_set_debug_records(pp_context *ctx, int mode) {
  if (!ctx) return PP_EINVAL;
  if (mode != PP_RECORDS_OFF && mode != PP_RECORDS_ON && mode != PP_RECORDS_PRODUCTION)
    return fail(ctx, PP_EINVAL, "records mode %d is not PP_RECORDS_OFF, _ON or _PRODUCTION", mode);
  ctx->records = mode != PP_RECORDS_OFF;
  ctx->records_wavelength = mode == PP_RECORDS_ON;
  return PP_OK;
}

pp_status pp_load_ice(pp_context *ctx, const pp_ice_header *h, const pp_ice_layer *layers) {
  if (!ctx || !h || (!layers && h->n_layers)) return ctx ? fail(ctx, PP_EINVAL, "null argument") : PP_EINVAL;
  if (h->n_layers < 1 || h->n_layers > kMaxLayers)
    return fail(ctx, PP_EINVAL, "n_layers %u outside 1..%u", h->n_layers, kMaxLayers);
  if (!finite(h->z_lo_m) || !finite(h->dz_m) || !(h->dz_m > 0))
    return fail(ctx, PP_EINVAL, "z_lo_m and dz_m must be finite with dz_m > 0");
  if (!finite(h->n_group) || !(h->n_group > 0)) return fail(ctx, PP_EINVAL, "n_group must be finite and > 0");
  std::vector<pp::DevLayer> L(h->n_layers);
  for (uint32_t i = 0; i < h->n_layers; ++i) {
    const pp_ice_layer &l = layers[i];
    if (!(l.abs_len_m > 0) || !(l.eff_scat_len_m > 0))
      return fail(ctx, PP_EINVAL, "layer %u: lengths must be > 0 (NaN rejected)", i);
    if (!finite(l.g) || !(l.g > -1.0f && l.g < 1.0f))
      return fail(ctx, PP_EINVAL, "layer %u: g must lie in (-1, 1)", i);
    const double g = l.g;
    const double a = 1.0 / static_cast<double>(l.abs_len_m);
    const double b = 1.0 / (static_cast<double>(l.eff_scat_len_m) * (1.0 - g));
    const float inf = std::numeric_limits<float>::infinity();
    L[i].coef = make_float4(static_cast<float>(a), static_cast<float>(b),
                            a > 0 ? static_cast<float>(1.0 / a) : inf,
                            b > 0 ? static_cast<float>(1.0 / b) : inf);
    L[i].hg = make_float4(static_cast<float>(1.0 - g), static_cast<float>(1.0 - g * g),
                          static_cast<float>(2.0 * g), 0.0f);
  }
  // boundary heights: bounds[i] is the bottom of layer i; the edge layers
  // extend to infinity
  std::vector<float> B(h->n_layers + 1);
  for (uint32_t i = 0; i <= h->n_layers; ++i)
    B[i] = static_cast<float>(static_cast<double>(h->z_lo_m) + static_cast<double>(i) * h->dz_m);
  B[0] = -std::numeric_limits<float>::infinity();
  B[h->n_layers] = std::numeric_limits<float>::infinity();
  if (ctx->device >= 0) {
    pp_status st = need_device(ctx);
    if (st != PP_OK) return st;
    if ((st = upload(ctx, &ctx->d_layers, L)) != PP_OK) return st;
    if ((st = upload(ctx, &ctx->d_bounds, B)) != PP_OK) return st;
  }
  ctx->ice = *h;
  ctx->layers = std::move(L);
  ctx->bounds = std::move(B);
  ctx->ice_loaded = true;
  ++ctx->results_gen;
  return PP_OK;
}

pp_status pp_load_geometry(pp_context *ctx, const pp_dom *doms, uint32_t n, float radius) {
  if (!ctx) return PP_EINVAL;
  if (n > 0 && !doms) return fail(ctx, PP_EINVAL, "null doms");
  if (n > (1u << 24)) return fail(ctx, PP_EINVAL, "more than 2^24 modules");
  if (!finite(radius) || !(radius > 0)) return fail(ctx, PP_EINVAL, "dom_radius_m must be finite and > 0");
  std::vector<std::pair<uint64_t, uint32_t>> keys(n);
  std::vector<uint32_t> strings;
  for (uint32_t k = 0; k < n; ++k) {
    if (!finite(doms[k].x) || !finite(doms[k].y) || !finite(doms[k].z))
      return fail(ctx, PP_EINVAL, "module %u: non-finite position", k);
    keys[k] = {(static_cast<uint64_t>(doms[k].string_id) << 32) | doms[k].om_index, k};
    strings.push_back(doms[k].string_id);
  }
  std::sort(keys.begin(), keys.end());
  for (uint32_t k = 1; k < n; ++k)
    if (keys[k].first == keys[k - 1].first)
      return fail(ctx, PP_EINVAL, "modules %u and %u share (string_id, om_index)", keys[k - 1].second, keys[k].second);
  std::sort(strings.begin(), strings.end());
  strings.erase(std::unique(strings.begin(), strings.end()), strings.end());
  if (strings.size() > kMaxStrings)
    return fail(ctx, PP_EINVAL, "%zu strings; at most %u", strings.size(), kMaxStrings);
  build_geometry(ctx, doms, n, radius, strings);
  ctx->n_doms = n;
  ctx->radius = radius;
  if (ctx->device >= 0) {
    pp_status st = need_device(ctx);
    if (st != PP_OK) return st;
    if ((st = upload(ctx, &ctx->d_strings, ctx->strings)) != PP_OK) return st;
    if ((st = upload(ctx, &ctx->d_cells, ctx->cells)) != PP_OK) return st;
    if ((st = upload(ctx, &ctx->d_doms, ctx->doms_sorted)) != PP_OK) return st;
    std::vector<float4> by_id(n);
    for (uint32_t k = 0; k < n; ++k) by_id[k] = make_float4(doms[k].x, doms[k].y, doms[k].z, 0.0f);
    if ((st = upload(ctx, &ctx->d_doms_by_id, by_id)) != PP_OK) return st;
  }
  ctx->geo_loaded = true;
  ++ctx->results_gen;
  return PP_OK;
}

pp_status pp_get_geometry_info(const pp_context *ctx, pp_geometry_info *out) {
  if (!ctx || !out) return PP_EINVAL;
  if (!ctx->geo_loaded) return PP_ESTATE;
  *out = ctx->geo;
  return PP_OK;
}

pp_status pp_geometry_cell(const pp_context *ctx, float x, float y, uint32_t *nearest, float *clearance) {
  if (!ctx || !nearest || !clearance) return PP_EINVAL;
  if (!ctx->geo_loaded) return PP_ESTATE;
  const pp_geometry_info &g = ctx->geo;
  const float inv = 1.0f / g.cell_m;
  const float fx = std::fmin(std::fmax((x - g.grid_x0_m) * inv, 0.0f), static_cast<float>(g.grid_nx - 1));
  const float fy = std::fmin(std::fmax((y - g.grid_y0_m) * inv, 0.0f), static_cast<float>(g.grid_ny - 1));
  const uint32_t word = ctx->cells[static_cast<size_t>(fy) * g.grid_nx + static_cast<size_t>(fx)];
  const uint32_t s1 = word & 0xFFFFu, hi = word & 0xFFFF0000u;
  *nearest = s1 == 0xFFFFu ? 0xFFFFFFFFu : s1;
  std::memcpy(clearance, &hi, 4);
  return PP_OK;
}

pp_status pp_submit(pp_context *ctx, const pp_source *src, uint32_t n, uint64_t *batch_out) {
  if (!ctx || !batch_out || (n > 0 && !src)) return ctx ? fail(ctx, PP_EINVAL, "null argument") : PP_EINVAL;
  if (!ctx->ice_loaded || !ctx->geo_loaded) return fail(ctx, PP_ESTATE, "load ice and geometry before submitting");
  Batch b;
  uint64_t total = 0;
  std::string err;
  if (build_sources(src, n, &b.src, &total, &err) != PP_OK) return fail(ctx, PP_EINVAL, "%s", err.c_str());
  b.n_photons = total;
  if (ctx->device >= 0) {
    pp_status st = need_device(ctx);
    if (st != PP_OK) return st;
    st = pool_upload(ctx, &b.d_src, b.src);
    if (st != PP_OK) {
      free_batch(ctx, b);
      return st;
    }
  }
  const uint64_t id = ctx->next_batch++;
  ctx->batches.emplace(id, std::move(b));
  *batch_out = id;
  return PP_OK;
}

pp_status pp_release(pp_context *ctx, uint64_t batch) {
  if (!ctx) return PP_EINVAL;
  Batch *b;
  pp_status st = find_batch(ctx, batch, &b);
  if (st != PP_OK) return st;
  if (ctx->device >= 0) (void)hipSetDevice(ctx->device);
  free_batch(ctx, *b);
  ctx->batches.erase(batch);
  return PP_OK;
}

pp_status pp_propagate(pp_context *ctx, uint64_t batch, void *hip_stream) {
  if (!ctx) return PP_EINVAL;
  Batch *b;
  pp_status st = find_batch(ctx, batch, &b);
  if (st != PP_OK) return st;
  if ((st = need_device(ctx)) != PP_OK) return st;
  return launch(ctx, *b, static_cast<hipStream_t>(hip_stream));
}

pp_status pp_hit_count(pp_context *ctx, uint64_t batch, uint64_t *n_total) {
  if (!ctx || !n_total) return PP_EINVAL;
  Batch *b;
  pp_status st = find_batch(ctx, batch, &b);
  if (st != PP_OK) return st;
  if ((st = need_device(ctx)) != PP_OK) return st;
  return complete_hits(ctx, *b, n_total);
}

pp_status pp_fetch_hits(pp_context *ctx, uint64_t batch, pp_hit *out, uint64_t cap, uint64_t *n_total) {
  if (!ctx || !n_total || (cap > 0 && !out)) return PP_EINVAL;
  Batch *b;
  pp_status st = find_batch(ctx, batch, &b);
  if (st != PP_OK) return st;
  if ((st = need_device(ctx)) != PP_OK) return st;
  uint64_t n = 0;
  if ((st = complete_hits(ctx, *b, &n)) != PP_OK) return st;
  *n_total = n;
  const uint64_t m = std::min(n, cap);
  if (m > 0) PP_HIP(ctx, hipMemcpy(out, b->d_hits, sizeof(pp_hit) * m, hipMemcpyDeviceToHost));
  return n > cap ? fail(ctx, PP_ETRUNC, "%llu hits, buffer holds %llu", (unsigned long long)n,
                        (unsigned long long)cap)
                 : PP_OK;
}

pp_status pp_fetch_hits_device(pp_context *ctx, uint64_t batch, void *dev_out, uint64_t cap, uint64_t *n_total,
                               void *hip_stream) {
  if (!ctx || !n_total || (cap > 0 && !dev_out)) return PP_EINVAL;
  Batch *b;
  pp_status st = find_batch(ctx, batch, &b);
  if (st != PP_OK) return st;
  if ((st = need_device(ctx)) != PP_OK) return st;
  uint64_t n = 0;
  if ((st = complete_hits(ctx, *b, &n)) != PP_OK) return st;
  *n_total = n;
  const uint64_t m = std::min(n, cap);
  if (m > 0) {
    PP_HIP(ctx, hipMemcpyAsync(dev_out, b->d_hits, sizeof(pp_hit) * m, hipMemcpyDeviceToDevice,
                               static_cast<hipStream_t>(hip_stream)));
    if ((st = note_use(ctx, *b, static_cast<hipStream_t>(hip_stream))) != PP_OK) return st;
  }
  return n > cap ? fail(ctx, PP_ETRUNC, "%llu hits, buffer holds %llu", (unsigned long long)n,
                        (unsigned long long)cap)
                 : PP_OK;
}

pp_status pp_dom_counts(pp_context *ctx, uint64_t batch, uint32_t *dev_counts, void *hip_stream) {
  if (!ctx || (!dev_counts && ctx->n_doms > 0)) return PP_EINVAL;
  Batch *b;
  pp_status st = find_batch(ctx, batch, &b);
  if (st != PP_OK) return st;
  if ((st = need_device(ctx)) != PP_OK) return st;
  if ((st = hits_ready_on(ctx, *b, static_cast<hipStream_t>(hip_stream))) != PP_OK) return st;
  PP_HIP(ctx, pp::launch_dom_histogram(b->d_hits, b->d_counters + pp::kHitCount, b->hit_cap, dev_counts,
                                       ctx->n_doms, static_cast<hipStream_t>(hip_stream)));
  return note_use(ctx, *b, static_cast<hipStream_t>(hip_stream));
}

pp_status pp_sort_hits(pp_hit *hits, uint64_t n) {
  if (n > 0 && !hits) return PP_EINVAL;
  std::sort(hits, hits + n, [](const pp_hit &a, const pp_hit &b) {
    return a.event_id != b.event_id ? a.event_id < b.event_id : a.photon_index < b.photon_index;
  });
  return PP_OK;
}

pp_status pp_dom_weights(pp_context *ctx, uint64_t batch, double *dev_sums, void *hip_stream) {
  if (!ctx || (!dev_sums && ctx->n_doms > 0)) return PP_EINVAL;
  Batch *b;
  pp_status st = find_batch(ctx, batch, &b);
  if (st != PP_OK) return st;
  if ((st = need_device(ctx)) != PP_OK) return st;
  if ((st = hits_ready_on(ctx, *b, static_cast<hipStream_t>(hip_stream))) != PP_OK) return st;
  PP_HIP(ctx, pp::launch_dom_weights(b->d_hits, b->d_counters + pp::kHitCount, b->hit_cap, dev_sums, ctx->n_doms,
                                     static_cast<hipStream_t>(hip_stream)));
  return note_use(ctx, *b, static_cast<hipStream_t>(hip_stream));
}

pp_status pp_fetch_records(pp_context *ctx, uint64_t batch, pp_photon_record *out, uint64_t first,
                           uint64_t count) {
  if (!ctx || (count > 0 && !out)) return PP_EINVAL;
  Batch *b;
  pp_status st = find_batch(ctx, batch, &b);
  if (st != PP_OK) return st;
  if ((st = need_device(ctx)) != PP_OK) return st;
  if (!b->propagated || !b->rec_valid) return fail(ctx, PP_ESTATE, "no records: enable them before pp_propagate");
  if (first > b->n_photons || count > b->n_photons - first) return fail(ctx, PP_EINVAL, "record range out of bounds");
  PP_HIP(ctx, hipEventSynchronize(b->ev1));
  std::vector<uint32_t> u(4 * count);
  std::vector<float> f(8 * count);
  uint32_t *du[] = {b->rec.fate, b->rec.dom, b->rec.n_iter, b->rec.n_cross};
  float *df[] = {b->rec.t, b->rec.x, b->rec.y, b->rec.z, b->rec.vx, b->rec.vy, b->rec.vz, b->rec.wavelength};
  for (int i = 0; i < 4; ++i)
    PP_HIP(ctx, hipMemcpy(u.data() + i * count, du[i] + first, 4 * count, hipMemcpyDeviceToHost));
  for (int i = 0; i < 8; ++i)
    PP_HIP(ctx, hipMemcpy(f.data() + i * count, df[i] + first, 4 * count, hipMemcpyDeviceToHost));
  for (uint64_t k = 0; k < count; ++k) {
    pp_photon_record &r = out[k];
    r.fate = u[k];
    r.dom_id = u[count + k];
    r.n_iter = u[2 * count + k];
    r.n_cross = u[3 * count + k];
    r.time_ns = f[k];
    r.x = f[count + k];
    r.y = f[2 * count + k];
    r.z = f[3 * count + k];
    r.vx = f[4 * count + k];
    r.vy = f[5 * count + k];
    r.vz = f[6 * count + k];
    r.wavelength_nm = f[7 * count + k];
  }
  return PP_OK;
}

pp_status pp_get_stats(pp_context *ctx, uint64_t batch, pp_stats *out) {
  if (!ctx || !out) return PP_EINVAL;
  Batch *b;
  pp_status st = find_batch(ctx, batch, &b);
  if (st != PP_OK) return st;
  if ((st = need_device(ctx)) != PP_OK) return st;
  unsigned long long c[pp::kNumCounters];
  if ((st = sync_counters(ctx, *b, c)) != PP_OK) return st;
  out->photons = c[pp::kStatPhotons];
  out->iterations = c[pp::kStatIterations];
  out->layer_crossings = c[pp::kStatCrossings];
  out->dom_tests = c[pp::kStatDomTests];
  out->hits = c[pp::kStatHits];
  out->absorbed = c[pp::kStatAbsorbed];
  out->capped = c[pp::kStatCapped];
  out->escaped = c[pp::kStatEscaped];
  float ms = 0;
  PP_HIP(ctx, hipEventElapsedTime(&ms, b->ev0, b->ev1));
  out->kernel_ms = ms;
  out->block_size = b->used.block_size;
  out->grid_blocks = b->used.grid_blocks;
  out->chunk_size = b->used.chunk_size;
  out->refill_interval = b->used.refill_interval;
  return PP_OK;
}

pp_status pp_autotune(pp_context *ctx, uint64_t batch, void *hip_stream, pp_launch_config *best) {
  if (!ctx) return PP_EINVAL;
  Batch *b;
  pp_status st = find_batch(ctx, batch, &b);
  if (st != PP_OK) return st;
  if ((st = need_device(ctx)) != PP_OK) return st;
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  const pp_launch_config base = ctx->cfg;
  pp_launch_config winner = base;
  float best_ms = -1.0f;
  const uint32_t blocks[] = {256, 512, 1024};
  const uint32_t chunks[] = {64, 256, 1024};
  const uint32_t refills[] = {2, 4, 8};
  bool first = true;
  for (uint32_t blk : blocks)
    for (uint32_t chk : chunks)
      for (uint32_t rf : refills) {
        pp_launch_config c = base;
        c.block_size = blk;
        c.chunk_size = chk;
        c.refill_interval = rf;
        c.grid_blocks = 0;
        ctx->cfg = c;
        if (first) {  // warm-up (allocations, code load)
          if ((st = launch(ctx, *b, stream)) != PP_OK) break;
          first = false;
        }
        if ((st = launch(ctx, *b, stream)) != PP_OK) break;
        float ms = 0;
        if (hipEventSynchronize(b->ev1) != hipSuccess || hipEventElapsedTime(&ms, b->ev0, b->ev1) != hipSuccess) {
          st = fail(ctx, PP_EDEVICE, "timing failed during autotune");
          break;
        }
        if (best_ms < 0 || ms < best_ms) {
          best_ms = ms;
          winner = c;
        }
      }
  ctx->cfg = st == PP_OK ? winner : base;
  if (st != PP_OK) return st;
  if (best) *best = winner;
  return PP_OK;
}

pp_status pp_graph_capture(pp_context *ctx, uint64_t batch, void *hip_stream) {
  if (!ctx) return PP_EINVAL;
  if (!hip_stream) return fail(ctx, PP_EINVAL, "graph capture needs a non-null stream");
  Batch *b;
  pp_status st = find_batch(ctx, batch, &b);
  if (st != PP_OK) return st;
  if ((st = need_device(ctx)) != PP_OK) return st;
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  Prepared p;
  if ((st = prepare(ctx, *b, &p)) != PP_OK) return st;
  drop_graph(*b);
  PP_HIP(ctx, hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  st = enqueue(ctx, *b, p, stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(stream, &g);
  if (st != PP_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(ctx, PP_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) return fail(ctx, PP_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e2));
  b->graph = exec;
  b->graph_cfg = p.used;
  b->graph_records = ctx->records;
  b->graph_rec_wavelength = ctx->records_wavelength;
  return PP_OK;
}

pp_status pp_graph_launch(pp_context *ctx, uint64_t batch, void *hip_stream) {
  if (!ctx) return PP_EINVAL;
  Batch *b;
  pp_status st = find_batch(ctx, batch, &b);
  if (st != PP_OK) return st;
  if ((st = need_device(ctx)) != PP_OK) return st;
  if (!b->graph) return fail(ctx, PP_ESTATE, "no captured graph for this batch (captured buffers changed?)");
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  PP_HIP(ctx, hipEventRecord(b->ev0, stream));
  PP_HIP(ctx, hipGraphLaunch(b->graph, stream));
  PP_HIP(ctx, hipEventRecord(b->ev1, stream));
  mark_propagated(*b, b->graph_cfg, b->graph_records, b->graph_rec_wavelength, stream);
  return PP_OK;
}

}  // extern "C"

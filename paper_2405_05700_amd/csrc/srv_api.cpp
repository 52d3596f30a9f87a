// Photon server (include/pp_server.h): a multi-producer request queue, a
// device-resident photon queue (rings of source records and work-queue
// entries in an arena allocated once within the HBM budget), and a
// scheduler thread that admits requests into the rings as space frees up
// and keeps up to max_inflight propagation launches in flight on separate
// HIP streams, each over a contiguous window of the queue.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/pp_server.h"
#include "pp_internal.h"

using namespace ppi;

namespace {

constexpr uint32_t kServerChunk = 256;  // photon ids per work-queue entry
constexpr uint64_t kNone = ~uint64_t{0};
constexpr size_t kCounterBlock = 256;   // bytes per launch slot's counters

double now_s() {
  static const auto t0 = std::chrono::steady_clock::now();
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

uint64_t chunks_of(const std::vector<pp::DevSource> &src, uint64_t total) {
  uint64_t n = 0;
  for (size_t i = 0; i < src.size(); ++i) {
    const uint64_t end = i + 1 < src.size() ? src[i + 1].seq_base : total;
    n += (end - src[i].seq_base + kServerChunk - 1) / kServerChunk;
  }
  return n;
}

// Circular buffer of `cap` records handed out as contiguous blocks in
// allocation order; blocks are released in any order and their space is
// reclaimed in allocation order. Positions are absolute counters (record
// index = position % cap); a block that would straddle the end starts at
// the next multiple of cap instead, the skipped records belonging to it.
struct Ring {
  uint64_t cap = 0;
  uint64_t head = 0, tail = 0;                 // [head, tail) is held
  std::deque<std::pair<uint64_t, bool>> held;  // (block end, released) in allocation order

  uint64_t start_for(uint64_t n) const {
    uint64_t start = tail;
    const uint64_t pos = start % cap;
    if (pos + n > cap) start += cap - pos;
    return start;
  }
  bool fits(uint64_t n) const { return n == 0 || (n <= cap && start_for(n) + n - head <= cap); }
  // Reserves n records (fits(n) must hold); returns the start position.
  uint64_t take(uint64_t n) {
    if (n == 0) return tail;
    const uint64_t start = start_for(n);
    tail = start + n;
    held.emplace_back(tail, false);
    return start;
  }
  void release(uint64_t end) {
    for (auto &b : held)
      if (b.first == end) b.second = true;
    while (!held.empty() && held.front().second) {
      head = held.front().first;
      held.pop_front();
    }
  }
};

enum State { kQueued, kResident, kLaunched, kDone };

struct Request {
  std::vector<pp::DevSource> dev;  // device records, seq_base relative to the request
  std::vector<uint32_t> events;    // distinct event ids of the request
  uint64_t photons = 0, chunks = 0, bytes = 0;
  double t_submit = 0, t_launch = 0, t_done = 0;
  State state = kQueued;
  uint64_t src_pos = 0, chunk_pos = 0;          // ring positions while resident
  uint64_t src_end = kNone, chunk_end = kNone;  // ring block ends (kNone: no block)
  pp_status status = PP_OK;
  std::vector<pp_hit> hits;
  std::vector<float> dom_expected;
  uint32_t batch_events = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_end = nullptr;
  unsigned long long *counters = nullptr;
  pp::DevHit *hits = nullptr;
  bool busy = false;
  std::vector<uint64_t> tickets;
  pp::PropagateArgs args{};
  uint32_t grid = 0, block = 0;
  uint64_t first_src = 0, n_src = 0;  // source window (ring positions)
};

}  // namespace

struct pp_server {
  pp_context *ctx = nullptr;
  pp_surrogate *sur = nullptr;
  pp_server_config cfg{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> backlog;   // queued on the host, arrival order
  std::deque<uint64_t> resident;  // in the device rings, not launched, ring order
  std::unordered_map<uint64_t, Request> reqs;
  uint64_t next_ticket = 1;
  pp_server_stats stats{};
  bool stop = false;
  std::string err;
  std::thread th;
  // arena; after creation only the scheduler thread touches the rings' contents
  void *arena = nullptr;
  uint64_t arena_bytes = 0, hit_cap = 0;
  pp::DevSource *d_src = nullptr;
  pp::DevChunk *d_chunks = nullptr;
  pp::DevSource *h_src = nullptr;  // pinned mirrors of the rings (staging of the uploads)
  pp::DevChunk *h_chunks = nullptr;
  Ring src_ring, chunk_ring;  // guarded by mu
  hipStream_t upload = nullptr;
  hipEvent_t ev_upload = nullptr, ev_ref = nullptr;
  std::vector<Slot> slots;
  LaunchShape shape{};
  std::vector<std::pair<double, double>> intervals;  // device intervals of finished launches (ms after ev_ref)
};

namespace {

void set_error(pp_server *s, const std::string &msg) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->err = msg;
}

std::string hip_msg(const char *what, hipError_t e) { return std::string(what) + ": " + hipGetErrorString(e); }

// Copies ring records [pos, pos + n) (never straddling the end) from the
// pinned mirror to the device on the upload stream.
template <class T>
hipError_t upload_range(T *dev, const T *host, uint64_t cap, uint64_t pos, uint64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t i = pos % cap;
  return hipMemcpyAsync(dev + i, host + i, sizeof(T) * n, hipMemcpyHostToDevice, st);
}

// Admission: moves waiting requests, in arrival order, into the rings while
// they fit (a request that does not fit waits, and so do the ones behind
// it, so large events are not starved), stages their records in the pinned
// mirrors and uploads them. Returns true if anything was admitted.
bool admit(pp_server *s) {
  std::vector<uint64_t> admitted;
  std::vector<Request *> rs;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    while (!s->backlog.empty()) {
      const uint64_t tk = s->backlog.front();
      Request &r = s->reqs[tk];
      const uint64_t n_src = r.dev.size();
      if (!s->src_ring.fits(n_src) || !s->chunk_ring.fits(r.chunks)) {
        s->stats.deferred += 1;
        break;
      }
      r.src_pos = s->src_ring.take(n_src);
      r.src_end = n_src ? s->src_ring.tail : kNone;
      r.chunk_pos = s->chunk_ring.take(r.chunks);
      r.chunk_end = r.chunks ? s->chunk_ring.tail : kNone;
      s->stats.bytes_in_use += r.bytes;
      s->stats.peak_bytes_in_use = std::max(s->stats.peak_bytes_in_use, s->stats.bytes_in_use);
      admitted.push_back(tk);
      rs.push_back(&r);  // element references of an unordered_map stay valid until it is erased
      s->backlog.pop_front();
    }
  }
  if (admitted.empty()) return false;
  // Staging and upload: an admitted request is in no launch yet, so nothing
  // in flight reads its ring records.
  const uint64_t scap = s->src_ring.cap, ccap = s->chunk_ring.cap;
  hipError_t e = hipSuccess;
  for (Request *r : rs) {
    for (size_t i = 0; i < r->dev.size(); ++i) s->h_src[(r->src_pos + i) % scap] = r->dev[i];
    uint64_t c = r->chunk_pos;
    for (size_t i = 0; i < r->dev.size(); ++i) {
      const uint64_t begin = r->dev[i].seq_base;
      const uint64_t end = i + 1 < r->dev.size() ? r->dev[i + 1].seq_base : r->photons;
      for (uint64_t l = 0; l < end - begin; l += kServerChunk, ++c) {
        pp::DevChunk &d = s->h_chunks[c % ccap];
        d.src = static_cast<uint32_t>((r->src_pos + i) % scap);
        d.count = static_cast<uint32_t>(std::min<uint64_t>(kServerChunk, end - begin - l));
        d.local = l;
      }
    }
  }
  // One copy per run of admitted blocks that follow one another in a ring
  // without crossing its end (blocks never straddle it), not one per block.
  auto upload_runs = [&](auto *dev, const auto *host, uint64_t cap, auto pos_of, auto count_of) -> hipError_t {
    uint64_t run_pos = 0, run_end = 0;
    for (Request *r : rs) {
      const uint64_t p = pos_of(r), n = count_of(r);
      if (n == 0) continue;
      if (run_end != run_pos && p == run_end && p % cap != 0) {
        run_end += n;
        continue;
      }
      if (run_end != run_pos) {
        const hipError_t u = upload_range(dev, host, cap, run_pos, run_end - run_pos, s->upload);
        if (u != hipSuccess) return u;
      }
      run_pos = p;
      run_end = p + n;
    }
    return run_end != run_pos ? upload_range(dev, host, cap, run_pos, run_end - run_pos, s->upload) : hipSuccess;
  };
  e = upload_runs(s->d_src, s->h_src, scap, [](const Request *r) { return r->src_pos; },
                  [](const Request *r) { return static_cast<uint64_t>(r->dev.size()); });
  if (e == hipSuccess)
    e = upload_runs(s->d_chunks, s->h_chunks, ccap, [](const Request *r) { return r->chunk_pos; },
                    [](const Request *r) { return r->chunks; });
  if (e == hipSuccess) e = hipEventRecord(s->ev_upload, s->upload);
  std::lock_guard<std::mutex> lk(s->mu);
  for (size_t i = 0; i < admitted.size(); ++i) {
    rs[i]->state = kResident;
    s->resident.push_back(admitted[i]);
  }
  if (e != hipSuccess) s->err = hip_msg("queue upload", e);
  return true;
}

// Forms a launch from the resident requests at the front of the queue: a
// run that is contiguous in both rings, one request per event id, within
// the caps on events and photons; enqueues it on the slot's stream after
// the uploads.
bool launch(pp_server *s, Slot &slot) {
  std::vector<uint64_t> take;
  uint64_t first_chunk = 0, n_chunks = 0, first_src = 0, n_src = 0, photons = 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    std::unordered_set<uint32_t> seen;
    while (!s->resident.empty() && take.size() < s->cfg.max_batch_events && photons < s->cfg.max_batch_photons) {
      const Request &r = s->reqs[s->resident.front()];
      bool ok = true;
      for (uint32_t ev : r.events) ok = ok && !seen.count(ev);
      // The run must be one window of each ring: a request that does not
      // follow on directly, or that starts again at the ring's first
      // record, begins the next launch.
      if (r.chunks && n_chunks &&
          (r.chunk_pos != first_chunk + n_chunks || r.chunk_pos % s->chunk_ring.cap == 0))
        ok = false;
      if (!r.dev.empty() && n_src && (r.src_pos != first_src + n_src || r.src_pos % s->src_ring.cap == 0))
        ok = false;
      if (!ok) break;
      if (take.empty() || n_chunks == 0) first_chunk = r.chunk_pos;
      if (take.empty() || n_src == 0) first_src = r.src_pos;
      for (uint32_t ev : r.events) seen.insert(ev);
      n_chunks += r.chunks;
      n_src += r.dev.size();
      photons += r.photons;
      take.push_back(s->resident.front());
      s->resident.pop_front();
    }
    if (take.empty()) return false;
    const double t = now_s();
    for (uint64_t tk : take) {
      Request &r = s->reqs[tk];
      r.state = kLaunched;
      r.t_launch = t;
      r.batch_events = static_cast<uint32_t>(take.size());
    }
    if (take.size() > 1) s->stats.shared_requests += take.size();
    for (const Slot &o : s->slots)
      if (o.busy && &o != &slot) {
        s->stats.overlapped_launches += 1;
        break;
      }
    s->stats.launches += 1;
  }
  slot.busy = true;
  slot.tickets = take;
  slot.first_src = first_src;
  slot.n_src = n_src;
  pp::PropagateArgs &a = slot.args;
  fill_args(s->ctx, s->shape, &a);
  a.sources = s->d_src;
  a.chunks = s->d_chunks + first_chunk % s->chunk_ring.cap;
  a.n_chunks = static_cast<uint32_t>(n_chunks);
  a.counters = slot.counters;
  a.hits = slot.hits;
  a.hit_capacity = s->hit_cap;
  slot.block = s->shape.block;
  slot.grid = clamp_grid(s->shape.grid, s->shape.block, n_chunks);
  hipError_t e = hipStreamWaitEvent(slot.stream, s->ev_upload, 0);
  if (e == hipSuccess) e = hipEventRecord(slot.ev_start, slot.stream);
  if (e == hipSuccess) e = pp::launch_reset(slot.counters, pp::kNumCounters, slot.stream);
  if (e == hipSuccess && n_chunks > 0)
    e = pp::launch_propagate(a, static_cast<int>(slot.grid), static_cast<int>(slot.block), slot.stream);
  if (e == hipSuccess) e = hipEventRecord(slot.ev_end, slot.stream);
  if (e != hipSuccess) set_error(s, hip_msg("launch", e));
  return true;
}

// Finishes a completed launch: hits copied back and split by event id
// (after a rerun into a larger temporary buffer if they overflowed the
// slot's), surrogate expectations if attached, ring space released,
// requests marked done.
void finish(pp_server *s, Slot &slot) {
  pp_context *ctx = s->ctx;
  pp_status st = PP_OK;
  std::string msg;
  unsigned long long cnt[pp::kNumCounters] = {};
  std::vector<pp_hit> hits;
  hipError_t e = hipEventSynchronize(slot.ev_end);
  if (e == hipSuccess) e = hipMemcpy(cnt, slot.counters, sizeof cnt, hipMemcpyDeviceToHost);
  float ms0 = 0, ms1 = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms0, s->ev_ref, slot.ev_start);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms1, s->ev_ref, slot.ev_end);
  const uint64_t n = cnt[pp::kHitCount];
  if (e == hipSuccess && n > s->hit_cap) {
    // overflow: the same launch again into a temporary buffer, if the budget allows
    const uint64_t bytes = sizeof(pp::DevHit) * n;
    if (s->arena_bytes + bytes > s->cfg.hbm_budget_bytes) {
      st = PP_EBUDGET;
      msg = "a launch produced " + std::to_string(n) + " hits: more than its buffer and the budget's remainder hold";
    } else {
      void *tmp = nullptr;
      e = hipMalloc(&tmp, bytes);
      if (e == hipSuccess) {
        pp::PropagateArgs a = slot.args;
        a.hits = static_cast<pp::DevHit *>(tmp);
        a.hit_capacity = n;
        e = pp::launch_reset(slot.counters, pp::kNumCounters, slot.stream);
        if (e == hipSuccess && a.n_chunks > 0)
          e = pp::launch_propagate(a, static_cast<int>(slot.grid), static_cast<int>(slot.block), slot.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(slot.stream);
        if (e == hipSuccess) e = hipMemcpy(cnt, slot.counters, sizeof cnt, hipMemcpyDeviceToHost);
        if (e == hipSuccess && cnt[pp::kHitCount] != n) {
          st = PP_EDEVICE;
          msg = "rerun after hit overflow gave a different hit count";
        }
        if (e == hipSuccess && st == PP_OK) {
          hits.resize(n);
          e = hipMemcpy(hits.data(), tmp, bytes, hipMemcpyDeviceToHost);
        }
        (void)hipFree(tmp);
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.overflow_bytes_peak = std::max<uint64_t>(s->stats.overflow_bytes_peak, bytes);
      }
    }
  } else if (e == hipSuccess && n > 0) {
    hits.resize(n);
    e = hipMemcpy(hits.data(), slot.hits, sizeof(pp_hit) * n, hipMemcpyDeviceToHost);
  }
  if (e != hipSuccess) {
    st = e == hipErrorOutOfMemory ? PP_ENOMEM : PP_EDEVICE;
    msg = hip_msg("finishing a launch", e);
  }
  // surrogate expectations of the launch's sources (a contiguous window of the source ring)
  std::vector<float> pairs;
  std::vector<uint64_t> src_offset;
  if (st == PP_OK && s->sur && slot.n_src > 0) {
    Batch b;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (uint64_t tk : slot.tickets) {
        const Request &r = s->reqs[tk];
        src_offset.push_back(b.src.size());
        for (const pp::DevSource &d : r.dev) {
          pp::DevSource x = d;
          x.seq_base += b.n_photons;
          b.src.push_back(x);
        }
        b.n_photons += r.photons;
      }
    }
    b.d_src = s->d_src + slot.first_src % s->src_ring.cap;
    pairs.resize(b.src.size() * static_cast<size_t>(ctx->n_doms));
    st = sur_predict_batch(s->sur, b, pairs.data());
    if (st != PP_OK) msg = pp_last_error(ctx);
  } else if (s->sur) {
    for (size_t i = 0; i < slot.tickets.size(); ++i) src_offset.push_back(0);
  }
  const double t = now_s();
  std::lock_guard<std::mutex> lk(s->mu);
  std::unordered_map<uint32_t, uint64_t> owner;
  for (uint64_t tk : slot.tickets)
    for (uint32_t ev : s->reqs[tk].events) owner[ev] = tk;
  for (const pp_hit &h : hits) {
    auto it = owner.find(h.event_id);
    if (it != owner.end()) s->reqs[it->second].hits.push_back(h);
  }
  for (size_t i = 0; i < slot.tickets.size(); ++i) {
    Request &r = s->reqs[slot.tickets[i]];
    if (s->sur && st == PP_OK) {
      r.dom_expected.assign(ctx->n_doms, 0.0f);
      for (size_t k = 0; k < r.dev.size() && !pairs.empty(); ++k) {
        const float *row = pairs.data() + (src_offset[i] + k) * ctx->n_doms;
        for (uint32_t d = 0; d < ctx->n_doms; ++d) r.dom_expected[d] += row[d];
      }
    }
    if (r.src_end != kNone) s->src_ring.release(r.src_end);
    if (r.chunk_end != kNone) s->chunk_ring.release(r.chunk_end);
    s->stats.bytes_in_use -= r.bytes;
    r.status = st;
    r.t_done = t;
    r.state = kDone;
    s->stats.completed += 1;
    s->stats.photons_completed += r.photons;
  }
  if (!msg.empty()) s->err = msg;
  if (ms1 > ms0) s->intervals.emplace_back(ms0, ms1);
  slot.busy = false;
  slot.tickets.clear();
  s->cv_done.notify_all();
}

void scheduler(pp_server *s) {
  (void)hipSetDevice(s->ctx->device);
  for (;;) {
    bool progressed = false;
    for (Slot &slot : s->slots)
      if (slot.busy && hipEventQuery(slot.ev_end) != hipErrorNotReady) {
        finish(s, slot);
        progressed = true;
      }
    progressed |= admit(s);
    for (Slot &slot : s->slots)
      if (!slot.busy) {
        if (!launch(s, slot)) break;
        progressed = true;
      }
    std::unique_lock<std::mutex> lk(s->mu);
    bool any_busy = false;
    for (const Slot &slot : s->slots) any_busy |= slot.busy;
    if (s->stop && s->backlog.empty() && s->resident.empty() && !any_busy) break;
    if (!progressed) s->cv_work.wait_for(lk, std::chrono::microseconds(any_busy ? 50 : 2000));
  }
}

void free_arena(pp_server *s) {
  for (Slot &slot : s->slots) {
    if (slot.stream) (void)hipStreamDestroy(slot.stream);
    if (slot.ev_start) (void)hipEventDestroy(slot.ev_start);
    if (slot.ev_end) (void)hipEventDestroy(slot.ev_end);
  }
  if (s->upload) (void)hipStreamDestroy(s->upload);
  if (s->ev_upload) (void)hipEventDestroy(s->ev_upload);
  if (s->ev_ref) (void)hipEventDestroy(s->ev_ref);
  if (s->arena) (void)hipFree(s->arena);
  if (s->h_src) (void)hipHostFree(s->h_src);
  if (s->h_chunks) (void)hipHostFree(s->h_chunks);
}

double union_length(std::vector<std::pair<double, double>> v) {
  std::sort(v.begin(), v.end());
  double total = 0, lo = 0, hi = 0;
  bool open = false;
  for (const auto &x : v) {
    if (!open || x.first > hi) {
      if (open) total += hi - lo;
      lo = x.first;
      hi = x.second;
      open = true;
    } else {
      hi = std::max(hi, x.second);
    }
  }
  if (open) total += hi - lo;
  return total;
}

}  // namespace

extern "C" {

uint64_t pp_server_request_bytes(uint32_t n_sources, uint64_t n_photons) {
  const uint64_t chunks = n_sources + n_photons / kServerChunk;  // upper bound on the entries
  return sizeof(pp::DevSource) * n_sources + sizeof(pp::DevChunk) * chunks;
}

pp_status pp_server_create(pp_context *ctx, const pp_server_config *cfg, pp_surrogate *sur, pp_server **out) {
  if (!ctx || !out) return PP_EINVAL;
  *out = nullptr;
  pp_status st = need_device(ctx);
  if (st != PP_OK) return st;
  if (!ctx->ice_loaded || !ctx->geo_loaded) return fail(ctx, PP_ESTATE, "load ice and geometry first");
  if (ctx->records) return fail(ctx, PP_ESTATE, "the server runs without debug records");
  pp_server_config c = cfg ? *cfg : pp_server_config{};
  if (!c.max_inflight) c.max_inflight = 4;
  if (!c.max_batch_events) c.max_batch_events = 4096;
  if (!c.hbm_budget_bytes) c.hbm_budget_bytes = 200000000000ull;
  if (!c.max_batch_photons) c.max_batch_photons = 200000000ull;
  if (c.max_inflight > 64) return fail(ctx, PP_EINVAL, "at most 64 launches in flight");
  const uint64_t B = c.hbm_budget_bytes;
  const uint64_t hit_cap = std::max<uint64_t>(64, std::min<uint64_t>(uint64_t{1} << 20, B / 4 / c.max_inflight / 32));
  const uint64_t chunk_cap = std::max<uint64_t>(64, std::min<uint64_t>(uint64_t{1} << 22, B / 4 / 16));
  const uint64_t src_cap = std::max<uint64_t>(64, std::min<uint64_t>(uint64_t{1} << 16, B / 16 / 80));
  auto align = [](uint64_t x) { return (x + 255) & ~uint64_t{255}; };
  const uint64_t src_bytes = align(sizeof(pp::DevSource) * src_cap);
  const uint64_t chunk_bytes = align(sizeof(pp::DevChunk) * chunk_cap);
  const uint64_t slot_bytes = kCounterBlock + align(sizeof(pp::DevHit) * hit_cap);
  const uint64_t arena = src_bytes + chunk_bytes + c.max_inflight * slot_bytes;
  if (arena > B)
    return fail(ctx, PP_EBUDGET, "the budget of %llu bytes cannot hold the server's smallest queue (%llu bytes)",
                (unsigned long long)B, (unsigned long long)arena);
  pp_server *s = new (std::nothrow) pp_server;
  if (!s) return PP_ENOMEM;
  s->ctx = ctx;
  s->sur = sur;
  s->cfg = c;
  s->hit_cap = hit_cap;
  s->src_ring.cap = src_cap;
  s->chunk_ring.cap = chunk_cap;
  if ((st = launch_shape(ctx, 0, false, &s->shape)) != PP_OK) {
    delete s;
    return st;
  }
  s->shape.chunk = kServerChunk;
  hipError_t e = hipMalloc(&s->arena, arena);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&s->h_src), sizeof(pp::DevSource) * src_cap);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&s->h_chunks), sizeof(pp::DevChunk) * chunk_cap);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->upload, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_upload, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreate(&s->ev_ref);
  if (e == hipSuccess) {
    char *p = static_cast<char *>(s->arena);
    s->d_src = reinterpret_cast<pp::DevSource *>(p);
    s->d_chunks = reinterpret_cast<pp::DevChunk *>(p + src_bytes);
    char *q = p + src_bytes + chunk_bytes;
    s->slots.resize(c.max_inflight);
    for (Slot &slot : s->slots) {
      slot.counters = reinterpret_cast<unsigned long long *>(q);
      slot.hits = reinterpret_cast<pp::DevHit *>(q + kCounterBlock);
      q += slot_bytes;
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&slot.stream, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreate(&slot.ev_start);
      if (e == hipSuccess) e = hipEventCreate(&slot.ev_end);
    }
  }
  // the device-clock reference of the launch intervals, and a first upload
  // event that the first launches can wait on
  if (e == hipSuccess) e = hipEventRecord(s->ev_ref, s->upload);
  if (e == hipSuccess) e = hipEventRecord(s->ev_upload, s->upload);
  if (e == hipSuccess) e = hipStreamSynchronize(s->upload);
  if (e != hipSuccess) {
    free_arena(s);
    delete s;
    return fail(ctx, e == hipErrorOutOfMemory ? PP_ENOMEM : PP_EDEVICE, "server arena of %llu bytes: %s",
                (unsigned long long)arena, hipGetErrorString(e));
  }
  s->arena_bytes = arena;
  s->stats.arena_bytes = arena;
  s->th = std::thread(scheduler, s);
  *out = s;
  return PP_OK;
}

void pp_server_destroy(pp_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->th.joinable()) s->th.join();
  (void)hipSetDevice(s->ctx->device);
  for (Slot &slot : s->slots)
    if (slot.stream) (void)hipStreamSynchronize(slot.stream);
  if (s->upload) (void)hipStreamSynchronize(s->upload);
  free_arena(s);
  delete s;
}

pp_status pp_server_submit(pp_server *s, const pp_source *src, uint32_t n, uint64_t *ticket) {
  if (!s || !ticket || (n > 0 && !src)) return PP_EINVAL;
  Request r;
  std::string err;
  if (build_sources(src, n, &r.dev, &r.photons, &err) != PP_OK) {
    set_error(s, err);
    return PP_EINVAL;
  }
  r.chunks = chunks_of(r.dev, r.photons);
  r.bytes = sizeof(pp::DevSource) * n + sizeof(pp::DevChunk) * r.chunks;
  for (uint32_t i = 0; i < n; ++i)
    if (std::find(r.events.begin(), r.events.end(), src[i].event_id) == r.events.end())
      r.events.push_back(src[i].event_id);
  r.t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (n > s->src_ring.cap || r.chunks > s->chunk_ring.cap || r.chunks > 0xFFFFFFFFull) {
      s->err = "request of " + std::to_string(n) + " sources and " + std::to_string(r.chunks) +
               " queue entries can never fit the device queue (" + std::to_string(s->src_ring.cap) + " sources, " +
               std::to_string(s->chunk_ring.cap) + " entries)";
      return PP_EBUDGET;
    }
    if (s->stop) {
      s->err = "server is stopping";
      return PP_ESTATE;
    }
    const uint64_t tk = s->next_ticket++;
    s->reqs.emplace(tk, std::move(r));
    s->backlog.push_back(tk);
    s->stats.submitted += 1;
    *ticket = tk;
  }
  s->cv_work.notify_one();
  return PP_OK;
}

pp_status pp_server_wait(pp_server *s, uint64_t ticket, pp_hit *out, uint64_t cap, float *dom_expected,
                         pp_request_info *info) {
  if (!s) return PP_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) {
    s->err = "unknown ticket";
    return PP_EINVAL;
  }
  // Another waiter on the same ticket may collect it meanwhile: look the
  // ticket up again after every wake-up, never re-create it.
  s->cv_done.wait(lk, [&] {
    it = s->reqs.find(ticket);
    return it == s->reqs.end() || it->second.state == kDone;
  });
  if (it == s->reqs.end()) {
    s->err = "ticket collected by another waiter";
    return PP_EINVAL;
  }
  if (it->second.status == PP_OK && it->second.hits.size() > cap) {
    // too small a buffer: report the size and keep the result for a retry
    if (info) {
      std::memset(info, 0, sizeof *info);
      info->n_hits = it->second.hits.size();
    }
    s->err = "hit buffer too small";
    return PP_ETRUNC;
  }
  Request r = std::move(it->second);
  s->reqs.erase(it);
  lk.unlock();
  const uint64_t m = std::min<uint64_t>(cap, r.hits.size());
  if (m && out) std::memcpy(out, r.hits.data(), sizeof(pp_hit) * m);
  if (dom_expected && !r.dom_expected.empty())
    std::memcpy(dom_expected, r.dom_expected.data(), sizeof(float) * r.dom_expected.size());
  if (info) {
    info->t_submit_s = r.t_submit;
    info->t_launch_s = r.t_launch;
    info->t_done_s = r.t_done;
    info->photons = r.photons;
    info->n_hits = r.hits.size();
    info->batch_events = r.batch_events;
    info->reserved = 0;
  }
  return r.status;
}

pp_status pp_server_get_stats(pp_server *s, pp_server_stats *out) {
  if (!s || !out) return PP_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->gpu_busy_s = union_length(s->intervals) / 1e3;
  double lo = 0, hi = 0;
  for (size_t i = 0; i < s->intervals.size(); ++i) {
    lo = i ? std::min(lo, s->intervals[i].first) : s->intervals[i].first;
    hi = i ? std::max(hi, s->intervals[i].second) : s->intervals[i].second;
  }
  out->gpu_span_s = (hi - lo) / 1e3;
  return PP_OK;
}

const char *pp_server_last_error(pp_server *s) {
  if (!s) return "";
  std::lock_guard<std::mutex> lk(s->mu);
  thread_local std::string copy;
  copy = s->err;
  return copy.c_str();
}

pp_status pp_server_run_clients(pp_server *srv, const pp_source *events, uint64_t n_events, uint32_t n_clients,
                                double rate_per_s, uint32_t outstanding, double duration_s, uint64_t seed,
                                double *latency_s, uint64_t cap, uint64_t *n_done, uint64_t *photons_done,
                                uint64_t *hits_done, double *wall_s) {
  if (!srv || n_clients == 0 || (rate_per_s <= 0 && outstanding == 0) || (n_events > 0 && !events) || !n_done ||
      !photons_done || !hits_done || !wall_s || (cap > 0 && !latency_s))
    return PP_EINVAL;
  std::mutex mu;
  uint64_t done = 0, photons = 0, hits = 0;
  pp_status first_bad = PP_OK;
  const double t0 = now_s();
  auto record = [&](pp_status st, const pp_request_info &info) {
    std::lock_guard<std::mutex> lk(mu);
    if (st != PP_OK) {
      if (first_bad == PP_OK) first_bad = st;
      return;
    }
    if (done < cap) latency_s[done] = info.t_done_s - info.t_submit_s;
    ++done;
    photons += info.photons;
    hits += info.n_hits;
  };
  auto collect = [&](uint64_t ticket) {
    std::vector<pp_hit> buf(64);
    pp_request_info info{};
    pp_status st;
    while ((st = pp_server_wait(srv, ticket, buf.data(), buf.size(), nullptr, &info)) == PP_ETRUNC)
      buf.resize(info.n_hits);
    record(st, info);
  };
  auto is_done = [&](uint64_t ticket) {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    return it == srv->reqs.end() || it->second.state == kDone;
  };
  auto client = [&](uint32_t c) {
    std::mt19937_64 rng(seed + c);
    std::exponential_distribution<double> gap(rate_per_s > 0 ? rate_per_s / n_clients : 1.0);
    std::deque<uint64_t> mine;
    const double t_end = t0 + duration_s;
    double next = t0 + (rate_per_s > 0 ? gap(rng) : 0.0);
    for (uint64_t i = c; i < n_events; i += n_clients) {
      if (rate_per_s > 0) {
        // open loop: collect finished requests until the next arrival time
        for (;;) {
          while (!mine.empty() && is_done(mine.front())) {
            collect(mine.front());
            mine.pop_front();
          }
          const double wait = next - now_s();
          if (wait <= 0) break;
          std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 2e-4)));
        }
      } else if (mine.size() >= outstanding) {
        collect(mine.front());
        mine.pop_front();
      }
      if (now_s() >= t_end) break;
      uint64_t tk = 0;
      const pp_status st = pp_server_submit(srv, events + i, 1, &tk);
      if (st != PP_OK) {
        record(st, pp_request_info{});
        break;
      }
      mine.push_back(tk);
      if (rate_per_s > 0) next += gap(rng);
    }
    while (!mine.empty()) {
      collect(mine.front());
      mine.pop_front();
    }
  };
  std::vector<std::thread> th;
  for (uint32_t c = 0; c < n_clients; ++c) th.emplace_back(client, c);
  for (auto &t : th) t.join();
  *wall_s = now_s() - t0;
  *n_done = done;
  *photons_done = photons;
  *hits_done = hits;
  return first_bad;
}

}  // extern "C"

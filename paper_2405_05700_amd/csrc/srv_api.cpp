// Photon server (include/pp_server.h): a multi-producer request queue, an
// HBM-budget admission policy and a scheduler thread that keeps up to
// max_inflight propagation launches in flight on separate HIP streams,
// forming each launch from every admissible request waiting at that moment.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/pp_server.h"
#include "pp_internal.h"

using namespace ppi;

namespace {

double now_s() {
  static const auto t0 = std::chrono::steady_clock::now();
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct Request {
  std::vector<pp_source> src;
  std::vector<uint32_t> events;  // distinct event ids of the request
  uint64_t photons = 0, bytes = 0;
  double t_submit = 0, t_launch = 0, t_done = 0;
  bool done = false;
  pp_status status = PP_OK;
  std::vector<pp_hit> hits;
  std::vector<float> dom_expected;
  uint32_t batch_events = 0;
};

struct Flight {
  uint64_t batch = 0;
  int stream = 0;
  uint64_t bytes = 0;
  std::vector<uint64_t> tickets;
  std::vector<uint32_t> src_offset;  // first source of each ticket in the batch
};

}  // namespace

struct pp_server {
  pp_context *ctx = nullptr;
  pp_surrogate *sur = nullptr;
  pp_server_config cfg{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Request> reqs;
  uint64_t next_ticket = 1;
  std::vector<hipStream_t> streams;
  std::vector<bool> stream_busy;
  std::vector<Flight> flights;  // scheduler thread only
  pp_server_stats stats{};
  bool stop = false;
  std::string err;
  std::thread th;
};

namespace {

void set_error(pp_server *s, const std::string &msg) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->err = msg;
}

// Finishes a completed launch: hits split by event id, optional surrogate
// expectations per request, batch released, requests marked done.
void finish(pp_server *s, Flight &f) {
  pp_context *ctx = s->ctx;
  uint64_t n = 0;
  std::vector<pp_hit> hits;
  pp_status st = pp_hit_count(ctx, f.batch, &n);
  if (st == PP_OK) {
    hits.resize(n);
    uint64_t tot = 0;
    st = pp_fetch_hits(ctx, f.batch, hits.data(), n, &tot);
  }
  std::vector<float> pairs;
  Batch *b = nullptr;
  (void)find_batch(ctx, f.batch, &b);
  const uint32_t n_src = b ? static_cast<uint32_t>(b->src.size()) : 0;
  if (st == PP_OK && s->sur && n_src > 0) {
    pairs.resize(static_cast<size_t>(n_src) * ctx->n_doms);
    st = pp_sur_predict_pairs(s->sur, f.batch, pairs.data(), pairs.size());
  }
  const std::string msg = st == PP_OK ? std::string() : std::string(pp_last_error(ctx));
  (void)pp_release(ctx, f.batch);
  const double t = now_s();
  std::lock_guard<std::mutex> lk(s->mu);
  std::unordered_map<uint32_t, uint64_t> owner;
  for (uint64_t tk : f.tickets)
    for (uint32_t e : s->reqs[tk].events) owner[e] = tk;
  for (const pp_hit &h : hits) {
    auto it = owner.find(h.event_id);
    if (it != owner.end()) s->reqs[it->second].hits.push_back(h);
  }
  for (size_t i = 0; i < f.tickets.size(); ++i) {
    Request &r = s->reqs[f.tickets[i]];
    if (!pairs.empty()) {
      r.dom_expected.assign(ctx->n_doms, 0.0f);
      for (size_t k = 0; k < r.src.size(); ++k) {
        const float *row = pairs.data() + static_cast<size_t>(f.src_offset[i] + k) * ctx->n_doms;
        for (uint32_t d = 0; d < ctx->n_doms; ++d) r.dom_expected[d] += row[d];
      }
    }
    r.status = st;
    r.t_done = t;
    r.done = true;
    s->stats.completed += 1;
    s->stats.photons_completed += r.photons;
  }
  if (!msg.empty()) s->err = msg;
  s->stats.bytes_in_use -= f.bytes;
  s->stream_busy[f.stream] = false;
  s->cv_done.notify_all();
}

void scheduler(pp_server *s) {
  pp_context *ctx = s->ctx;
  (void)hipSetDevice(ctx->device);
  for (;;) {
    bool progressed = false;
    // completions
    for (size_t i = 0; i < s->flights.size();) {
      Batch *b = nullptr;
      const bool ready = find_batch(ctx, s->flights[i].batch, &b) != PP_OK || hipEventQuery(b->ev1) == hipSuccess;
      if (ready) {
        finish(s, s->flights[i]);
        s->flights.erase(s->flights.begin() + static_cast<long>(i));
        progressed = true;
      } else {
        ++i;
      }
    }
    // admission of the waiting requests into one new launch
    std::vector<uint64_t> take;
    int stream = -1;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->stop && s->queue.empty() && s->flights.empty()) break;
      if (!s->queue.empty() && s->flights.size() < s->cfg.max_inflight) {
        for (size_t k = 0; k < s->stream_busy.size(); ++k)
          if (!s->stream_busy[k]) {
            stream = static_cast<int>(k);
            break;
          }
      }
      if (stream >= 0) {
        const uint32_t n = static_cast<uint32_t>(s->queue.size());
        std::vector<uint64_t> bytes(n), photons(n);
        std::vector<uint32_t> ev(n);
        for (uint32_t i = 0; i < n; ++i) {
          const Request &r = s->reqs[s->queue[i]];
          bytes[i] = r.bytes;
          photons[i] = r.photons;
          ev[i] = r.events.empty() ? 0xFFFFFFFFu : r.events[0];
        }
        std::vector<uint8_t> sel(n, 0);
        pp_server_admit_plan(n, bytes.data(), ev.data(), photons.data(), s->stats.bytes_in_use,
                             s->cfg.hbm_budget_bytes, s->cfg.max_batch_events, s->cfg.max_batch_photons, sel.data());
        // requests carrying several event ids: drop any that collide with
        // an already selected one (they wait for the next launch)
        std::unordered_set<uint32_t> used;
        std::deque<uint64_t> rest;
        uint64_t add = 0;
        for (uint32_t i = 0; i < n; ++i) {
          const uint64_t tk = s->queue[i];
          Request &r = s->reqs[tk];
          bool ok = sel[i] != 0;
          for (uint32_t e : r.events) ok = ok && !used.count(e);
          if (ok) {
            for (uint32_t e : r.events) used.insert(e);
            take.push_back(tk);
            add += r.bytes;
            r.t_launch = now_s();
          } else {
            rest.push_back(tk);
            s->stats.deferred += 1;
          }
        }
        s->queue.swap(rest);
        s->stats.bytes_in_use += add;
        s->stats.peak_bytes_in_use = std::max(s->stats.peak_bytes_in_use, s->stats.bytes_in_use);
        if (!take.empty()) {
          s->stream_busy[stream] = true;
          s->stats.launches += 1;
        }
      }
    }
    if (!take.empty()) {
      Flight f;
      f.stream = stream;
      std::vector<pp_source> all;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        for (uint64_t tk : take) {
          Request &r = s->reqs[tk];
          f.src_offset.push_back(static_cast<uint32_t>(all.size()));
          all.insert(all.end(), r.src.begin(), r.src.end());
          f.bytes += r.bytes;
          r.batch_events = static_cast<uint32_t>(take.size());
        }
      }
      f.tickets = take;
      pp_status st = pp_submit(ctx, all.data(), static_cast<uint32_t>(all.size()), &f.batch);
      if (st == PP_OK) st = pp_propagate(ctx, f.batch, s->streams[stream]);
      if (st == PP_OK) {
        s->flights.push_back(f);
      } else {
        const std::string msg = pp_last_error(ctx);
        std::lock_guard<std::mutex> lk(s->mu);
        for (uint64_t tk : take) {
          Request &r = s->reqs[tk];
          r.status = st;
          r.done = true;
          r.t_done = now_s();
        }
        s->err = msg;
        s->stats.bytes_in_use -= f.bytes;
        s->stream_busy[stream] = false;
        s->cv_done.notify_all();
      }
      progressed = true;
    }
    if (!progressed) {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait_for(lk, std::chrono::microseconds(s->flights.empty() ? 2000 : 50));
    }
  }
}

}  // namespace

extern "C" {

uint32_t pp_server_admit_plan(uint32_t n, const uint64_t *bytes, const uint32_t *event_ids, const uint64_t *photons,
                              uint64_t bytes_in_use, uint64_t budget, uint32_t max_events, uint64_t max_photons,
                              uint8_t *take) {
  uint32_t taken = 0;
  uint64_t used = bytes_in_use, ph = 0;
  std::unordered_set<uint32_t> seen;
  for (uint32_t i = 0; i < n; ++i) {
    take[i] = 0;
    if (taken >= max_events || ph >= max_photons) continue;
    if (used > budget || bytes[i] > budget - used) continue;
    if (seen.count(event_ids[i])) continue;
    take[i] = 1;
    seen.insert(event_ids[i]);
    used += bytes[i];
    ph += photons[i];
    ++taken;
  }
  return taken;
}

uint64_t pp_server_request_bytes(uint32_t n_sources, uint64_t n_photons) {
  return batch_device_bytes(n_sources, n_photons, 64, default_hit_capacity(n_photons));
}

pp_status pp_server_create(pp_context *ctx, const pp_server_config *cfg, pp_surrogate *sur, pp_server **out) {
  if (!ctx || !out) return PP_EINVAL;
  *out = nullptr;
  pp_status st = need_device(ctx);
  if (st != PP_OK) return st;
  if (!ctx->ice_loaded || !ctx->geo_loaded) return fail(ctx, PP_ESTATE, "load ice and geometry first");
  pp_server *s = new (std::nothrow) pp_server;
  if (!s) return PP_ENOMEM;
  s->ctx = ctx;
  s->sur = sur;
  pp_server_config c = cfg ? *cfg : pp_server_config{};
  if (!c.max_inflight) c.max_inflight = 4;
  if (!c.max_batch_events) c.max_batch_events = 4096;
  if (!c.hbm_budget_bytes) c.hbm_budget_bytes = 200000000000ull;
  if (!c.max_batch_photons) c.max_batch_photons = 200000000ull;
  s->cfg = c;
  for (uint32_t i = 0; i < c.max_inflight; ++i) {
    hipStream_t h;
    if (hipStreamCreateWithFlags(&h, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      return fail(ctx, PP_EDEVICE, "hipStreamCreateWithFlags failed");
    }
    s->streams.push_back(h);
    s->stream_busy.push_back(false);
  }
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
  for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
  delete s;
}

pp_status pp_server_submit(pp_server *s, const pp_source *src, uint32_t n, uint64_t *ticket) {
  if (!s || !ticket || (n > 0 && !src)) return PP_EINVAL;
  Request r;
  std::vector<pp::DevSource> dev;
  std::string err;
  if (build_sources(src, n, &dev, &r.photons, &err) != PP_OK) {
    set_error(s, err);
    return PP_EINVAL;
  }
  r.src.assign(src, src + n);
  for (uint32_t i = 0; i < n; ++i)
    if (std::find(r.events.begin(), r.events.end(), src[i].event_id) == r.events.end())
      r.events.push_back(src[i].event_id);
  r.bytes = pp_server_request_bytes(n, r.photons);
  r.t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (r.bytes > s->cfg.hbm_budget_bytes) {
      s->err = "request needs " + std::to_string(r.bytes) + " device bytes, over the budget";
      return PP_EBUDGET;
    }
    if (s->stop) {
      s->err = "server is stopping";
      return PP_ESTATE;
    }
    const uint64_t tk = s->next_ticket++;
    s->reqs.emplace(tk, std::move(r));
    s->queue.push_back(tk);
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
  s->cv_done.wait(lk, [&] { return s->reqs[ticket].done; });
  if (s->reqs[ticket].status == PP_OK && s->reqs[ticket].hits.size() > cap) {
    // too small a buffer: report the size and keep the result for a retry
    if (info) {
      std::memset(info, 0, sizeof *info);
      info->n_hits = s->reqs[ticket].hits.size();
    }
    s->err = "hit buffer too small";
    return PP_ETRUNC;
  }
  Request r = std::move(s->reqs[ticket]);
  s->reqs.erase(ticket);
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
  return PP_OK;
}

const char *pp_server_last_error(pp_server *s) {
  if (!s) return "";
  std::lock_guard<std::mutex> lk(s->mu);
  thread_local std::string copy;
  copy = s->err;
  return copy.c_str();
}

}  // extern "C"

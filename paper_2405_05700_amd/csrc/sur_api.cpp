// Host side of the surrogate C ABI (include/pp_surrogate.h): parameter and
// Adam state, training set (features and Monte Carlo labels on the device),
// minibatch forward/backward on the matrix cores, and chunked inference.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "../../include/pp_surrogate.h"
#include "pp_internal.h"
#include "sur_device.h"

using namespace ppi;

struct pp_surrogate {
  pp_context *ctx = nullptr;
  int device = -1;  // the context's device (teardown does not read the context)
  int n_doms = 0;
  // parameters (f32 master), gradient, Adam moments, bf16 copies
  float *theta = nullptr, *grad = nullptr, *adam_m = nullptr, *adam_v = nullptr;
  uint16_t *wb = nullptr, *wt = nullptr;
  int64_t adam_t = 0;
  float4 *doms_by_id = nullptr;
  // training set; with pair selection (far_stride > 1) each row is the pair
  // pair_of_row[row] with loss weight w[row], else row = pair and weight 1
  int64_t P = 0, P_pad = 0;
  uint16_t *X = nullptr;
  float *mu_base = nullptr, *nph = nullptr, *k = nullptr, *n_t = nullptr, *s1 = nullptr, *s2 = nullptr;
  float near_m = INFINITY;
  uint32_t far_stride = 1;
  float cut_m = INFINITY;  // inference distance cut
  int64_t *pair_of_row = nullptr;
  float *w = nullptr;
  // minibatch work buffers (capacity Mcap rows): bf16 feature-major copies
  // of the inputs, activations and output gradients for the weight
  // gradients, and the fixed-order reduction parts (per 32-row block: bias
  // column sums and loss; per K slice: weight-gradient partials, capacity
  // ws_splits slices)
  int64_t Mcap = 0;
  uint16_t *XT = nullptr, *HT[4] = {}, *dYT = nullptr, *dZT[4] = {};
  float *col_part = nullptr;
  double *loss_part = nullptr;
  float *ws = nullptr;
  int ws_splits = 0;
  double *d_loss = nullptr;
  double *epoch_loss = nullptr;  // device accumulator while training, else null
  uint64_t shuffle_seed = 0;
  uint64_t epochs_done = 0;
  // inference buffers (capacity Icap rows; photons per source, capacity
  // NScap, kept between calls so inference allocates nothing once warm)
  int64_t Icap = 0, NScap = 0;
  float *i_src_nph = nullptr;
  float *i_mu = nullptr;
};

namespace {

constexpr int64_t kInferRows = 1 << 21;  // pairs per inference chunk

int64_t round64(int64_t n) { return (n + 63) / 64 * 64; }

template <class T>
pp_status dalloc(pp_context *ctx, T **p, int64_t n) {
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  PP_HIP(ctx, hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * std::max<int64_t>(n, 1)));
  return PP_OK;
}

template <class T>
void dfree(T *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// Runs f when the returned object goes out of scope.
template <class F>
struct OnExit {
  F f;
  ~OnExit() { f(); }
};
template <class F>
OnExit<F> on_exit(F f) {
  return OnExit<F>{f};
}

const float *bias_ptr(const pp_surrogate *s, int l) { return s->theta + sur::b_offset(l); }
const uint16_t *wb_ptr(const pp_surrogate *s, int l) { return s->wb + sur::wb_offset(l); }
const uint16_t *wt_ptr(const pp_surrogate *s, int l) { return s->wt + sur::wb_offset(l); }

// K slices of the weight gradients over M minibatch rows: kWgradSplits, or
// one per 32-row block when there are fewer.
int wgrad_splits(int64_t M) {
  return static_cast<int>(std::min<int64_t>(sur::kWgradSplits, M / sur::kTrainRows));
}

pp_status ensure_work(pp_surrogate *s, int64_t M) {
  pp_context *ctx = s->ctx;
  pp_status st;
  if (M > s->Mcap) {
    if ((st = dalloc(ctx, &s->XT, M * sur::kInPad)) != PP_OK) return st;
    for (int l = 0; l < 4; ++l) {
      if ((st = dalloc(ctx, &s->HT[l], M * sur::kHidden)) != PP_OK) return st;
      if ((st = dalloc(ctx, &s->dZT[l], M * sur::kHidden)) != PP_OK) return st;
    }
    if ((st = dalloc(ctx, &s->dYT, M * sur::kOutPad)) != PP_OK) return st;
    if ((st = dalloc(ctx, &s->col_part, (M / sur::kTrainRows) * sur::kBiasCols)) != PP_OK) return st;
    if ((st = dalloc(ctx, &s->loss_part, M / sur::kTrainRows)) != PP_OK) return st;
    s->Mcap = M;
  }
  const int splits = wgrad_splits(M);
  if (splits > s->ws_splits) {
    if ((st = dalloc(ctx, &s->ws, int64_t{splits} * sur::wb_count())) != PP_OK) return st;
    s->ws_splits = splits;
  }
  return PP_OK;
}

pp_status check_rows(pp_surrogate *s, int64_t first, int64_t count) {
  if (count <= 0 || first < 0 || first + count > s->P)
    return fail(s->ctx, PP_EINVAL, "rows [%lld, %lld) invalid: must lie within %lld pairs", (long long)first,
                (long long)(first + count), (long long)s->P);
  if (count > (int64_t{1} << 30)) return fail(s->ctx, PP_EINVAL, "at most 2^30 rows per pass");
  return PP_OK;
}

// One pass over the minibatch of training rows (mul (first + i) + add) mod P,
// i < count: forward, loss and backward, the gradient left in s->grad and the
// loss sum in s->d_loss (and added to s->epoch_loss if set); with adam, also
// the Adam step with step size lr. Three launches on stream st.
pp_status train_pass(pp_surrogate *s, uint64_t mul, uint64_t add, int64_t first, int64_t count, bool adam,
                     float lr, hipStream_t st) {
  pp_context *ctx = s->ctx;
  using namespace sur;
  const int64_t M = round64(count);
  pp_status rc = ensure_work(s, M);
  if (rc != PP_OK) return rc;
  TrainArgs t{};
  t.X = s->X;
  t.mu_base = s->mu_base;
  t.nph = s->nph;
  t.k = s->k;
  t.n_t = s->n_t;
  t.s1 = s->s1;
  t.s2 = s->s2;
  t.w = s->w;
  t.P = static_cast<uint64_t>(s->P);
  t.mul = mul;
  t.add = add;
  t.first = first;
  t.count = static_cast<int>(count);
  t.M = static_cast<int>(M);
  t.inv_norm = 1.0f / static_cast<float>(count);
  for (int l = 0; l < kLayers; ++l) {
    t.wb[l] = wb_ptr(s, l);
    t.wt[l] = wt_ptr(s, l);
    t.b[l] = bias_ptr(s, l);
  }
  t.XT = s->XT;
  t.dYT = s->dYT;
  for (int l = 0; l < 4; ++l) {
    t.HT[l] = s->HT[l];
    t.dZT[l] = s->dZT[l];
  }
  t.col_part = s->col_part;
  t.loss_part = s->loss_part;
  PP_HIP(ctx, launch_train_rows(t, st));
  WgradArgs g{};
  g.A[0] = s->dZT[0];
  g.B[0] = s->XT;
  for (int l = 1; l < 4; ++l) {
    g.A[l] = s->dZT[l];
    g.B[l] = s->HT[l - 1];
  }
  g.A[4] = s->dYT;
  g.B[4] = s->HT[3];
  g.M = static_cast<int>(M);
  g.splits = wgrad_splits(M);
  g.ws = s->ws;
  PP_HIP(ctx, launch_wgrad(g, st));
  AdamArgs a{};
  a.theta = s->theta;
  a.grad = s->grad;
  a.m = s->adam_m;
  a.v = s->adam_v;
  a.wb = s->wb;
  a.wt = s->wt;
  a.ws = s->ws;
  a.splits = g.splits;
  a.col_part = s->col_part;
  a.loss_part = s->loss_part;
  a.n_blocks = static_cast<int>(M / kTrainRows);
  a.loss_sum = s->d_loss;
  a.loss_epoch = s->epoch_loss;
  a.adam = adam ? 1 : 0;
  if (adam) {
    s->adam_t += 1;
    a.lr = lr;
    a.c1 = 1.0f - std::pow(0.9f, static_cast<float>(s->adam_t));
    a.c2 = 1.0f - std::pow(0.999f, static_cast<float>(s->adam_t));
  }
  PP_HIP(ctx, launch_reduce_adam(a, st));
  return PP_OK;
}

uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// He-uniform initialisation (fan-in of the real inputs), zero biases, zero
// padded input columns and padded outputs, output layer scaled by 0.1.
std::vector<float> init_params(uint64_t seed) {
  std::vector<float> th(sur::param_count(), 0.0f);
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> uni(-1.0, 1.0);
  for (int l = 0; l < sur::kLayers; ++l) {
    const int n_in = sur::in_dim(l), n_out = sur::out_dim(l);
    const double lim = std::sqrt(6.0 / (l == 0 ? sur::kInReal : n_in)) * (l == sur::kLayers - 1 ? 0.1 : 1.0);
    for (int o = 0; o < n_out; ++o)
      for (int i = 0; i < n_in; ++i) {
        const bool pad = (l == 0 && i >= sur::kInReal) || (l == sur::kLayers - 1 && o >= sur::kOutReal);
        const double w = lim * uni(rng);
        th[sur::w_offset(l) + static_cast<int64_t>(o) * n_in + i] = pad ? 0.0f : static_cast<float>(w);
      }
  }
  return th;
}

pp_status upload_params(pp_surrogate *s, const float *host) {
  PP_HIP(s->ctx, hipMemcpy(s->theta, host, sizeof(float) * sur::param_count(), hipMemcpyHostToDevice));
  PP_HIP(s->ctx, hipMemset(s->adam_m, 0, sizeof(float) * sur::param_count()));
  PP_HIP(s->ctx, hipMemset(s->adam_v, 0, sizeof(float) * sur::param_count()));
  s->adam_t = 0;
  PP_HIP(s->ctx, sur::launch_pack_weights(s->theta, s->wb, s->wt, nullptr));
  PP_HIP(s->ctx, hipDeviceSynchronize());
  return PP_OK;
}

sur::FeatureArgs feature_args(pp_surrogate *s, const Batch &b, const float *src_nph) {
  pp_context *ctx = s->ctx;
  sur::FeatureArgs f{};
  f.sources = b.d_src;
  f.src_nph = src_nph;
  f.n_sources_set = static_cast<int>(b.src.size());
  f.doms = s->doms_by_id;
  f.n_doms = s->n_doms;
  f.layers = ctx->d_layers;
  f.n_layers = static_cast<int>(ctx->ice.n_layers);
  f.z_lo = ctx->ice.z_lo_m;
  f.inv_dz = static_cast<float>(1.0 / ctx->ice.dz_m);
  f.radius = ctx->radius;
  return f;
}

std::vector<float> source_photons(const Batch &b) {
  std::vector<float> n(b.src.size());
  for (size_t i = 0; i < b.src.size(); ++i) {
    const uint64_t end = i + 1 < b.src.size() ? b.src[i + 1].seq_base : b.n_photons;
    n[i] = static_cast<float>(end - b.src[i].seq_base);
  }
  return n;
}

pp_status check_cherenkov(pp_context *ctx, const Batch &b) {
  for (size_t i = 0; i < b.src.size(); ++i)
    if (b.src[i].ids.x != PP_SOURCE_CHERENKOV)
      return fail(ctx, PP_EINVAL, "surrogate sources must be Cherenkov segments (source %zu is not)", i);
  return PP_OK;
}

// Runs the fused network over every pair of batch b: expected hits are added
// to dom_sums (if not null) and, if pair_sink is given, produced per pair in
// chunks of whole sources (pair_sink(mu, first_source, n_sources)).
template <class Sink>
pp_status infer(pp_surrogate *s, Batch &b, hipStream_t st, double *dom_sums, Sink *pair_sink) {
  pp_context *ctx = s->ctx;
  using namespace sur;
  const int64_t n_src = static_cast<int64_t>(b.src.size());
  pp_status rc = PP_OK;
  const std::vector<float> nph = source_photons(b);
  if (static_cast<int64_t>(nph.size()) > s->NScap) {
    if ((rc = dalloc(ctx, &s->i_src_nph, static_cast<int64_t>(nph.size()))) != PP_OK) return rc;
    s->NScap = static_cast<int64_t>(nph.size());
  }
  float *d_src_nph = s->i_src_nph;
  if (!nph.empty())
    PP_HIP(ctx, hipMemcpyAsync(d_src_nph, nph.data(), sizeof(float) * nph.size(), hipMemcpyHostToDevice, st));
  FusedArgs a{};
  a.f = feature_args(s, b, d_src_nph);
  for (int l = 0; l < kLayers; ++l) {
    a.w[l] = wb_ptr(s, l);
    a.b[l] = bias_ptr(s, l);
  }
  a.dom_sums = dom_sums;
  a.cut2 = std::isinf(s->cut_m) ? INFINITY : s->cut_m * s->cut_m;
  // sources per launch: all of them, or as many as the per-pair buffer holds
  const int64_t per_launch =
      pair_sink ? std::max<int64_t>(1, kInferRows / std::max(s->n_doms, 1)) : std::max<int64_t>(n_src, 1);
  if (pair_sink) {
    const int64_t cap = per_launch * s->n_doms;
    if (cap > s->Icap) {
      if ((rc = dalloc(ctx, &s->i_mu, cap)) != PP_OK) return rc;
      s->Icap = cap;
    }
    a.pair_mu = s->i_mu;
  }
  for (int64_t s0 = 0; s0 < n_src && rc == PP_OK; s0 += per_launch) {
    const int64_t ns = std::min(per_launch, n_src - s0);
    a.f.first_pair = s0 * s->n_doms;
    a.f.n_pairs = ns * s->n_doms;
    const hipError_t e = launch_infer_fused(a, st);
    if (e != hipSuccess) {
      rc = fail(ctx, PP_EDEVICE, "fused inference launch: %s", hipGetErrorString(e));
      break;
    }
    if (pair_sink) rc = (*pair_sink)(s->i_mu, s0, ns);
  }
  (void)hipStreamSynchronize(st);  // also keeps nph alive until its copy has run
  return rc;
}

}  // namespace

extern "C" {

uint64_t pp_sur_param_count(void) { return static_cast<uint64_t>(sur::param_count()); }

uint32_t pp_sur_feature_count(void) { return static_cast<uint32_t>(sur::kInReal); }

pp_status pp_sur_create(pp_context *ctx, uint64_t init_seed, pp_surrogate **out) {
  if (!ctx || !out) return PP_EINVAL;
  *out = nullptr;
  pp_status st = need_device(ctx);
  if (st != PP_OK) return st;
  if (!ctx->ice_loaded || !ctx->geo_loaded) return fail(ctx, PP_ESTATE, "load ice and geometry first");
  pp_surrogate *s = new (std::nothrow) pp_surrogate;
  if (!s) return PP_ENOMEM;
  s->ctx = ctx;
  s->device = ctx->device;
  s->n_doms = static_cast<int>(ctx->n_doms);
  const int64_t np = sur::param_count();
  if ((st = dalloc(ctx, &s->theta, np)) != PP_OK || (st = dalloc(ctx, &s->grad, np)) != PP_OK ||
      (st = dalloc(ctx, &s->adam_m, np)) != PP_OK || (st = dalloc(ctx, &s->adam_v, np)) != PP_OK ||
      (st = dalloc(ctx, &s->wb, sur::wb_count())) != PP_OK || (st = dalloc(ctx, &s->wt, sur::wb_count())) != PP_OK ||
      (st = dalloc(ctx, &s->d_loss, 1)) != PP_OK) {
    pp_sur_destroy(s);
    return st;
  }
  // Every gradient element a step computes is overwritten by it; the
  // output-layer bias entries past the real outputs are never computed and
  // stay 0.
  if (sur::launch_zero_f32(s->grad, np, nullptr) != hipSuccess) {
    pp_sur_destroy(s);
    return fail(ctx, PP_EDEVICE, "clearing the gradient failed");
  }
  // module centres in module-id order
  std::vector<float4> by_id(std::max<size_t>(ctx->doms_sorted.size(), 1));
  for (const float4 &d : ctx->doms_sorted) {
    uint32_t id;
    std::memcpy(&id, &d.w, 4);
    by_id[id] = d;
  }
  if ((st = dalloc(ctx, &s->doms_by_id, static_cast<int64_t>(by_id.size()))) != PP_OK) {
    pp_sur_destroy(s);
    return st;
  }
  (void)hipMemcpy(s->doms_by_id, by_id.data(), sizeof(float4) * by_id.size(), hipMemcpyHostToDevice);
  s->shuffle_seed = init_seed ^ 0x5DEECE66Dull;
  const std::vector<float> th = init_params(init_seed);
  if ((st = upload_params(s, th.data())) != PP_OK) {
    pp_sur_destroy(s);
    return st;
  }
  *out = s;
  return PP_OK;
}

void pp_sur_destroy(pp_surrogate *s) {
  if (!s) return;
  if (s->device >= 0) (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  dfree(s->theta), dfree(s->grad), dfree(s->adam_m), dfree(s->adam_v), dfree(s->wb), dfree(s->wt);
  dfree(s->doms_by_id), dfree(s->X), dfree(s->mu_base), dfree(s->nph);
  dfree(s->k), dfree(s->n_t), dfree(s->s1), dfree(s->s2), dfree(s->pair_of_row), dfree(s->w);
  dfree(s->XT), dfree(s->dYT), dfree(s->d_loss);
  for (int l = 0; l < 4; ++l) dfree(s->HT[l]), dfree(s->dZT[l]);
  dfree(s->ws), dfree(s->col_part), dfree(s->loss_part);
  dfree(s->i_mu), dfree(s->i_src_nph);
  delete s;
}

pp_status pp_sur_get_params(pp_surrogate *s, float *out, uint64_t n) {
  if (!s || !out) return PP_EINVAL;
  if (n != pp_sur_param_count()) return fail(s->ctx, PP_EINVAL, "expected %llu parameters", (unsigned long long)pp_sur_param_count());
  PP_HIP(s->ctx, hipSetDevice(s->ctx->device));
  PP_HIP(s->ctx, hipDeviceSynchronize());
  PP_HIP(s->ctx, hipMemcpy(out, s->theta, sizeof(float) * n, hipMemcpyDeviceToHost));
  return PP_OK;
}

pp_status pp_sur_set_params(pp_surrogate *s, const float *in, uint64_t n) {
  if (!s || !in) return PP_EINVAL;
  if (n != pp_sur_param_count()) return fail(s->ctx, PP_EINVAL, "expected %llu parameters", (unsigned long long)pp_sur_param_count());
  PP_HIP(s->ctx, hipSetDevice(s->ctx->device));
  for (uint64_t i = 0; i < n; ++i)
    if (!std::isfinite(in[i])) return fail(s->ctx, PP_EINVAL, "parameter %llu is not finite", (unsigned long long)i);
  return upload_params(s, in);
}

pp_status pp_sur_set_training_set(pp_surrogate *s, uint64_t batch) {
  if (!s) return PP_EINVAL;
  pp_context *ctx = s->ctx;
  pp_status st = need_device(ctx);
  if (st != PP_OK) return st;
  Batch *b;
  if ((st = find_batch(ctx, batch, &b)) != PP_OK) return st;
  if ((st = check_cherenkov(ctx, *b)) != PP_OK) return st;
  uint64_t n_hits = 0;
  if ((st = complete_hits(ctx, *b, &n_hits)) != PP_OK) return st;
  const int64_t n_src = static_cast<int64_t>(b->src.size());
  // event id -> source index (each source its own event)
  uint32_t max_event = 0;
  for (const auto &d : b->src) max_event = std::max(max_event, d.ids.y);
  if (max_event > (1u << 26)) return fail(ctx, PP_EINVAL, "event ids up to 2^26 supported for training");
  std::vector<int32_t> ev(max_event + 1, -1);
  for (int64_t i = 0; i < n_src; ++i) {
    if (ev[b->src[i].ids.y] >= 0) return fail(ctx, PP_EINVAL, "training sources need distinct event ids");
    ev[b->src[i].ids.y] = static_cast<int32_t>(i);
  }
  const int64_t n_all = n_src * static_cast<int64_t>(s->n_doms);
  // pair selection: rows are every pair, or the kept ones in source-major order
  dfree(s->pair_of_row);
  dfree(s->w);
  // staging buffers, freed on every exit
  float *d_src_nph = nullptr;
  int32_t *d_ev = nullptr, *d_row_of_pair = nullptr;
  uint32_t *d_count = nullptr;
  int64_t *d_offset = nullptr;
  unsigned long long *d_s1q = nullptr, *d_s2q = nullptr;
  const auto cleanup = on_exit([&] {
    dfree(d_src_nph), dfree(d_ev), dfree(d_row_of_pair), dfree(d_count), dfree(d_offset), dfree(d_s1q), dfree(d_s2q);
  });
  if (s->far_stride > 1 && n_src > 0) {
    if (n_all >= (int64_t{1} << 31)) return fail(ctx, PP_EINVAL, "pair selection supports up to 2^31 pairs");
    sur::SelectArgs a{};
    a.sources = b->d_src;
    a.n_sources = static_cast<int>(n_src);
    a.doms = s->doms_by_id;
    a.n_doms = s->n_doms;
    a.near2 = std::isinf(s->near_m) ? INFINITY : s->near_m * s->near_m;
    a.far_stride = s->far_stride;
    if ((st = dalloc(ctx, &d_count, n_src)) != PP_OK) return st;
    a.count = d_count;
    PP_HIP(ctx, sur::launch_select(a, false, nullptr));
    std::vector<uint32_t> count(n_src);
    PP_HIP(ctx, hipMemcpy(count.data(), d_count, sizeof(uint32_t) * n_src, hipMemcpyDeviceToHost));
    dfree(d_count);
    std::vector<int64_t> offset(n_src);
    int64_t total = 0;
    for (int64_t i = 0; i < n_src; ++i) offset[i] = total, total += count[i];
    if ((st = dalloc(ctx, &d_offset, n_src)) != PP_OK || (st = dalloc(ctx, &s->pair_of_row, total)) != PP_OK ||
        (st = dalloc(ctx, &s->w, round64(total))) != PP_OK || (st = dalloc(ctx, &d_row_of_pair, n_all)) != PP_OK)
      return st;
    PP_HIP(ctx, hipMemcpy(d_offset, offset.data(), sizeof(int64_t) * n_src, hipMemcpyHostToDevice));
    PP_HIP(ctx, sur::launch_zero_f32(s->w, round64(total), nullptr));
    a.row_offset = d_offset;
    a.n_rows = total;
    a.pair_of_row = s->pair_of_row;
    a.row_of_pair = d_row_of_pair;
    a.w = s->w;
    PP_HIP(ctx, sur::launch_select(a, true, nullptr));
    PP_HIP(ctx, hipDeviceSynchronize());
    s->P = total;
  } else {
    s->P = n_all;
  }
  s->P_pad = round64(s->P);
  const int64_t R = s->P_pad;
  if ((st = dalloc(ctx, &s->X, R * sur::kInPad)) != PP_OK ||
      (st = dalloc(ctx, &s->mu_base, R)) != PP_OK || (st = dalloc(ctx, &s->nph, R)) != PP_OK ||
      (st = dalloc(ctx, &s->k, R)) != PP_OK || (st = dalloc(ctx, &s->n_t, R)) != PP_OK ||
      (st = dalloc(ctx, &s->s1, R)) != PP_OK || (st = dalloc(ctx, &s->s2, R)) != PP_OK)
    return st;
  const std::vector<float> nph = source_photons(*b);
  if ((st = dalloc(ctx, &d_src_nph, n_src)) != PP_OK) return st;
  if ((st = dalloc(ctx, &d_ev, static_cast<int64_t>(ev.size()))) != PP_OK) return st;
  PP_HIP(ctx, hipMemcpy(d_src_nph, nph.data(), sizeof(float) * nph.size(), hipMemcpyHostToDevice));
  PP_HIP(ctx, hipMemcpy(d_ev, ev.data(), sizeof(int32_t) * ev.size(), hipMemcpyHostToDevice));
  sur::FeatureArgs f = feature_args(s, *b, d_src_nph);
  f.first_pair = 0;
  f.n_pairs = s->P;
  f.pair_of_row = s->pair_of_row;
  f.X = s->X;
  f.mu_base = s->mu_base;
  f.nph = s->nph;
  PP_HIP(ctx, sur::launch_features(f, nullptr));
  PP_HIP(ctx, sur::launch_zero_f32(s->k, R, nullptr));
  PP_HIP(ctx, sur::launch_zero_f32(s->n_t, R, nullptr));
  if ((st = dalloc(ctx, &d_s1q, R)) != PP_OK || (st = dalloc(ctx, &d_s2q, R)) != PP_OK) return st;
  const float time_per_m = static_cast<float>(static_cast<double>(ctx->ice.n_group) / 0.299792458);
  PP_HIP(ctx, sur::launch_labels(b->d_hits, b->d_counters + pp::kHitCount, b->hit_cap, d_ev,
                                 static_cast<uint32_t>(ev.size()), b->d_src, s->doms_by_id, s->n_doms, ctx->radius,
                                 time_per_m, d_row_of_pair, s->k, s->n_t, d_s1q, d_s2q, s->s1, s->s2, R, nullptr));
  PP_HIP(ctx, hipDeviceSynchronize());
  return PP_OK;
}

pp_status pp_sur_set_sampling(pp_surrogate *s, float near_m, uint32_t far_stride) {
  if (!s) return PP_EINVAL;
  if (!(near_m >= 0.0f) || far_stride == 0)
    return fail(s->ctx, PP_EINVAL, "near_m must be >= 0 (or +inf) and far_stride >= 1");
  s->near_m = near_m;
  s->far_stride = far_stride;
  return PP_OK;
}

pp_status pp_sur_set_inference_cut(pp_surrogate *s, float cut_m) {
  if (!s) return PP_EINVAL;
  if (!(cut_m > 0.0f)) return fail(s->ctx, PP_EINVAL, "cut_m must be > 0 (or +inf)");
  s->cut_m = cut_m;
  return PP_OK;
}

pp_status pp_sur_get_training_pairs(pp_surrogate *s, uint64_t first, uint64_t count, uint64_t *pair,
                                    float *weight) {
  if (!s) return PP_EINVAL;
  pp_context *ctx = s->ctx;
  if (first + count > static_cast<uint64_t>(s->P)) return fail(ctx, PP_EINVAL, "rows out of range");
  PP_HIP(ctx, hipSetDevice(ctx->device));
  PP_HIP(ctx, hipDeviceSynchronize());
  if (pair && count) {
    if (s->pair_of_row)
      PP_HIP(ctx, hipMemcpy(pair, s->pair_of_row + first, sizeof(uint64_t) * count, hipMemcpyDeviceToHost));
    else
      for (uint64_t r = 0; r < count; ++r) pair[r] = first + r;
  }
  if (weight && count) {
    if (s->w)
      PP_HIP(ctx, hipMemcpy(weight, s->w + first, sizeof(float) * count, hipMemcpyDeviceToHost));
    else
      std::fill(weight, weight + count, 1.0f);
  }
  return PP_OK;
}

pp_status pp_sur_training_size(const pp_surrogate *s, uint64_t *n) {
  if (!s || !n) return PP_EINVAL;
  *n = static_cast<uint64_t>(s->P);
  return PP_OK;
}

pp_status pp_sur_get_training_rows(pp_surrogate *s, uint64_t first, uint64_t count, float *features, float *mu_base,
                                   float *k, float *n_t, float *s1, float *s2) {
  if (!s) return PP_EINVAL;
  pp_context *ctx = s->ctx;
  if (first + count > static_cast<uint64_t>(s->P)) return fail(ctx, PP_EINVAL, "rows out of range");
  PP_HIP(ctx, hipSetDevice(ctx->device));
  PP_HIP(ctx, hipDeviceSynchronize());
  if (features) {
    std::vector<uint16_t> xb(count * sur::kInPad);
    PP_HIP(ctx, hipMemcpy(xb.data(), s->X + first * sur::kInPad, sizeof(uint16_t) * xb.size(), hipMemcpyDeviceToHost));
    for (uint64_t r = 0; r < count; ++r)
      for (int q = 0; q < sur::kInReal; ++q) {
        const uint32_t u = static_cast<uint32_t>(xb[r * sur::kInPad + q]) << 16;
        std::memcpy(&features[r * sur::kInReal + q], &u, 4);
      }
  }
  float *dst[5] = {mu_base, k, n_t, s1, s2};
  float *src[5] = {s->mu_base, s->k, s->n_t, s->s1, s->s2};
  for (int i = 0; i < 5; ++i)
    if (dst[i] && count) PP_HIP(ctx, hipMemcpy(dst[i], src[i] + first, sizeof(float) * count, hipMemcpyDeviceToHost));
  return PP_OK;
}

pp_status pp_sur_loss_grad(pp_surrogate *s, uint64_t first, uint64_t count, double *loss, float *grad) {
  if (!s) return PP_EINVAL;
  pp_status st = need_device(s->ctx);
  if (st != PP_OK) return st;
  if ((st = check_rows(s, static_cast<int64_t>(first), static_cast<int64_t>(count))) != PP_OK) return st;
  if ((st = train_pass(s, 1, 0, static_cast<int64_t>(first), static_cast<int64_t>(count), false, 0.0f, nullptr)) !=
      PP_OK)
    return st;
  PP_HIP(s->ctx, hipDeviceSynchronize());
  if (loss) {
    double l = 0;
    PP_HIP(s->ctx, hipMemcpy(&l, s->d_loss, sizeof(double), hipMemcpyDeviceToHost));
    *loss = l / static_cast<double>(count);
  }
  if (grad) PP_HIP(s->ctx, hipMemcpy(grad, s->grad, sizeof(float) * sur::param_count(), hipMemcpyDeviceToHost));
  return PP_OK;
}

pp_status pp_sur_train_step(pp_surrogate *s, uint64_t first, uint64_t count, float lr, double *loss) {
  if (!s) return PP_EINVAL;
  pp_status st = need_device(s->ctx);
  if (st != PP_OK) return st;
  if ((st = check_rows(s, static_cast<int64_t>(first), static_cast<int64_t>(count))) != PP_OK) return st;
  if ((st = train_pass(s, 1, 0, static_cast<int64_t>(first), static_cast<int64_t>(count), true, lr, nullptr)) !=
      PP_OK)
    return st;
  PP_HIP(s->ctx, hipDeviceSynchronize());
  if (loss) {
    double l = 0;
    PP_HIP(s->ctx, hipMemcpy(&l, s->d_loss, sizeof(double), hipMemcpyDeviceToHost));
    *loss = l / static_cast<double>(count);
  }
  return PP_OK;
}

pp_status pp_sur_train(pp_surrogate *s, uint32_t epochs, uint32_t batch_size, float lr, float lr_final,
                       void *hip_stream, float *epoch_loss) {
  if (!s) return PP_EINVAL;
  pp_context *ctx = s->ctx;
  pp_status st = need_device(ctx);
  if (st != PP_OK) return st;
  if (batch_size == 0 || batch_size % 64 != 0 || batch_size > (1u << 30))
    return fail(ctx, PP_EINVAL, "batch_size must be a positive multiple of 64, at most 2^30");
  if (!(lr >= 0.0f) || !(lr_final >= 0.0f) || !std::isfinite(lr) || !std::isfinite(lr_final))
    return fail(ctx, PP_EINVAL, "learning rates must be finite and non-negative");
  if (s->P == 0) return fail(ctx, PP_ESTATE, "no training set");
  if (static_cast<uint64_t>(s->P) >= (1ull << 32)) return fail(ctx, PP_EINVAL, "training set above 2^32 rows");
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  double *d_epoch = nullptr;
  if ((st = dalloc(ctx, &d_epoch, 1)) != PP_OK) return st;
  s->epoch_loss = d_epoch;
  const uint64_t P = static_cast<uint64_t>(s->P);
  const int64_t steps_per_epoch = (s->P + batch_size - 1) / batch_size;
  const double total_steps = static_cast<double>(steps_per_epoch) * epochs;
  int64_t step = 0;
  for (uint32_t e = 0; e < epochs; ++e) {
    // this epoch's row order: p(r) = (mul r + add) mod P with mul coprime to
    // P, mul / P stepping through the golden-ratio sequence so consecutive
    // rows come from sources spread over the whole set
    std::mt19937_64 rng(s->shuffle_seed + 0x9E3779B97F4A7C15ull * (s->epochs_done + 1));
    double frac = std::fmod(0.6180339887498949 * static_cast<double>(s->epochs_done + 1), 1.0);
    if (frac < 0.1 || frac > 0.9) frac = 0.5 * frac + 0.25;
    uint64_t mul = std::max<uint64_t>(1, static_cast<uint64_t>(frac * static_cast<double>(P))) % P;
    if (mul == 0) mul = 1;
    while (gcd64(mul, P) != 1) mul = mul + 1 < P ? mul + 1 : 1;
    const uint64_t add = rng() % P;
    s->epochs_done += 1;
    PP_HIP(ctx, sur::launch_zero_f64(d_epoch, 1, stream));
    for (int64_t first = 0; first < s->P; first += batch_size, ++step) {
      const int64_t count = std::min<int64_t>(batch_size, s->P - first);
      // cosine decay from lr to lr_final over this call's steps
      const double c = 0.5 * (1.0 + std::cos(M_PI * static_cast<double>(step) / total_steps));
      const float lr_t = static_cast<float>(lr_final + (lr - lr_final) * c);
      if ((st = train_pass(s, mul, add, first, count, true, lr_t, stream)) != PP_OK) break;
    }
    if (st != PP_OK) break;
    if (epoch_loss) {
      double l = 0;
      PP_HIP(ctx, hipMemcpyAsync(&l, d_epoch, sizeof(double), hipMemcpyDeviceToHost, stream));
      PP_HIP(ctx, hipStreamSynchronize(stream));
      epoch_loss[e] = static_cast<float>(l / static_cast<double>(s->P));
    }
  }
  s->epoch_loss = nullptr;
  PP_HIP(ctx, hipStreamSynchronize(stream));
  dfree(d_epoch);
  return st;
}

pp_status pp_sur_expected_hits(pp_surrogate *s, uint64_t batch, double *dev_dom_sums, void *hip_stream) {
  if (!s || !dev_dom_sums) return PP_EINVAL;
  pp_context *ctx = s->ctx;
  pp_status st = need_device(ctx);
  if (st != PP_OK) return st;
  Batch *b;
  if ((st = find_batch(ctx, batch, &b)) != PP_OK) return st;
  if ((st = check_cherenkov(ctx, *b)) != PP_OK) return st;
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  PP_HIP(ctx, sur::launch_zero_f64(dev_dom_sums, s->n_doms, stream));
  using NoSink = pp_status (*)(const float *, int64_t, int64_t);
  return infer<NoSink>(s, *b, stream, dev_dom_sums, nullptr);
}

}  // extern "C"

namespace ppi {

pp_status sur_predict_batch(pp_surrogate *s, Batch &b, float *out) {
  pp_context *ctx = s->ctx;
  pp_status st = check_cherenkov(ctx, b);
  if (st != PP_OK) return st;
  auto sink = [&](const float *mu, int64_t s0, int64_t ns) -> pp_status {
    PP_HIP(ctx, hipMemcpy(out + s0 * s->n_doms, mu, sizeof(float) * ns * s->n_doms, hipMemcpyDeviceToHost));
    return PP_OK;
  };
  return infer(s, b, nullptr, nullptr, &sink);
}

}  // namespace ppi

extern "C" {

pp_status pp_sur_predict_pairs(pp_surrogate *s, uint64_t batch, float *out, uint64_t n) {
  if (!s || !out) return PP_EINVAL;
  pp_context *ctx = s->ctx;
  pp_status st = need_device(ctx);
  if (st != PP_OK) return st;
  Batch *b;
  if ((st = find_batch(ctx, batch, &b)) != PP_OK) return st;
  if ((st = check_cherenkov(ctx, *b)) != PP_OK) return st;
  if (n != b->src.size() * static_cast<uint64_t>(s->n_doms)) return fail(ctx, PP_EINVAL, "output size mismatch");
  auto sink = [&](const float *mu, int64_t s0, int64_t ns) -> pp_status {
    PP_HIP(ctx, hipMemcpy(out + s0 * s->n_doms, mu, sizeof(float) * ns * s->n_doms, hipMemcpyDeviceToHost));
    return PP_OK;
  };
  return infer(s, *b, nullptr, nullptr, &sink);
}

}  // extern "C"

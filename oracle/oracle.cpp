// FP64 CPU oracle for photon propagation through layered ice.
//
// TEST INFRASTRUCTURE ONLY. This file is the plain, slow reference that
// judges the GPU path. Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark may load it; the product path never does.
// It shares no code, header, table or constant generator with the HIP path.
//
// What it computes (Meagher & van Santen, "Parallelizing Air Shower
// Simulation for Background Characterization in IceCube", Sec. 2, photon
// propagation paragraph): light sources emit photons; the ice is split into
// 10 m horizontal layers, each with its own absorption and scattering
// coefficients; for each photon a Monte Carlo draws the distance to the next
// scatter, then a new direction from the scattering physics, and repeats
// until the photon reaches an optical module (a hit) or is absorbed. A hit
// carries the producing particle's id, the hit time and a weight (Sec. 4,
// hit-record paragraph).
//
// The paper gives no formulas for these steps. Every step below follows a
// textbook definition, and every choice the paper leaves open is one of the
// numbered readings listed with the design notes:
//   * random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
//     key = 64-bit seed, counter = (block k, event id, photon index lo, hi);
//     block 0 feeds emission, block 2+j feeds loop iteration j;
//   * u32 -> uniform: (2*(w >> 9) + 1) * 2^-24, exact in FP32 and FP64;
//   * analog absorption: one optical-depth budget per photon drawn at
//     emission, a fresh scattering optical depth per iteration, both
//     consumed layer by layer (tie order absorb <= scatter <= boundary);
//   * Henyey-Greenstein scattering with the layer's mean cosine g;
//   * direction rotation about the current direction with the orthonormal
//     basis of Duff et al., JCGT 6(1) 2017;
//   * optical modules are spheres; the first sphere crossed along a step is
//     hit (ties go to the lower module id) and the photon ends there;
//   * time advances by path length * n_group / c; hit weight is 1.
//
// Everything runs in double precision. Photons are independent; threads take
// static contiguous slices of the requested photon list, so results do not
// depend on the thread count.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

namespace {

const double kInf = std::numeric_limits<double>::infinity();
const double kPi = 3.14159265358979323846;
const double kLightSpeed = 0.299792458;  // metres per nanosecond

enum Fate : uint32_t { kAbsorbed = 0, kHit = 1, kCapped = 2, kEscaped = 3 };
const uint32_t kNoDom = 0xFFFFFFFFu;

// ---------------------------------------------------------------- Philox --
// Philox4x32 with 10 rounds, as defined by Salmon et al. (SC'11): each round
// multiplies counter words 0 and 2 by two fixed odd constants, and the new
// counter is (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));
// between rounds the key is bumped by the two Weyl constants.
void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = static_cast<uint64_t>(M0) * c0;
    const uint64_t p1 = static_cast<uint64_t>(M1) * c2;
    const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n1 = static_cast<uint32_t>(p1);
    const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
    const uint32_t n3 = static_cast<uint32_t>(p0);
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// One 4-word block of the photon's stream: counter = (k, event, index lo, hi).
void photon_block(uint64_t seed, uint32_t k, uint32_t event, uint64_t photon_index,
                  uint32_t w[4]) {
  const uint32_t ctr[4] = {k, event, static_cast<uint32_t>(photon_index),
                           static_cast<uint32_t>(photon_index >> 32)};
  const uint32_t key[2] = {static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32)};
  philox4x32_10(ctr, key, w);
}

// u in (0, 1): the centre of one of 2^23 equal bins, an odd multiple of 2^-24.
double uniform(uint32_t w) { return (2.0 * static_cast<double>(w >> 9) + 1.0) * 0x1p-24; }

// ------------------------------------------------------------ geometry --
struct Vec {
  double x, y, z;
};
Vec operator+(Vec a, Vec b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
Vec operator-(Vec a, Vec b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
Vec operator*(double s, Vec a) { return {s * a.x, s * a.y, s * a.z}; }
double dot(Vec a, Vec b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
Vec normalized(Vec a) { return (1.0 / std::sqrt(dot(a, a))) * a; }

// Orthonormal basis (e1, e2) perpendicular to the unit vector n, built with
// the branch-free construction of Duff et al. (JCGT 2017), which has no
// singular direction.
void basis(Vec n, Vec *e1, Vec *e2) {
  const double sign = std::copysign(1.0, n.z);
  const double a = -1.0 / (sign + n.z);
  const double b = n.x * n.y * a;
  *e1 = {1.0 + sign * n.x * n.x * a, sign * b, -sign * n.x};
  *e2 = {b, sign + n.y * n.y * a, -n.y};
}

// Direction at polar cosine mu = 1 - om and azimuth 2*pi*phi_turns about v.
Vec rotate(Vec v, double om, double phi_turns) {
  const double mu = 1.0 - om;
  const double sin_t = std::sqrt(om * (2.0 - om));
  const double phi = 2.0 * kPi * phi_turns;
  Vec e1, e2;
  basis(v, &e1, &e2);
  const Vec out = mu * v + sin_t * (std::cos(phi) * e1 + std::sin(phi) * e2);
  return normalized(out);
}

// Henyey-Greenstein: returns 1 - mu for uniform u. The textbook inverse CDF
// mu = (1 + g^2 - ((1 - g^2) / (1 - g + 2 g u))^2) / (2 g) is rewritten,
// exactly, as 1 - mu = (1 - g)(1 - u)(s + 1 - g) / w with w = 1 - g + 2 g u
// and s = (1 - g^2) / w. This form has no division by g (g = 0 gives the
// isotropic mu = 2u - 1) and no cancellation near mu = 1.
double hg_one_minus_mu(double g, double u) {
  const double w = 1.0 - g + 2.0 * g * u;
  const double s = (1.0 - g * g) / w;
  return (1.0 - g) * (1.0 - u) * (s + 1.0 - g) / w;
}

// ----------------------------------------------------------------- model --
struct Ice {
  double z_lo = 0, dz = 10;
  int n_layers = 0;
  double n_group = 1.35;
  std::vector<double> abs_coef, scat_coef, g;  // a = 1/lambda_a, b = 1/(lambda_e (1 - g))
  // Wavelength dependence of the coefficients (the table holds them at
  // lambda_ref): a(l) = a (l / lambda_ref)^-kappa_abs, b(l) likewise with
  // kappa_scat; lambda_ref = 0 means none.
  double lambda_ref = 0, kappa_abs = 0, kappa_scat = 0;
};

// Hit weight: acceptance A(lambda), linear between table values at
// l0 + k dl (held constant beyond the ends), times a polynomial P(c) in the
// cosine c of the angle between the photon's direction and the inward
// surface normal where it meets the module. An empty table means weight 1.
struct Acceptance {
  std::vector<double> table, poly;
  double l0 = 0, dl = 1;
};

struct Source {
  int type = 0;  // 0 isotropic point, 1 Cherenkov track segment
  uint32_t event = 0, particle = 0;
  Vec pos{0, 0, 0}, dir{0, 0, 1};
  double t0 = 0, length = 0, cos_ck = 0, sin_ck = 0, lmin = 405, lmax = 405;
  uint64_t n_photons = 0, first_index = 0;
};

struct Doms {
  std::vector<Vec> c;
  double r = 0.1651;
  // optional per-string pre-filter: for each string, the DOM ids it holds,
  // its horizontal centre and its reach (largest horizontal DOM offset + r)
  std::vector<std::vector<uint32_t>> string_doms;
  std::vector<double> sx, sy, reach;
};

struct Photon {
  Vec p, v;
  double t, tau_a, lambda;
  int layer;
};

struct Record {
  uint32_t fate, dom, n_iter, n_cross;
  double t, x, y, z, vx, vy, vz, lambda, weight;
};

// Layer i covers [z_lo + i dz, z_lo + (i+1) dz); the edge layers extend to
// infinity. The index is taken from z only at emission.
int layer_of(const Ice &ice, double z) {
  const double f = std::floor((z - ice.z_lo) / ice.dz);
  if (!(f >= 0.0)) return 0;
  if (f >= ice.n_layers - 1) return ice.n_layers - 1;
  return static_cast<int>(f);
}

// Emission from Philox block 0 (words w0..w3).
Photon emit(const Ice &ice, const Source &s, uint64_t seed, uint64_t photon_index) {
  uint32_t w[4];
  photon_block(seed, 0, s.event, photon_index, w);
  Photon ph;
  if (s.type == 0) {
    // isotropic point: cos(theta) = 2 u0 - 1, azimuth 2 pi u1
    const double ct = 2.0 * uniform(w[0]) - 1.0;
    const double st = std::sqrt((1.0 - ct) * (1.0 + ct));
    const double phi = 2.0 * kPi * uniform(w[1]);
    ph.p = s.pos;
    ph.v = {st * std::cos(phi), st * std::sin(phi), ct};
    ph.t = s.t0;
  } else {
    // Cherenkov segment: uniform point along the track, fixed cone angle
    // about the track direction, azimuth 2 pi u1; the emitting particle
    // moves at the speed of light.
    const double sdist = uniform(w[0]) * s.length;
    ph.p = s.pos + sdist * s.dir;
    ph.t = s.t0 + sdist / kLightSpeed;
    const double psi = 2.0 * kPi * uniform(w[1]);
    Vec e1, e2;
    basis(s.dir, &e1, &e2);
    ph.v = normalized(s.cos_ck * s.dir + s.sin_ck * (std::cos(psi) * e1 + std::sin(psi) * e2));
  }
  ph.tau_a = -std::log(uniform(w[2]));
  if (s.lmin == s.lmax) {
    ph.lambda = s.lmin;
  } else {
    // inverse CDF of a density proportional to 1/lambda^2 on [lmin, lmax]
    const double inv = 1.0 / s.lmin - uniform(w[3]) * (1.0 / s.lmin - 1.0 / s.lmax);
    ph.lambda = 1.0 / inv;
  }
  ph.layer = layer_of(ice, ph.p.z);
  return ph;
}

// First sphere crossed along the segment [p, p + len v]; ties in distance go
// to the lower id. A sphere that contains p is ignored. Returns kNoDom if
// none; *t_hit receives the distance along v.
struct HitTest {
  double best_t;
  uint32_t best_id;
  uint64_t tests;
};

void test_sphere(const Doms &doms, uint32_t id, Vec p, Vec v, double len, HitTest *h) {
  h->tests++;
  const Vec d = p - doms.c[id];
  const double b = dot(d, v);
  const Vec perp = d - b * v;
  const double disc = doms.r * doms.r - dot(perp, perp);
  if (disc < 0.0) return;
  if (dot(d, d) < doms.r * doms.r) return;  // starts inside: ignored
  const double t = -b - std::sqrt(disc);
  if (!(t >= 0.0 && t <= len)) return;
  if (t < h->best_t || (t == h->best_t && id < h->best_id)) {
    h->best_t = t;
    h->best_id = id;
  }
}

HitTest find_hit(const Doms &doms, int mode, Vec p, Vec v, double len) {
  HitTest h{kInf, kNoDom, 0};
  if (mode == 0) {
    // brute force: every module, ascending id
    for (uint32_t id = 0; id < doms.c.size(); ++id) test_sphere(doms, id, p, v, len, &h);
  } else {
    // exact pre-filter: a string whose horizontal centre lies farther than
    // len + reach from p cannot be crossed by the segment
    for (size_t s = 0; s < doms.string_doms.size(); ++s) {
      const double dx = doms.sx[s] - p.x, dy = doms.sy[s] - p.y;
      const double lim = len + doms.reach[s] + 1e-6;
      if (dx * dx + dy * dy > lim * lim) continue;
      for (uint32_t id : doms.string_doms[s]) test_sphere(doms, id, p, v, len, &h);
    }
  }
  return h;
}

struct Counters {
  uint64_t photons = 0, iterations = 0, crossings = 0, dom_tests = 0;
  uint64_t hits = 0, absorbed = 0, capped = 0, escaped = 0;
};

// Propagates one photon to its end. The loop follows the paper's order:
// distance to the next scatter, move (absorbed or hitting a module on the
// way ends the photon), new direction, repeat.
double hit_weight(const Acceptance &acc, const Doms &doms, uint32_t dom, const Photon &ph) {
  if (acc.table.empty()) return 1.0;
  double A = acc.table[0];
  if (acc.table.size() > 1) {
    const double x = std::min(std::max((ph.lambda - acc.l0) / acc.dl, 0.0),
                              static_cast<double>(acc.table.size() - 1));
    const size_t k = std::min(static_cast<size_t>(x), acc.table.size() - 2);
    const double f = x - static_cast<double>(k);
    A = acc.table[k] * (1.0 - f) + acc.table[k + 1] * f;
  }
  const Vec n = (1.0 / doms.r) * (ph.p - doms.c[dom]);  // outward unit normal at the hit point
  const double c = std::min(std::max(-dot(ph.v, n), 0.0), 1.0);
  double P = 0.0;
  for (size_t k = acc.poly.size(); k-- > 0;) P = P * c + acc.poly[k];
  return A * P;
}

Record propagate(const Ice &ice, const Doms &doms, const Acceptance &acc, const Source &src,
                 uint64_t seed, uint64_t photon_index, uint64_t step_cap, int mode, Counters *cnt) {
  Photon ph = emit(ice, src, seed, photon_index);
  const double time_per_m = ice.n_group / kLightSpeed;
  // the photon's coefficients are the table's scaled to its wavelength
  const double sa = ice.lambda_ref > 0 ? std::pow(ph.lambda / ice.lambda_ref, -ice.kappa_abs) : 1.0;
  const double sb = ice.lambda_ref > 0 ? std::pow(ph.lambda / ice.lambda_ref, -ice.kappa_scat) : 1.0;
  Record rec{};
  rec.dom = kNoDom;
  rec.lambda = ph.lambda;
  rec.weight = 1.0;
  uint32_t fate = kCapped;
  uint64_t iter = 0;
  uint32_t n_cross = 0;
  while (iter < step_cap) {
    uint32_t w[4];
    photon_block(seed, static_cast<uint32_t>(2 + iter), src.event, photon_index, w);
    ++iter;
    double tau_s = -std::log(uniform(w[0]));

    // Walk the layers from the current point, consuming both optical-depth
    // budgets, until one is exhausted. Distances to layer boundaries come
    // from the carried layer index and the current boundary height.
    double len = 0.0, zc = ph.p.z;
    int i = ph.layer;
    enum { kStepAbsorb, kStepScatter, kStepEscape } step_end;
    const int dir = ph.v.z > 0.0 ? 1 : (ph.v.z < 0.0 ? -1 : 0);
    for (;;) {
      const double a = ice.abs_coef[i] * sa, b = ice.scat_coef[i] * sb;
      const double d_abs = a > 0.0 ? ph.tau_a / a : kInf;
      const double d_sca = b > 0.0 ? tau_s / b : kInf;
      double d_bnd = kInf;
      if (dir > 0 && i < ice.n_layers - 1) {
        d_bnd = std::max(0.0, (ice.z_lo + (i + 1) * ice.dz - zc) / ph.v.z);
      } else if (dir < 0 && i > 0) {
        d_bnd = std::max(0.0, (ice.z_lo + i * ice.dz - zc) / ph.v.z);
      }
      if (d_abs == kInf && d_sca == kInf && d_bnd == kInf) {
        // nothing stops the photon: it leaves along a straight line
        len = kInf;
        step_end = kStepEscape;
        break;
      }
      if (d_abs <= d_sca && d_abs <= d_bnd) {
        len += d_abs;
        ph.tau_a = 0.0;
        step_end = kStepAbsorb;
        break;
      }
      if (d_sca <= d_bnd) {
        len += d_sca;
        ph.tau_a = std::max(0.0, ph.tau_a - a * d_sca);
        tau_s = 0.0;
        step_end = kStepScatter;
        break;
      }
      len += d_bnd;
      ph.tau_a = std::max(0.0, ph.tau_a - a * d_bnd);
      tau_s = std::max(0.0, tau_s - b * d_bnd);
      zc = ice.z_lo + (dir > 0 ? i + 1 : i) * ice.dz;
      i += dir;
      ++n_cross;
    }
    ph.layer = i;

    const HitTest h = find_hit(doms, mode, ph.p, ph.v, len);
    cnt->dom_tests += h.tests;
    if (h.best_id != kNoDom) {
      ph.p = ph.p + h.best_t * ph.v;
      ph.t += h.best_t * time_per_m;
      fate = kHit;
      rec.dom = h.best_id;
      rec.weight = hit_weight(acc, doms, h.best_id, ph);
      break;
    }
    if (step_end == kStepEscape) {
      fate = kEscaped;
      break;
    }
    ph.p = ph.p + len * ph.v;
    ph.t += len * time_per_m;
    if (step_end == kStepAbsorb) {
      fate = kAbsorbed;
      break;
    }
    // scatter: Henyey-Greenstein polar angle with the layer's g, uniform
    // azimuth
    const double om = hg_one_minus_mu(ice.g[ph.layer], uniform(w[1]));
    ph.v = rotate(ph.v, om, uniform(w[2]));
  }
  rec.fate = fate;
  rec.n_iter = static_cast<uint32_t>(iter);
  rec.n_cross = n_cross;
  rec.t = ph.t;
  rec.x = ph.p.x;
  rec.y = ph.p.y;
  rec.z = ph.p.z;
  rec.vx = ph.v.x;
  rec.vy = ph.v.y;
  rec.vz = ph.v.z;
  cnt->photons++;
  cnt->iterations += iter;
  cnt->crossings += n_cross;
  cnt->hits += fate == kHit;
  cnt->absorbed += fate == kAbsorbed;
  cnt->capped += fate == kCapped;
  cnt->escaped += fate == kEscaped;
  return rec;
}

}  // namespace

// ------------------------------------------------------------- C ABI --
extern "C" {

// Philox4x32-10 blocks for n (counter, key) pairs: ctr is n x 4, key n x 2,
// out n x 4 words.
void orc_philox(uint64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out) {
  for (uint64_t i = 0; i < n; ++i) philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

void orc_uniform(uint64_t n, const uint32_t *w, double *u) {
  for (uint64_t i = 0; i < n; ++i) u[i] = uniform(w[i]);
}

void orc_hg_one_minus_mu(uint64_t n, double g, const double *u, double *om) {
  for (uint64_t i = 0; i < n; ++i) om[i] = hg_one_minus_mu(g, u[i]);
}

// v: n x 3 unit vectors; om, phi_turns: n; out: n x 3
void orc_rotate(uint64_t n, const double *v, const double *om, const double *phi_turns,
                double *out) {
  for (uint64_t i = 0; i < n; ++i) {
    const Vec r = rotate({v[3 * i], v[3 * i + 1], v[3 * i + 2]}, om[i], phi_turns[i]);
    out[3 * i] = r.x;
    out[3 * i + 1] = r.y;
    out[3 * i + 2] = r.z;
  }
}

// v: n x 3; e1, e2: n x 3
void orc_basis(uint64_t n, const double *v, double *e1, double *e2) {
  for (uint64_t i = 0; i < n; ++i) {
    Vec a, b;
    basis({v[3 * i], v[3 * i + 1], v[3 * i + 2]}, &a, &b);
    e1[3 * i] = a.x, e1[3 * i + 1] = a.y, e1[3 * i + 2] = a.z;
    e2[3 * i] = b.x, e2[3 * i + 1] = b.y, e2[3 * i + 2] = b.z;
  }
}

// First-hit query: n segments (p n x 3, v n x 3, len n) against a set of
// spheres; ids out (0xFFFFFFFF = none) and distances.
void orc_first_hit(uint64_t n, const double *p, const double *v, const double *len,
                   uint32_t n_dom, const double *dom_xyz, double radius, uint32_t *id_out,
                   double *t_out) {
  Doms doms;
  doms.r = radius;
  for (uint32_t k = 0; k < n_dom; ++k)
    doms.c.push_back({dom_xyz[3 * k], dom_xyz[3 * k + 1], dom_xyz[3 * k + 2]});
  for (uint64_t i = 0; i < n; ++i) {
    const HitTest h = find_hit(doms, 0, {p[3 * i], p[3 * i + 1], p[3 * i + 2]},
                               {v[3 * i], v[3 * i + 1], v[3 * i + 2]}, len[i]);
    id_out[i] = h.best_id;
    t_out[i] = h.best_t;
  }
}

// Inputs shared by orc_emit and orc_run.
//   ice: z_lo, dz, n_layers, n_group; per layer abs_len (m), eff_scat_len (m,
//        lambda_e = lambda_s / (1 - g)), g. Infinite lengths mean no
//        absorption / no scattering in that layer.
//   sources (n_src): type, event, particle; sf is n_src x 11 doubles
//        (x, y, z, dx, dy, dz, t0_ns, length_m, cherenkov_deg, lambda_min,
//        lambda_max); n_photons; first_photon_index.
struct OrcInputs {
  double z_lo, dz;
  int32_t n_layers;
  double n_group;
  const double *abs_len, *eff_scat_len, *g;
  uint32_t n_dom;
  const double *dom_xyz;
  const int32_t *dom_string;
  double dom_radius;
  uint32_t n_src;
  const int32_t *src_type;
  const uint32_t *src_event, *src_particle;
  const double *src_f;
  const uint64_t *src_n, *src_first;
  // wavelength dependence: lambda_ref (0: none), kappa_abs, kappa_scat
  double lambda_ref, kappa_abs, kappa_scat;
  // hit acceptance: n_acc table values at acc_l0 + k acc_dl (0: weight 1)
  // and n_poly coefficients of P(c), lowest order first
  uint32_t n_acc, n_poly;
  double acc_l0, acc_dl;
  const double *acc, *poly;
};

static void build_model(const OrcInputs *in, Ice *ice, Doms *doms, std::vector<Source> *src,
                        Acceptance *acc = nullptr) {
  ice->lambda_ref = in->lambda_ref;
  ice->kappa_abs = in->kappa_abs;
  ice->kappa_scat = in->kappa_scat;
  if (acc && in->n_acc > 0) {
    acc->table.assign(in->acc, in->acc + in->n_acc);
    acc->poly.assign(in->poly, in->poly + in->n_poly);
    acc->l0 = in->acc_l0;
    acc->dl = in->acc_dl;
  }
  ice->z_lo = in->z_lo;
  ice->dz = in->dz;
  ice->n_layers = in->n_layers;
  ice->n_group = in->n_group;
  for (int i = 0; i < in->n_layers; ++i) {
    const double g = in->g[i];
    ice->g.push_back(g);
    ice->abs_coef.push_back(1.0 / in->abs_len[i]);
    ice->scat_coef.push_back(1.0 / (in->eff_scat_len[i] * (1.0 - g)));
  }
  doms->r = in->dom_radius;
  for (uint32_t k = 0; k < in->n_dom; ++k)
    doms->c.push_back({in->dom_xyz[3 * k], in->dom_xyz[3 * k + 1], in->dom_xyz[3 * k + 2]});
  if (in->dom_string) {
    std::vector<int32_t> keys(in->dom_string, in->dom_string + in->n_dom);
    std::vector<int32_t> uniq = keys;
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    doms->string_doms.assign(uniq.size(), {});
    for (uint32_t k = 0; k < in->n_dom; ++k) {
      const size_t s = std::lower_bound(uniq.begin(), uniq.end(), keys[k]) - uniq.begin();
      doms->string_doms[s].push_back(k);
    }
    for (const auto &ids : doms->string_doms) {
      double cx = 0, cy = 0;
      for (uint32_t k : ids) cx += doms->c[k].x, cy += doms->c[k].y;
      cx /= ids.size();
      cy /= ids.size();
      double reach = 0;
      for (uint32_t k : ids)
        reach = std::max(reach, std::hypot(doms->c[k].x - cx, doms->c[k].y - cy));
      doms->sx.push_back(cx);
      doms->sy.push_back(cy);
      doms->reach.push_back(reach + doms->r);
    }
  }
  for (uint32_t j = 0; j < in->n_src; ++j) {
    const double *f = in->src_f + 11 * j;
    Source s;
    s.type = in->src_type[j];
    s.event = in->src_event[j];
    s.particle = in->src_particle[j];
    s.pos = {f[0], f[1], f[2]};
    s.dir = s.type == 1 ? normalized({f[3], f[4], f[5]}) : Vec{0, 0, 1};
    s.t0 = f[6];
    s.length = f[7];
    s.cos_ck = std::cos(f[8] * kPi / 180.0);
    s.sin_ck = std::sin(f[8] * kPi / 180.0);
    s.lmin = f[9];
    s.lmax = f[10];
    s.n_photons = in->src_n[j];
    s.first_index = in->src_first[j];
    src->push_back(s);
  }
}

// Emission state of selected photons (cap-free): p, v, t, tau_a, lambda,
// layer. out_f is n x 9 (x y z vx vy vz t tau_a lambda), out_layer n.
int orc_emit(const OrcInputs *in, uint64_t seed, uint64_t n_sel, const uint64_t *sel_src,
             const uint64_t *sel_local, double *out_f, int32_t *out_layer) {
  Ice ice;
  Doms doms;
  std::vector<Source> src;
  build_model(in, &ice, &doms, &src);
  for (uint64_t i = 0; i < n_sel; ++i) {
    if (sel_src[i] >= src.size()) return -1;
    const Source &s = src[sel_src[i]];
    const Photon ph = emit(ice, s, seed, s.first_index + sel_local[i]);
    double *o = out_f + 9 * i;
    o[0] = ph.p.x, o[1] = ph.p.y, o[2] = ph.p.z;
    o[3] = ph.v.x, o[4] = ph.v.y, o[5] = ph.v.z;
    o[6] = ph.t, o[7] = ph.tau_a, o[8] = ph.lambda;
    out_layer[i] = ph.layer;
  }
  return 0;
}

// Propagates photons to their end.
//   selection: if n_sel > 0, the listed (source, local photon number) pairs;
//     if n_sel == 0, every photon of every source, in source order.
//   dom_mode: 0 brute force over all modules, 1 exact per-string pre-filter
//     (needs dom_string).
//   outputs (each may be NULL):
//     rec_u n x 4 (fate, dom id, iterations, layer crossings),
//     rec_f n x 9 (t, x, y, z, vx, vy, vz, lambda, hit weight (1 unless hit)),
//     dom_counts n_dom (hits per module),
//     counters 8 (photons, iterations, crossings, dom tests, hits, absorbed,
//       capped, escaped).
// Returns 0, or -1 on a bad selection.
int orc_run(const OrcInputs *in, uint64_t seed, uint64_t step_cap, int32_t dom_mode,
            int32_t n_threads, uint64_t n_sel, const uint64_t *sel_src,
            const uint64_t *sel_local, uint32_t *rec_u, double *rec_f, uint64_t *dom_counts,
            uint64_t *counters) {
  Ice ice;
  Doms doms;
  Acceptance acc;
  std::vector<Source> src;
  build_model(in, &ice, &doms, &src, &acc);
  if (dom_mode == 1 && !in->dom_string) return -1;

  // The work list: (source, local photon number) per output slot.
  std::vector<uint64_t> prefix(src.size() + 1, 0);
  for (size_t j = 0; j < src.size(); ++j) prefix[j + 1] = prefix[j] + src[j].n_photons;
  const uint64_t n = n_sel > 0 ? n_sel : prefix.back();
  if (n_sel > 0) {
    for (uint64_t i = 0; i < n_sel; ++i)
      if (sel_src[i] >= src.size() || sel_local[i] >= src[sel_src[i]].n_photons) return -1;
  }
  if (n_threads < 1) n_threads = 1;
  std::vector<Counters> cnt(n_threads);
  std::vector<std::vector<uint64_t>> counts(n_threads,
                                            std::vector<uint64_t>(dom_counts ? in->n_dom : 0, 0));
  auto worker = [&](int tid) {
    const uint64_t lo = n * tid / n_threads, hi = n * (tid + 1) / n_threads;
    size_t s = 0;
    for (uint64_t i = lo; i < hi; ++i) {
      uint64_t local;
      if (n_sel > 0) {
        s = sel_src[i];
        local = sel_local[i];
      } else {
        s = std::upper_bound(prefix.begin(), prefix.end(), i) - prefix.begin() - 1;
        local = i - prefix[s];
      }
      const Record r = propagate(ice, doms, acc, src[s], seed, src[s].first_index + local, step_cap,
                                 dom_mode, &cnt[tid]);
      if (rec_u) {
        rec_u[4 * i] = r.fate, rec_u[4 * i + 1] = r.dom;
        rec_u[4 * i + 2] = r.n_iter, rec_u[4 * i + 3] = r.n_cross;
      }
      if (rec_f) {
        double *o = rec_f + 9 * i;
        o[0] = r.t, o[1] = r.x, o[2] = r.y, o[3] = r.z;
        o[4] = r.vx, o[5] = r.vy, o[6] = r.vz, o[7] = r.lambda, o[8] = r.weight;
      }
      if (dom_counts && r.fate == kHit) counts[tid][r.dom]++;
    }
  };
  std::vector<std::thread> pool;
  for (int tid = 1; tid < n_threads; ++tid) pool.emplace_back(worker, tid);
  worker(0);
  for (auto &th : pool) th.join();

  if (dom_counts) {
    for (uint32_t k = 0; k < in->n_dom; ++k) {
      uint64_t c = 0;
      for (int tid = 0; tid < n_threads; ++tid) c += counts[tid][k];
      dom_counts[k] = c;
    }
  }
  if (counters) {
    Counters t;
    for (const Counters &c : cnt) {
      t.photons += c.photons, t.iterations += c.iterations, t.crossings += c.crossings;
      t.dom_tests += c.dom_tests, t.hits += c.hits, t.absorbed += c.absorbed;
      t.capped += c.capped, t.escaped += c.escaped;
    }
    const uint64_t v[8] = {t.photons, t.iterations, t.crossings, t.dom_tests,
                           t.hits,    t.absorbed,   t.capped,    t.escaped};
    std::memcpy(counters, v, sizeof v);
  }
  return 0;
}

}  // extern "C"

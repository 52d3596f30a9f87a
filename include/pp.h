/*
 * pp.h - C ABI of the MI355X photon-propagation library (libpp).
 *
 * The library propagates optical photons from light sources through ice made
 * of horizontal layers, each with its own absorption and scattering, until
 * each photon is absorbed or reaches an optical module (DOM), and returns
 * the hits. This is the GPU stage of the air-shower simulation chain of
 * Meagher & van Santen, "Parallelizing Air Shower Simulation for Background
 * Characterization in IceCube": energy losses inside the detector are light
 * sources (Sec. 2), the ice is split into 10 m layers with their own
 * scattering and absorption coefficients (Sec. 2), a Monte Carlo draws the
 * distance to the next scatter and a new direction until the photon hits a
 * module or is absorbed (Sec. 2), and each hit is stored compactly as the
 * producing particle's id, the hit time and a weight (Sec. 4, hit-record
 * paragraph). The paper's photon server takes blocks of light-emitting steps
 * from many events at once (Sec. 4, propagation-client paragraph); here a
 * block of sources is one submitted batch.
 *
 * Conventions for every entry point:
 *   - Host pointers are read during the call only; the library copies what
 *     it keeps. Output pointers are caller-owned. The context owns all device
 *     memory it allocates.
 *   - Errors are returned as pp_status; pp_last_error() gives a message.
 *     Nothing throws across the ABI.
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - Units: metres, nanoseconds, nanometres. z points up.
 *   - Results depend only on (seed, event_id, photon_index, inputs): never on
 *     batch composition, launch configuration or hardware scheduling.
 *     Randomness is Philox4x32-10 (Salmon et al., SC'11) with key = seed and
 *     counter = (block k, event_id, photon_index low, high); block 0 is
 *     emission, block 2 + j is propagation step j.
 */
#ifndef PP_H_
#define PP_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pp_context pp_context;

typedef enum {
  PP_OK = 0,
  PP_EINVAL = -1,  /* invalid argument or input value */
  PP_ENOMEM = -2,  /* device or host allocation failed */
  PP_EDEVICE = -3, /* HIP runtime error, or no device on this context */
  PP_ESTATE = -4,  /* call out of order (e.g. submit before loading ice) */
  PP_ETRUNC = -5,  /* output buffer smaller than the result; *n_total set */
  PP_EBUDGET = -6  /* request larger than the device-memory budget */
} pp_status;

/* Ice model (Sec. 2: 10 m layers with their own scattering and absorption).
 * Layer i covers z in [z_lo_m + i dz_m, z_lo_m + (i+1) dz_m); layer 0 is the
 * lowest and the two edge layers extend to infinity. A photon's layer is
 * taken from its z once, at emission, and then changed only by crossings. */
typedef struct {
  float z_lo_m;      /* bottom of layer 0 */
  float dz_m;        /* layer thickness, > 0 */
  uint32_t n_layers; /* 1 .. 1024 */
  float n_group;     /* group refractive index: time advances by path * n_group / c */
} pp_ice_header;

typedef struct {
  float abs_len_m;      /* absorption length lambda_a > 0 (+inf: no absorption) */
  float eff_scat_len_m; /* effective scattering length lambda_e = lambda_s / (1 - g) > 0
                           (+inf: no scattering) */
  float g;              /* Henyey-Greenstein mean cosine, -1 < g < 1 */
} pp_ice_layer;

/* Optical module: a sphere of the geometry's common radius. The module id of
 * row k of the array passed to pp_load_geometry is k. Modules sharing a
 * string_id form a string (a near-vertical line); (string_id, om_index)
 * pairs must be unique. */
typedef struct {
  float x, y, z;
  uint32_t string_id;
  uint32_t om_index;
} pp_dom;

enum { PP_SOURCE_POINT = 0, PP_SOURCE_CHERENKOV = 1 };

/* Light source (Sec. 2: energy losses in the detector are the light sources).
 *   PP_SOURCE_POINT: isotropic emission from (x, y, z) at t0_ns; direction,
 *     length and cherenkov_deg are ignored.
 *   PP_SOURCE_CHERENKOV: a straight track segment from (x, y, z) along the
 *     unit vector (dx, dy, dz) (|d| within 1e-3 of 1; renormalised) of
 *     length_m, travelled at the speed of light from t0_ns; photons leave at
 *     cherenkov_deg to the track, from a point uniform along it.
 * Wavelengths: lambda_min_nm == lambda_max_nm gives that fixed wavelength,
 * otherwise a density proportional to 1/lambda^2 on [min, max].
 * Photons of a source get photon indices first_photon_index ..
 * first_photon_index + n_photons - 1 within event event_id; index ranges of
 * one event must not overlap within a batch. n_photons == 0 is allowed. */
typedef struct {
  uint32_t type;
  uint32_t event_id;
  uint32_t particle_id;
  uint32_t reserved0;
  float x, y, z;
  float dx, dy, dz;
  float t0_ns;
  float length_m;
  float cherenkov_deg;
  float lambda_min_nm;
  float lambda_max_nm;
  float reserved1;
  uint64_t n_photons;
  uint64_t first_photon_index;
} pp_source; /* 80 bytes */

/* Hit (Sec. 4: the compact record keeps the producing particle's id, the
 * hit time and a weight; the event id, photon index and module id identify
 * it). weight is 1 unless an acceptance is set with pp_set_acceptance (the
 * paper gives no photoelectron-probability formula). */
typedef struct {
  uint64_t photon_index;
  uint32_t event_id;
  uint32_t particle_id;
  uint32_t dom_id;
  float time_ns;
  float weight;
  uint32_t reserved;
} pp_hit; /* 32 bytes */

enum { PP_FATE_ABSORBED = 0, PP_FATE_HIT = 1, PP_FATE_CAPPED = 2, PP_FATE_ESCAPED = 3 };

/* Per-photon terminal record, for parity checks only (Sec. 4 calls such
 * diagnostic records useful for debugging and unnecessary in production, so
 * they are off by default). Position and direction are those at the end: the
 * hit point, the absorption point, the point after the last capped step, or
 * for an escaping photon the start of its infinite last step. */
typedef struct {
  uint32_t fate;   /* PP_FATE_* */
  uint32_t dom_id; /* hit module, 0xFFFFFFFF otherwise */
  uint32_t n_iter; /* propagation steps taken */
  uint32_t n_cross;/* layer boundaries crossed */
  float time_ns;
  float x, y, z;
  float vx, vy, vz;
  float wavelength_nm;
} pp_photon_record; /* 48 bytes */

typedef struct {
  uint64_t photons;         /* photons emitted */
  uint64_t iterations;      /* propagation steps */
  uint64_t layer_crossings;
  uint64_t dom_tests;       /* ray-sphere tests performed */
  uint64_t hits, absorbed, capped, escaped;
  float kernel_ms;          /* device time of the propagation kernel */
  uint32_t block_size;      /* launch actually used: threads per workgroup, */
  uint32_t grid_blocks;     /*   workgroups, */
  uint32_t chunk_size;      /*   photon ids per queue grab, */
  uint32_t refill_interval; /*   passes between refills */
} pp_stats;

/* Launch parameters. They change speed only, never results. Zero picks the
 * default. */
typedef struct {
  uint32_t block_size;  /* threads per workgroup, multiple of 64, <= 1024 (default 256, or larger
                           when the modules are staged in LDS, so that a CU runs 24 wavefronts) */
  uint32_t chunk_size;  /* photon ids taken per queue grab by one wavefront (default 256) */
  uint32_t grid_blocks; /* workgroups launched (default: enough to fill every CU) */
  uint32_t refill_interval; /* passes between refills of a wavefront's ended lanes
                               (default 4) */
  uint64_t hit_capacity;/* initial device hit-buffer size in hits (default from photons) */
} pp_launch_config;

typedef struct {
  uint32_t n_doms, n_strings;
  uint32_t grid_nx, grid_ny;
  float grid_x0_m, grid_y0_m, cell_m;
  float max_reach_m; /* largest horizontal DOM offset from its string centre + radius */
} pp_geometry_info;

/* Creates a context on HIP device hip_device (>= 0) with the given Philox
 * seed. hip_device == -1 creates a host-only context: loading and
 * submission work (validation, geometry indexing) but device calls return
 * PP_EDEVICE. *out receives the context; on failure *out is NULL. */
pp_status pp_create(int hip_device, uint64_t seed, pp_context **out);

/* Frees the context and all its device memory (including cached batch
 * buffers); NULL is a no-op. Synchronises the streams of pending batches
 * first. */
void pp_destroy(pp_context *ctx);

/* Message of the last error on ctx (NULL ctx: last pp_create failure).
 * Valid until the next call on ctx. */
const char *pp_last_error(const pp_context *ctx);

/* Sets / reads launch parameters for later pp_propagate calls. PP_EINVAL
 * on a block size that is not a multiple of 64 in 64..1024. */
pp_status pp_set_launch_config(pp_context *ctx, const pp_launch_config *cfg);
pp_status pp_get_launch_config(const pp_context *ctx, pp_launch_config *cfg);

/* Number of propagation steps after which a photon stops as
 * PP_FATE_CAPPED (default 100000; 0 stops every photon at emission). Unlike
 * the launch parameters this changes results. At most 2^31. */
pp_status pp_set_step_cap(pp_context *ctx, uint64_t step_cap);

/* Loads (replaces) the layered ice model; copies it. layers has
 * header->n_layers entries, index 0 lowest. PP_EINVAL on non-finite header
 * values, dz <= 0, n_group <= 0, lengths <= 0 or NaN, g outside (-1, 1), or
 * n_layers outside 1..1024. */
pp_status pp_load_ice(pp_context *ctx, const pp_ice_header *header, const pp_ice_layer *layers);

/* Loads (replaces) the module geometry (5160 modules between 1450 m and
 * 2450 m depth in the paper's detector, Sec. 1), copies it, and builds the
 * string table and horizontal search grid used to find candidate modules.
 * n_doms 0 .. 2^24, at most 512 strings; dom_radius_m > 0. PP_EINVAL on
 * non-finite coordinates or duplicate (string_id, om_index). */
pp_status pp_load_geometry(pp_context *ctx, const pp_dom *doms, uint32_t n_doms,
                           float dom_radius_m);
pp_status pp_get_geometry_info(const pp_context *ctx, pp_geometry_info *out);

/* Host-side query of the search grid at (x, y): the string tested for every
 * photon in that cell (0xFFFFFFFF if none) and a lower bound on the
 * horizontal distance from any point of the cell to any other string's
 * reach (+inf if none). For tests of the grid's conservativeness. */
pp_status pp_geometry_cell(const pp_context *ctx, float x, float y, uint32_t *nearest_string,
                           float *clearance_m);

/* Submits a batch of n_sources light sources (a block of light-emitting
 * steps, Sec. 4); copies and validates them, uploads them to the device and
 * returns a batch handle in *batch_out. Needs ice and geometry loaded
 * (PP_ESTATE otherwise). PP_EINVAL on a bad type, non-finite values, a
 * non-unit direction, lambda_min > lambda_max or <= 0, index overflow, or
 * overlapping photon-index ranges within one event. */
pp_status pp_submit(pp_context *ctx, const pp_source *sources, uint32_t n_sources,
                    uint64_t *batch_out);

/* Releases a batch. Its device buffers go back to the context's cache for
 * later batches (blocks up to 256 MB, at most 8 GB cached; larger ones are
 * freed), after waiting for the batch's propagation and for any device
 * fetch or count it enqueued; work on other streams is not waited for. */
pp_status pp_release(pp_context *ctx, uint64_t batch);

/* Wavelength dependence of the ice (Sec. 2, photon-propagation paragraph:
 * every 10 m layer has its own scattering and absorption coefficients; the
 * paper states no law for their change with wavelength). With this set, the
 * loaded layer table holds the coefficients at lambda_ref_nm and a photon
 * of wavelength l sees a (l / lambda_ref)^-kappa_abs and
 * b (l / lambda_ref)^-kappa_scat; g is unchanged. The photon's wavelength is
 * drawn at emission (fixed, or 1/l^2 on [lambda_min, lambda_max]). NULL
 * restores wavelength-independent optics (the default). Applies to later
 * pp_propagate calls and graph captures. PP_EINVAL unless lambda_ref_nm > 0
 * and |kappa| <= 10. */
typedef struct {
  float lambda_ref_nm;  /* wavelength of the loaded coefficients */
  float kappa_abs;      /* absorption exponent */
  float kappa_scat;     /* scattering exponent */
  float reserved;
} pp_chromatic;
pp_status pp_set_chromatic(pp_context *ctx, const pp_chromatic *c);

/* Hit weight (Sec. 2: a photon that meets a module makes a photoelectron
 * with a probability that depends on its position, direction, time and
 * wavelength; the paper gives no formula). With this set, each hit's weight
 * is A(l) P(c): A linear between table[k] at lambda0_nm + k dlambda_nm
 * (held constant beyond the ends), P(c) = sum_k poly[k] c^k, and c the
 * cosine of the angle between the photon's direction and the inward surface
 * normal where it meets the module (0..1). Deterministic: no random draws.
 * NULL restores weight 1 (the default). The arrays are copied. PP_EINVAL
 * unless 1 <= n_table <= 256 with finite values >= 0, dlambda_nm > 0 when
 * n_table > 1, and 1 <= n_poly <= 8 finite coefficients. */
typedef struct {
  float lambda0_nm, dlambda_nm;
  uint32_t n_table, n_poly;
  const float *table;
  const float *poly;
} pp_acceptance;
pp_status pp_set_acceptance(pp_context *ctx, const pp_acceptance *acc);

/* Turns per-photon terminal records on or off for later pp_propagate calls
 * (48 bytes of device memory per photon). mode:
 *   PP_RECORDS_OFF: no records (the default).
 *   PP_RECORDS_ON: records, written by the kernel variant that draws each
 *     photon's wavelength (so wavelength_nm is always set).
 *   PP_RECORDS_PRODUCTION: records written by the same kernel variant that
 *     runs with records off, i.e. the arithmetic the hits come from; that
 *     variant draws no wavelength unless the optics or an acceptance need
 *     it, and then wavelength_nm is 0.
 * A photon's path, fate and hit are the same in every mode (the wavelength
 * has a random word of its own). PP_EINVAL on another mode. */
enum { PP_RECORDS_OFF = 0, PP_RECORDS_ON = 1, PP_RECORDS_PRODUCTION = 2 };
pp_status pp_set_debug_records(pp_context *ctx, int mode);

/* Propagates every photon of the batch (Sec. 2: the distance to the next
 * scatter drawn by Monte Carlo from the layer's scattering coefficient, a
 * new direction from the scattering physics, repeated until the photon
 * reaches a module or is absorbed): one persistent kernel on hip_stream (a
 * hipStream_t; NULL is the null stream), asynchronous. Ice, geometry and
 * sources are already resident on the device. May be called again on the
 * same batch; the result is the same. */
pp_status pp_propagate(pp_context *ctx, uint64_t batch, void *hip_stream);

/* Number of hits (synchronises the batch's stream). If the device hit buffer
 * overflowed, the batch is propagated again with a large enough buffer
 * first; the rerun gives the same hits. */
pp_status pp_hit_count(pp_context *ctx, uint64_t batch, uint64_t *n_total);

/* Copies up to cap hits into host memory out (order unspecified) and sets
 * *n_total: the compact records of Sec. 4 (hit-record paragraph: particle
 * id, time, weight), plus event, photon index and module. Returns
 * PP_ETRUNC if n_total > cap (cap hits copied). */
pp_status pp_fetch_hits(pp_context *ctx, uint64_t batch, pp_hit *out, uint64_t cap,
                        uint64_t *n_total);

/* Sorts n hits in host memory by (event_id, photon_index), the order in
 * which a client takes an event's hits back (Sec. 4: hits return to the
 * process that sent the event). A photon has at most one hit, so the order
 * is unique. Host only, no context needed; PP_EINVAL if hits is NULL with
 * n > 0. */
pp_status pp_sort_hits(pp_hit *hits, uint64_t n);

/* Same, into device memory dev_out (e.g. a torch tensor's data_ptr), copied
 * on hip_stream. */
pp_status pp_fetch_hits_device(pp_context *ctx, uint64_t batch, void *dev_out, uint64_t cap,
                               uint64_t *n_total, void *hip_stream);

/* Per-module hit counts: writes n_doms uint32 counts into device memory
 * dev_counts on hip_stream, from the batch's hits on the device. The work on
 * hip_stream waits for the batch's propagation, whatever stream that ran on.
 * The counts cover every hit: if the hit buffer could have overflowed
 * (fewer slots than photons), the call first checks the count as
 * pp_hit_count does (so it synchronises the batch's stream, and reruns the
 * batch on overflow), unless a propagation of this batch has already been
 * found to fit its buffer with the same ice, geometry, step cap, optics and
 * acceptance (the hits are then the same); otherwise it does not
 * synchronise. */
pp_status pp_dom_counts(pp_context *ctx, uint64_t batch, uint32_t *dev_counts, void *hip_stream);

/* Per-module sums of hit weights: writes n_doms doubles into device memory
 * dev_sums on hip_stream (same ordering and completeness as pp_dom_counts). With the
 * default unit weights they equal the counts; with a hit acceptance
 * (pp_set_acceptance) they are the detected-light expectation per module,
 * the weighted histogram of the hits (Sec. 4: a hit carries a weight). The
 * order of the additions is not fixed, so the last bits may vary between
 * calls. */
pp_status pp_dom_weights(pp_context *ctx, uint64_t batch, double *dev_sums, void *hip_stream);

/* Copies terminal records first .. first + count - 1 of the batch (photons
 * numbered in submission order: source by source, index by index) into
 * host memory out. Needs debug records on when the batch was propagated.
 * wavelength_nm is the photon's drawn wavelength, or 0 under
 * PP_RECORDS_PRODUCTION when the kernel drew none. */
pp_status pp_fetch_records(pp_context *ctx, uint64_t batch, pp_photon_record *out,
                           uint64_t first, uint64_t count);

/* Counters and kernel time of the batch's last propagation (synchronises):
 * photons, steps, layer crossings, module tests and fates, the figures
 * behind the GPU-utilisation and time-per-shower comparison of Sec. 5
 * (Table 1). */
pp_status pp_get_stats(pp_context *ctx, uint64_t batch, pp_stats *out);

/* Batched uneven events. The paper's server aggregates light-emitting steps
 * from many events and clients to keep the GPU busy, because one small
 * event at a time starves it (Sec. 3, GPU-utilisation finding; Sec. 4,
 * propagation-server paragraph). A batch may hold any number of events of
 * any size: the propagation kernel is persistent and its wavefronts steal
 * chunks of photon ids from one queue, so a 1e8-photon event and a
 * 1e3-photon event share the device without imbalance. */

/* Times the batch under a fixed set of launch configurations (workgroup
 * size 256/512/1024, chunk size 64/256/1024, refill interval 2/4/8), each one
 * full propagation on hip_stream, and keeps the fastest as the context's
 * launch configuration (also written to *best if non-NULL). Results do not
 * change; only speed does. Synchronises the stream. */
pp_status pp_autotune(pp_context *ctx, uint64_t batch, void *hip_stream, pp_launch_config *best);

/* Captures the batch's propagation (counter reset and kernel, with the
 * context's current launch configuration and debug-record setting) into a
 * HIP graph held by the batch. hip_stream must be a non-null stream; it is
 * used only for the capture. The graph is dropped when the batch's buffers
 * change (hit-buffer growth, a new chunk size) or the batch is released. */
pp_status pp_graph_capture(pp_context *ctx, uint64_t batch, void *hip_stream);

/* Launches the captured graph on hip_stream: equivalent to pp_propagate
 * with the captured configuration. PP_ESTATE if no graph is held. */
pp_status pp_graph_launch(pp_context *ctx, uint64_t batch, void *hip_stream);

/* Propagation that allocates nothing, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc. It submits, propagates and counts in one call, with
 * the same kernel and therefore the same hits as pp_submit + pp_propagate +
 * pp_fetch_hits_device on the same sources.
 *   sources, n_sources: light sources in host memory, as for pp_submit (same
 *     validation); at most PP_STATIC_MAX_SOURCES of them.
 *   dev_hits, hit_cap: caller-owned device buffer of hit_cap pp_hit records;
 *     the hits are written there, in unspecified order.
 *   n_total: receives the number of hits. PP_ETRUNC if it exceeds hit_cap:
 *     then hit_cap of the hits are written (which ones is unspecified) and
 *     the call can be repeated with a larger buffer for the same hits.
 *   stats: if non-NULL, receives the counters of the propagation and the
 *     launch used; kernel_ms is 0 (the call records no events).
 * The sources, the work queue and the counters live in a fixed 16 MiB device
 * array that the library holds on each GPU it runs on until the process
 * ends; no hipMalloc, hipFree or other allocating routine is called. The
 * call runs on hip_stream and synchronises it before returning. Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU (from
 * several threads or contexts) race and must be serialised by the caller.
 * PP_ESTATE if ice or geometry is missing or debug records are on (they need
 * per-photon memory); PP_EINVAL on bad sources, more than
 * PP_STATIC_MAX_SOURCES sources, or a photon count whose work queue cannot
 * fit the array even in chunks of 2^31 photon ids. */
#define PP_STATIC_MAX_SOURCES 32768u
pp_status pp_propagate_static(pp_context *ctx, const pp_source *sources, uint32_t n_sources, pp_hit *dev_hits,
                              uint64_t hit_cap, uint64_t *n_total, pp_stats *stats, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* PP_H_ */

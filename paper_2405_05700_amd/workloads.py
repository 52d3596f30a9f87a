"""Seeded synthetic inputs: ice tables, detector geometries and light sources.

This module only builds input arrays. It holds none of the propagation
arithmetic and is shared by the FP64 oracle's tests and by the GPU path.
Every stored value is float32 (or an integer), so both sides start from
bit-identical inputs.

The paper (Meagher & van Santen, Sec. 1 and Sec. 2) describes a detector of
5160 optical modules between 1450 m and 2450 m depth in ice made of 10 m
layers with their own scattering and absorption. The real geometry and ice
tables are not in the paper; the generators below build synthetic stand-ins
of the same shape:

* ``tiny_point_source``: one isotropic point source, 20 homogeneous layers of
  10 m (absorption length 100 m, effective scattering length 25 m, g = 0.9),
  one string of 60 modules 30 m away with 17 m vertical spacing, module 30
  level with the source.
* ``full_detector``: 86 strings x 60 modules on a 125 m triangular lattice,
  171 layers of 10 m with a smooth depth profile and a dust bump at 2000 m
  depth, 1000 Cherenkov track segments of 10 m.
* ``random_tiny``: small random geometries used to compare the grid search
  with brute force.

The record layouts below match the C structs declared in ``include/pp.h``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Layouts of the C-ABI structs (little endian, natural alignment).
ICE_LAYER_DTYPE = np.dtype(
    [("abs_len_m", "<f4"), ("eff_scat_len_m", "<f4"), ("g", "<f4")], align=True)
DOM_DTYPE = np.dtype(
    [("x", "<f4"), ("y", "<f4"), ("z", "<f4"), ("string_id", "<u4"), ("om_index", "<u4")],
    align=True)
SOURCE_DTYPE = np.dtype(
    [("type", "<u4"), ("event_id", "<u4"), ("particle_id", "<u4"), ("reserved0", "<u4"),
     ("x", "<f4"), ("y", "<f4"), ("z", "<f4"),
     ("dx", "<f4"), ("dy", "<f4"), ("dz", "<f4"),
     ("t0_ns", "<f4"), ("length_m", "<f4"), ("cherenkov_deg", "<f4"),
     ("lambda_min_nm", "<f4"), ("lambda_max_nm", "<f4"), ("reserved1", "<f4"),
     ("n_photons", "<u8"), ("first_photon_index", "<u8")], align=True)
assert ICE_LAYER_DTYPE.itemsize == 12
assert DOM_DTYPE.itemsize == 20
assert SOURCE_DTYPE.itemsize == 80

SOURCE_POINT = 0
SOURCE_CHERENKOV = 1

DOM_RADIUS_M = 0.1651
N_GROUP = 1.35


@dataclasses.dataclass
class Workload:
    """Everything one propagation run needs, in the C-ABI layouts."""
    name: str
    z_lo_m: float
    dz_m: float
    n_group: float
    layers: np.ndarray      # ICE_LAYER_DTYPE, index 0 = lowest z
    doms: np.ndarray        # DOM_DTYPE; the module id is the row index
    dom_radius_m: float
    sources: np.ndarray     # SOURCE_DTYPE
    # optional wavelength dependence of the layer coefficients:
    # (lambda_ref_nm, kappa_abs, kappa_scat), coefficients scale as
    # (lambda / lambda_ref)^-kappa; None: independent of wavelength
    chromatic: tuple | None = None
    # optional hit acceptance: {"l0": nm, "dl": nm, "table": [...],
    # "poly": [...]} (weight = table interpolated at the photon's
    # wavelength x polynomial in the cosine of incidence); None: weight 1
    acceptance: dict | None = None

    @property
    def n_photons(self) -> int:
        return int(self.sources["n_photons"].sum())

    def with_sources(self, sources: np.ndarray, name: str | None = None) -> "Workload":
        return dataclasses.replace(self, sources=sources, name=name or self.name)

    def with_radius(self, r: float) -> "Workload":
        return dataclasses.replace(self, dom_radius_m=float(np.float32(r)))


def f32(x) -> float:
    return float(np.float32(x))


def make_layers(abs_len, eff_scat_len, g) -> np.ndarray:
    abs_len = np.asarray(abs_len, dtype=np.float64)
    out = np.zeros(abs_len.shape[0], dtype=ICE_LAYER_DTYPE)
    out["abs_len_m"] = abs_len
    out["eff_scat_len_m"] = eff_scat_len
    out["g"] = g
    return out


def point_source(x=0.0, y=0.0, z=0.0, n_photons=100_000, wavelength_nm=405.0,
                 event_id=0, particle_id=0, first_photon_index=0, t0_ns=0.0) -> np.ndarray:
    s = np.zeros(1, dtype=SOURCE_DTYPE)
    s["type"] = SOURCE_POINT
    s["event_id"] = event_id
    s["particle_id"] = particle_id
    s["x"], s["y"], s["z"] = x, y, z
    s["dz"] = 1.0
    s["t0_ns"] = t0_ns
    s["lambda_min_nm"] = wavelength_nm
    s["lambda_max_nm"] = wavelength_nm
    s["n_photons"] = n_photons
    s["first_photon_index"] = first_photon_index
    return s


def tiny_point_source(n_photons: int = 100_000, dom_radius_m: float = DOM_RADIUS_M,
                      abs_len_m: float = 100.0, eff_scat_len_m: float = 25.0,
                      g: float = 0.9) -> Workload:
    """One point source of 405 nm photons at the origin; 20 layers of 10 m
    over z in [-100, 100) m (the edge layers extend beyond); one string at
    (30, 0) with module k at z = 17 (k - 30) m, k = 0..59."""
    layers = make_layers(np.full(20, abs_len_m), np.full(20, eff_scat_len_m), np.full(20, g))
    doms = np.zeros(60, dtype=DOM_DTYPE)
    doms["x"] = 30.0
    doms["y"] = 0.0
    doms["z"] = 17.0 * (np.arange(60) - 30)
    doms["string_id"] = 0
    doms["om_index"] = np.arange(60)
    return Workload("tiny_point_source", -100.0, 10.0, f32(N_GROUP), layers, doms,
                    f32(dom_radius_m), point_source(n_photons=n_photons))


def hex_string_sites(n_strings: int = 86, spacing_m: float = 125.0) -> np.ndarray:
    """The n sites of a triangular lattice {spacing (i + j/2), spacing j sqrt(3)/2}
    nearest the origin, ordered by (radius, azimuth in [0, 2 pi), i, j).
    For 86 sites this is the 91-site hexagon of five rings minus five of
    its six corners."""
    sites = []
    for i in range(-12, 13):
        for j in range(-12, 13):
            r2 = i * i + i * j + j * j           # radius^2 / spacing^2, exact
            x = i + j / 2.0
            y = j * math.sqrt(3.0) / 2.0
            az = math.atan2(y, x) % (2.0 * math.pi)
            sites.append((r2, az, i, j, x * spacing_m, y * spacing_m))
    sites.sort(key=lambda s: s[:4])
    return np.array([[s[4], s[5]] for s in sites[:n_strings]], dtype=np.float64)


def full_detector_ice():
    """171 layers of 10 m covering depths 1100-2810 m (z = 1950 m - depth),
    index 0 deepest. Smooth profile lambda_a = 120 + 40 tanh((d - 1700)/200) m,
    lambda_e = 30 + 15 tanh((d - 1700)/200) m, both divided by a dust factor
    1 + 3 exp(-(d - 2000)^2 / (2 * 25.5^2)) (a 60 m FWHM bump); g = 0.9.
    Values are taken at layer centres."""
    n = 171
    z_lo = 1950.0 - 2810.0
    centre_depth = 2810.0 - 10.0 * (np.arange(n) + 0.5)
    tanh = np.tanh((centre_depth - 1700.0) / 200.0)
    dust = 1.0 + 3.0 * np.exp(-0.5 * ((centre_depth - 2000.0) / 25.5) ** 2)
    abs_len = (120.0 + 40.0 * tanh) / dust
    eff_scat = (30.0 + 15.0 * tanh) / dust
    return z_lo, make_layers(abs_len, eff_scat, np.full(n, 0.9))


def full_detector_doms() -> np.ndarray:
    """86 strings x 60 modules; module k of a string sits at depth
    1450 + k * 1000/59 m, i.e. z = 500 - k * 1000/59 m. Module id =
    string * 60 + k."""
    sites = hex_string_sites(86)
    doms = np.zeros(86 * 60, dtype=DOM_DTYPE)
    k = np.arange(60)
    for s, (x, y) in enumerate(sites):
        rows = slice(60 * s, 60 * (s + 1))
        doms["x"][rows] = x
        doms["y"][rows] = y
        doms["z"][rows] = 1950.0 - (1450.0 + k * 1000.0 / 59.0)
        doms["string_id"][rows] = s
        doms["om_index"][rows] = k
    return doms


def cherenkov_segments(n_sources: int, photons_per_source, seed: int = 0,
                       length_m: float = 10.0, first_event_id: int = 0) -> np.ndarray:
    """Muon track segments with start points uniform in the cylinder
    r <= 500 m, |z| <= 500 m, down-going directions with cos(zenith)
    uniform in [0.2, 1] and uniform azimuth; 41 degree Cherenkov cone;
    wavelengths 300-600 nm with density proportional to 1/lambda^2.
    Draw order from numpy default_rng(seed): radius fraction, position
    azimuth, z, cos(zenith), direction azimuth, each as one vector over the
    sources. Each segment is its own event (event id = first_event_id + i)
    with particle id i and photon indices starting at 0."""
    rng = np.random.default_rng(seed)
    r = 500.0 * np.sqrt(rng.random(n_sources))
    phi = 2.0 * np.pi * rng.random(n_sources)
    z = rng.uniform(-500.0, 500.0, n_sources)
    cz = rng.uniform(0.2, 1.0, n_sources)
    az = 2.0 * np.pi * rng.random(n_sources)
    sz = np.sqrt(1.0 - cz * cz)
    d = np.stack([sz * np.cos(az), sz * np.sin(az), -cz], axis=1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    s = np.zeros(n_sources, dtype=SOURCE_DTYPE)
    s["type"] = SOURCE_CHERENKOV
    s["event_id"] = first_event_id + np.arange(n_sources)
    s["particle_id"] = np.arange(n_sources)
    s["x"], s["y"], s["z"] = r * np.cos(phi), r * np.sin(phi), z
    s["dx"], s["dy"], s["dz"] = d[:, 0], d[:, 1], d[:, 2]
    s["length_m"] = length_m
    s["cherenkov_deg"] = 41.0
    s["lambda_min_nm"] = 300.0
    s["lambda_max_nm"] = 600.0
    s["n_photons"] = photons_per_source
    s["first_photon_index"] = 0
    return s


def full_detector(n_sources: int = 1000, photons_per_source: int = 100_000,
                  seed: int = 0) -> Workload:
    z_lo, layers = full_detector_ice()
    return Workload("full_detector", f32(z_lo), 10.0, f32(N_GROUP), layers,
                    full_detector_doms(), f32(DOM_RADIUS_M),
                    cherenkov_segments(n_sources, photons_per_source, seed))


def near_module_segments(w: Workload, n_sources: int, photons_per_source, seed: int = 0,
                         r_min: float = 3.0, r_max: float = 120.0, targets=None,
                         length_m: float = 10.0, first_event_id: int = 0) -> np.ndarray:
    """Cherenkov segments (as in cherenkov_segments) whose centres lie at a
    log-uniform distance in [r_min, r_max] m from a module, in a uniform
    direction; the module is drawn uniformly from `targets` (default: all
    modules of w), cycling through them in order if targets is given.
    Segments whose centre would fall inside a module are pushed out to
    r_min. Draw order from numpy default_rng(seed): target (if not given),
    distance fraction, offset cos(theta), offset azimuth, cos(zenith),
    direction azimuth."""
    rng = np.random.default_rng(seed)
    if targets is None:
        tgt = rng.integers(0, len(w.doms), n_sources)
    else:
        tgt = np.resize(np.asarray(targets), n_sources)
    r = r_min * (r_max / r_min) ** rng.random(n_sources)
    ct = rng.uniform(-1.0, 1.0, n_sources)
    ph = 2.0 * np.pi * rng.random(n_sources)
    cz = rng.uniform(0.2, 1.0, n_sources)
    az = 2.0 * np.pi * rng.random(n_sources)
    st = np.sqrt(1.0 - ct * ct)
    off = np.stack([st * np.cos(ph), st * np.sin(ph), ct], 1) * r[:, None]
    m = np.stack([w.doms["x"], w.doms["y"], w.doms["z"]], 1).astype(np.float64)[tgt]
    centre = m + off
    sz = np.sqrt(1.0 - cz * cz)
    d = np.stack([sz * np.cos(az), sz * np.sin(az), -cz], axis=1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    start = centre - 0.5 * length_m * d
    s = np.zeros(n_sources, dtype=SOURCE_DTYPE)
    s["type"] = SOURCE_CHERENKOV
    s["event_id"] = first_event_id + np.arange(n_sources)
    s["particle_id"] = np.arange(n_sources)
    s["x"], s["y"], s["z"] = start[:, 0], start[:, 1], start[:, 2]
    s["dx"], s["dy"], s["dz"] = d[:, 0], d[:, 1], d[:, 2]
    s["length_m"] = length_m
    s["cherenkov_deg"] = 41.0
    s["lambda_min_nm"] = 300.0
    s["lambda_max_nm"] = 600.0
    s["n_photons"] = photons_per_source
    return s


def structured_modules(w: Workload, window_m: float = 30.0, rel: float = 0.2) -> np.ndarray:
    """Ids of the modules whose surroundings have strongly depth-dependent
    optics: some layer within window_m above or below the module has an
    absorption or scattering coefficient differing from the module's own
    layer by more than a factor 1 + rel. In the full-detector ice these are
    the modules in and around the dust layer."""
    L = w.layers
    a = 1.0 / L["abs_len_m"].astype(np.float64)
    b = 1.0 / (L["eff_scat_len_m"].astype(np.float64) * (1.0 - L["g"].astype(np.float64)))
    z = w.doms["z"].astype(np.float64)

    def layer(zz):
        return np.clip(np.floor((zz - w.z_lo_m) / w.dz_m), 0, len(L) - 1).astype(np.int64)

    own = layer(z)
    dev = np.zeros(len(z))
    for off in np.arange(-window_m, window_m + 1e-9, 0.5 * w.dz_m):
        li = layer(z + off)
        dev = np.maximum(dev, np.maximum(np.abs(np.log(a[li] / a[own])), np.abs(np.log(b[li] / b[own]))))
    return np.nonzero(dev > np.log1p(rel))[0]


def training_targets(w: Workload, n: int, structured_frac: float = 0.4, seed: int = 0) -> np.ndarray:
    """Target modules for n training segments: a fraction structured_frac
    drawn uniformly from structured_modules(w), the rest uniformly from all
    modules, in shuffled order (numpy default_rng(seed): all-module draws,
    structured draws, shuffle)."""
    rng = np.random.default_rng(seed)
    n_s = int(round(structured_frac * n))
    hard = structured_modules(w)
    if len(hard) == 0:
        n_s = 0
    t = np.concatenate([rng.integers(0, len(w.doms), n - n_s), rng.choice(hard, n_s) if n_s else
                        np.zeros(0, np.int64)])
    rng.shuffle(t)
    return t


def power_law_energies(n_events: int, seed: int = 0, index: float = 2.7,
                       e_min: float = 1e2, e_max: float = 1e7) -> np.ndarray:
    """Energies (GeV) from a density proportional to E^-index on
    [e_min, e_max], by inverse CDF of numpy default_rng(seed) uniforms."""
    rng = np.random.default_rng(seed)
    u = rng.random(n_events)
    a = 1.0 - index
    return (e_min ** a + u * (e_max ** a - e_min ** a)) ** (1.0 / a)


def uneven_events(n_events: int = 4096, seed: int = 0,
                  photons_per_gev: float = 10.0) -> Workload:
    """Batched uneven events: one Cherenkov segment per event in the full
    detector, carrying round(10 E) photons for E drawn from E^-2.7 on
    [1e2, 1e7] GeV (1e3 to 1e8 photons per event)."""
    e = power_law_energies(n_events, seed)
    n = np.rint(photons_per_gev * e).astype(np.uint64)
    w = full_detector(n_sources=n_events, photons_per_source=1, seed=seed + 1)
    src = w.sources.copy()
    src["n_photons"] = n
    return w.with_sources(src, "uneven_events")


def random_tiny(seed: int, n_strings: int = 3, doms_per_string: int = 5,
                radius_m: float = 1.5) -> Workload:
    """A few short, slightly tilted strings near a point source in
    homogeneous-ish layered ice; large modules so hits are common. Used to
    check that the grid search returns exactly the brute-force result."""
    rng = np.random.default_rng(seed)
    n_layers = int(rng.integers(3, 12))
    layers = make_layers(rng.uniform(20.0, 80.0, n_layers), rng.uniform(5.0, 30.0, n_layers),
                         rng.uniform(0.0, 0.95, n_layers))
    doms = np.zeros(n_strings * doms_per_string, dtype=DOM_DTYPE)
    for s in range(n_strings):
        cx, cy = rng.uniform(-25.0, 25.0, 2)
        tilt = rng.normal(0.0, 0.3, 2)
        z0 = rng.uniform(-30.0, 0.0)
        spacing = rng.uniform(4.0, 9.0)
        for k in range(doms_per_string):
            row = s * doms_per_string + k
            z = z0 + spacing * k
            doms[row] = (cx + tilt[0] * k, cy + tilt[1] * k, z, s, k)
    z_lo = float(rng.uniform(-60.0, -20.0))
    return Workload(f"random_tiny_{seed}", f32(z_lo), 10.0, f32(N_GROUP), layers, doms,
                    f32(radius_m), point_source(*rng.uniform(-5.0, 5.0, 3), n_photons=2000))

"""Surrogate + Monte Carlo: per-module expected hits of clusters of Cherenkov
segments, taken from the learned surrogate where an ensemble of networks
agrees and from Monte Carlo where it does not.

The surrogate answers for all (segment, module) pairs at once; the Monte
Carlo stays the fallback and the judge (the paper's point that the optics of
the ice make simple light models inaccurate, Sec. 1 and Sec. 2, is why the
fallback exists). Host orchestration only: every network evaluation and every
propagated photon runs in libpp's kernels; this module sums small
per-cluster arrays and decides which modules fall back.

Error measure. A Monte Carlo estimate from n hits has relative standard
error 1/sqrt(n), so 2500 hits give the 2% error; over many modules 68.3% of
such estimates fall within 2% of the truth and 95.4% within 4%. The
surrogate's answer for a module is accepted when it is at least as good in
that sense: the fallback rule is calibrated on held-out modules with a known
truth so that the accepted ones meet both fractions and none of them is off
by more than 10% (five standard errors of such an estimate).
"""
from __future__ import annotations

import dataclasses

import numpy as np

HITS_FOR_2PCT = 2500
WITHIN_2PCT, WITHIN_4PCT = 0.683, 0.954  # Gaussian one- and two-sigma coverage
MAX_ACCEPTED = 0.10                      # five standard errors of a 2% Monte Carlo estimate


def cluster_light(members, batch: int, n_sources: int, cluster_of_source: np.ndarray, n_clusters: int):
    """Expected hits L[m, c, j] of module j from the segments of cluster c,
    per network m (pp_sur_predict_pairs of every pair, summed per cluster)."""
    cos = np.asarray(cluster_of_source)
    out = None
    for mi, m in enumerate(members):
        pairs = m.predict_pairs(batch, n_sources)
        if out is None:
            out = np.zeros((len(members), n_clusters, pairs.shape[1]))
        for c in range(n_clusters):
            out[mi, c] = pairs[cos == c].sum(0, dtype=np.float64)
    return out


def ensemble_spread(L: np.ndarray):
    """Per-module ensemble mean of the total expected hits and the members'
    relative standard deviation about it."""
    tot = L.sum(1)
    mean = tot.mean(0)
    sd = tot.std(0, ddof=1) if len(tot) > 1 else np.zeros_like(mean)
    return mean, sd / np.maximum(mean, 1e-300)


def within_fractions(rel: np.ndarray):
    a = np.abs(rel)
    return float((a <= 0.02).mean()) if len(a) else 1.0, float((a <= 0.04).mean()) if len(a) else 1.0


def calibrate_threshold(spread: np.ndarray, rel: np.ndarray) -> float:
    """Largest spread threshold t such that the modules with spread < t
    reach both Monte Carlo coverages (68.3% within 2%, 95.4% within 4%) and
    none of them is off by more than MAX_ACCEPTED (five of Monte Carlo's
    standard errors). rel: their relative errors against the truth. 0 if
    none does."""
    order = np.argsort(spread, kind="stable")
    s, a = spread[order], np.abs(rel[order])
    n = np.arange(1, len(s) + 1)
    ok2 = np.cumsum(a <= 0.02) >= WITHIN_2PCT * n
    ok4 = np.cumsum(a <= 0.04) >= WITHIN_4PCT * n
    ok_max = np.maximum.accumulate(a) <= MAX_ACCEPTED
    good = np.nonzero(ok2 & ok4 & ok_max)[0]
    if len(good) == 0:
        return 0.0
    k = good[-1]  # the first k + 1 modules in spread order pass
    return float(s[k + 1]) if k + 1 < len(s) else float("inf")


@dataclasses.dataclass
class Plan:
    """Monte Carlo runs of a plan: photons per segment of each cluster that
    runs (0: not run), and the modules each cluster's run must resolve."""
    photons: np.ndarray  # per cluster
    modules: dict        # cluster -> module ids


def plan_mc(L_mean: np.ndarray, modules: np.ndarray, photons_ref: float, cap: float) -> Plan:
    """Monte Carlo sized to give HITS_FOR_2PCT hits on the dimmest of the
    given modules: each module is simulated by the cluster that lights it
    most (by the ensemble's cluster light L_mean[c, j] at photons_ref
    photons per segment), with enough photons per segment for its dimmest
    module, at most cap."""
    n_cl = L_mean.shape[0]
    photons = np.zeros(n_cl)
    per = {}
    if len(modules):
        owner = np.argmax(L_mean[:, modules], axis=0)
        for c in np.unique(owner):
            mods = modules[owner == c]
            dim = L_mean[c, mods].min()
            photons[c] = min(cap, np.ceil(HITS_FOR_2PCT * photons_ref / max(dim, 1e-300)))
            per[int(c)] = mods
    return Plan(photons, per)


def plan_sources(segments: np.ndarray, cluster_of_source: np.ndarray, plan: Plan, first_index: int):
    """The segments of every cluster that runs, with the plan's photon
    count and photon indices from first_index on (independent of any run
    that used indices below it)."""
    run = plan.photons[cluster_of_source] > 0
    src = segments[run].copy()
    src["n_photons"] = plan.photons[cluster_of_source[run]].astype(np.uint64)
    src["first_photon_index"] = np.uint64(first_index)
    return src


def merge(L_mean: np.ndarray, counts: np.ndarray, plan: Plan, photons_ref: float, modules: np.ndarray):
    """Per-module expectation at photons_ref photons per segment for the
    given modules: every cluster that ran contributes its Monte Carlo count
    scaled to photons_ref, every other cluster the ensemble's expectation."""
    ran = plan.photons > 0
    scale = np.where(ran, photons_ref / np.maximum(plan.photons, 1), 0.0)
    mc = (counts[:, modules] * scale[:, None]).sum(0)
    sur = L_mean[~ran][:, modules].sum(0)
    return mc + sur


def evaluate(ctx, det, members, n_sets: int = 4, truth_photons: int = 400_000_000, cut_m: float = 300.0,
             graded_per_1e8: float = 1e4, clusters: int = 40, per_cluster: int = 4, log=None) -> dict:
    """Surrogate+MC and plain Monte Carlo, both executed, on held-out
    clusters; returns times, photon counts and accuracies.

    Set q (q = 0 .. n_sets - 1) draws `clusters` target modules of det from
    numpy default_rng(404 + 101 q) and per_cluster segments 4-20 m from each
    (workloads.near_module_segments, seed 202 + 1000 q); segment i of a set
    belongs to the cluster of target i % clusters. Truth: truth_photons per
    segment; graded modules have at least graded_per_1e8 truth hits per 1e8
    photons per segment. Set 0 calibrates the fallback threshold
    (calibrate_threshold); sets 1.. are graded. Per graded set:
    * surrogate+MC: the ensemble's per-cluster light for every module; the
      graded modules whose spread reaches the threshold fall back to Monte
      Carlo of the cluster that lights them most (plan_mc); merged per module;
    * plain MC: every cluster simulated for its dimmest graded module.
    The two Monte Carlo legs run as one batch each (timed with HIP events),
    with photon indices above the truth's, independent of it. The truth
    only grades; nothing in either leg reads it."""
    import time

    import torch

    from . import workloads as W

    say = log or (lambda msg: None)
    T = int(truth_photons)
    for m in members:
        m.set_inference_cut(cut_m)
    s = torch.cuda.current_stream()
    n_src = clusters * per_cluster
    sets, truth_photons_all, truth_ms = [], 0, 0.0
    for q in range(n_sets):
        targets = np.random.default_rng(404 + 101 * q).choice(len(det.doms), clusters, replace=False)
        seg = W.near_module_segments(det, n_src, T, seed=202 + 1000 * q, r_min=4.0, r_max=20.0,
                                     targets=targets, first_event_id=n_src * q)
        b = ctx.submit(seg)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        ctx.propagate(b, s)
        e1.record(s)
        truth = ctx.dom_counts(b, stream=s).cpu().numpy().astype(np.float64)
        torch.cuda.synchronize()
        truth_ms += e0.elapsed_time(e1)
        truth_photons_all += int(seg["n_photons"].sum())
        graded = np.nonzero(truth >= graded_per_1e8 * T / 1e8)[0]
        sets.append({"seg": seg, "batch": b, "truth": truth, "graded": graded,
                     "cluster": np.arange(n_src) % clusters})
        say(f"surrogate+MC: truth of set {q} ({len(graded)} graded modules)")
    mc_rate = truth_photons_all / (truth_ms / 1e3)

    cluster_light(members, sets[0]["batch"], n_src, sets[0]["cluster"], clusters)  # warm-up
    torch.cuda.synchronize()
    t_sur = 0.0
    for k, S in enumerate(sets):
        t0 = time.perf_counter()
        L = cluster_light(members, S["batch"], n_src, S["cluster"], clusters)
        mean, spread = ensemble_spread(L)
        dt = time.perf_counter() - t0
        if k > 0:
            t_sur += dt
        S.update({"L": L.mean(0), "mean": mean, "spread": spread})
    cal = sets[0]
    g = cal["graded"]
    tau = calibrate_threshold(cal["spread"][g], cal["mean"][g] / cal["truth"][g] - 1.0)

    legs = {}
    for leg in ("fallback", "plain"):
        srcs, owner = [], {}
        for k, S in enumerate(sets[1:], start=1):
            g = S["graded"]
            mods = g[S["spread"][g] >= tau] if leg == "fallback" else g
            S[leg + "_plan"] = plan_mc(S["L"], mods, T, cap=T)
            srcs.append(plan_sources(S["seg"], S["cluster"], S[leg + "_plan"], first_index=T))
            for e, c in zip(S["seg"]["event_id"], S["cluster"]):
                owner[int(e)] = (k, int(c))
        src = np.concatenate(srcs)
        ms, hits = 0.0, None
        if len(src):
            b = ctx.submit(src)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            ctx.propagate(b, s)
            e1.record(s)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            hits = ctx.fetch_hits(b)
            ctx.release(b)
        for k, S in enumerate(sets[1:], start=1):
            counts = np.zeros((clusters, len(det.doms)))
            if hits is not None and len(hits):
                kc = np.array([owner[int(e)] for e in hits["event_id"]], np.int64).reshape(-1, 2)
                mine = kc[:, 0] == k
                np.add.at(counts, (kc[mine, 1], hits["dom_id"][mine].astype(np.int64)), 1.0)
            S[leg + "_est"] = merge(S["L"], counts, S[leg + "_plan"], T, S["graded"])
        legs[leg] = {"photons": int(src["n_photons"].sum()) if len(src) else 0, "kernel_s": ms / 1e3}
        say(f"surrogate+MC: {leg} Monte Carlo, {legs[leg]['photons']:.3e} photons in {ms / 1e3:.3f} s")

    def errors(est_of):
        rel = np.concatenate([est_of(S) / S["truth"][S["graded"]] - 1.0 for S in sets[1:]])
        w2, w4 = within_fractions(rel)
        return {"within_2pct": w2, "within_4pct": w4,
                "p68_abs_rel_error": float(np.quantile(np.abs(rel), 0.683)) if len(rel) else 0.0,
                "median_abs_rel_error": float(np.median(np.abs(rel))) if len(rel) else 0.0,
                "max_abs_rel_error": float(np.abs(rel).max()) if len(rel) else 0.0}

    graded_all = sum(len(S["graded"]) for S in sets[1:])
    n_fb = sum(int((S["spread"][S["graded"]] >= tau).sum()) for S in sets[1:])
    t_plain, t_hyb = legs["plain"]["kernel_s"], t_sur + legs["fallback"]["kernel_s"]
    # fallback for exactly the modules the truth puts outside 2% (no real run can choose so)
    t_upper = t_sur
    for S in sets[1:]:
        g = S["graded"]
        bad = g[np.abs(S["mean"][g] / S["truth"][g] - 1.0) > 0.02]
        t_upper += plan_mc(S["L"], bad, T, cap=T).photons.sum() * per_cluster / mc_rate
    return {"eval_sets": n_sets, "calibration_sets": 1, "clusters_graded": clusters * (n_sets - 1),
            "segments_per_cluster": per_cluster, "truth_photons_per_source": T, "infer_cut_m": cut_m,
            "graded_modules": graded_all, "mc_photons_per_s": mc_rate,
            "fallback_spread_threshold": tau, "fallback_modules": n_fb,
            "fallback_frac": n_fb / max(graded_all, 1),
            "clusters_with_mc": sum(int((S["fallback_plan"].photons > 0).sum()) for S in sets[1:]),
            "t_surrogate_s": t_sur, "t_fallback_mc_s": legs["fallback"]["kernel_s"], "t_plain_mc_s": t_plain,
            "fallback_mc_photons": legs["fallback"]["photons"], "plain_mc_photons": legs["plain"]["photons"],
            "speedup_at_2pct": t_plain / t_hyb if t_hyb > 0 else None,
            "accuracy": {"surrogate_plus_mc": errors(lambda S: S["fallback_est"]),
                         "plain_mc": errors(lambda S: S["plain_est"]),
                         "surrogate_alone": errors(lambda S: S["mean"][S["graded"]])},
            "speedup_truth_selected_fallback": t_plain / t_upper if t_upper > 0 else None}

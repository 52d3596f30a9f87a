"""The learned surrogate on the GPU against its FP64 oracle.

Features, labels, forward outputs and gradients of the BF16/FP32-accumulate
network are compared with oracle/mlp_oracle.py fed the same bf16-rounded
features and weights, so the only differences are the kernel's own
roundings: each stored activation and each backward operand is rounded to
bf16 (relative error at most u = 2^-9 ~ 1.95e-3) and every sum is FP32.

Tolerances, from u:
* forward: the predicted mean is exp of the output, and the output's error
  is a sum of many independent roundings of both signs, so the typical
  (median) relative error of the mean stays below one unit u: FWD_MEDIAN =
  2e-3. The tail, where one output's inputs cancel, gets ten units: FWD_P99
  = 2e-2.
* loss: a sum of 4096 per-row terms whose rounding errors mostly cancel:
  LOSS_REL = 5e-3 (2.5 u).
* gradients: each element of a gradient tensor sums products of two
  rounded operands (2 u each) over the rows; with no cancellation that is
  at most 2 u relative, and the cancellation between rows of opposite sign
  measured on these sets stays below a factor 5, so the relative Frobenius
  error per tensor is held to GRAD_REL = 2e-2 (10 u) and its cosine to the
  oracle's gradient to GRAD_COS = 0.9995 (an angle below 1.8 degrees).
A 3% error in one tensor, or a missing term, fails these.
"""
import sys

import numpy as np
import pytest

from paper_2405_05700_amd import workloads as W

pytestmark = pytest.mark.gpu

FWD_MEDIAN, FWD_P99 = 2e-3, 2e-2
LOSS_REL = 5e-3
GRAD_REL, GRAD_COS = 2e-2, 0.9995


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available()
    from paper_2405_05700_amd import pp, surrogate
    from oracle import mlp_oracle
    return pp, surrogate, mlp_oracle


def bf16_round(x):
    x = np.ascontiguousarray(x, np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def propagated(pp, w, seed=0):
    ctx = pp.Context(0, seed=seed)
    ctx.load_workload(w)
    b = ctx.submit(w.sources)
    ctx.propagate(b)
    return ctx, b


def flatten(M, params):
    return np.concatenate([np.concatenate([W_.ravel(), b]) for W_, b in params]).astype(np.float32)


def unflatten(M, theta):
    out, o = [], 0
    for n_out, n_in in M.LAYER_SHAPES:
        W_ = theta[o:o + n_out * n_in].reshape(n_out, n_in).astype(np.float64)
        o += n_out * n_in
        b = theta[o:o + n_out].astype(np.float64)
        o += n_out
        out.append([W_, b])
    return out


@pytest.fixture(scope="module")
def small_set(mods):
    pp, surrogate, M = mods
    w = W.full_detector(n_sources=4, photons_per_source=200_000, seed=11)
    ctx, b = propagated(pp, w)
    sur = surrogate.Surrogate(ctx, seed=1)
    sur.set_training_set(b)
    return w, ctx, b, sur


def test_features_and_labels(mods, small_set):
    pp, surrogate, M = mods
    w, ctx, b, sur = small_set
    n_dom = len(w.doms)
    P = sur.training_size()
    assert P == 4 * n_dom
    rows = sur.training_rows(0, P)
    assert rows["features"].shape[1] == M.IN_REAL
    src = np.repeat(np.arange(4), n_dom)
    dom = np.tile(np.arange(n_dom), 4)
    X, mub, R = M.pair_features(w, src, dom)
    diff = np.abs(rows["features"] - X[:, :M.IN_REAL])
    ok = (diff <= 0.008 * np.abs(X[:, :M.IN_REAL]) + 2e-3).all(1)
    say("feature rows within bf16 tolerance", ok.mean())
    assert ok.mean() >= 0.999
    assert np.allclose(rows["mu_base"], mub, rtol=2e-3, atol=1e-30)
    # labels against the fetched hits (event id = source index here)
    hits = ctx.fetch_hits(b)
    pair = hits["event_id"].astype(np.int64) * n_dom + hits["dom_id"]
    k = np.bincount(pair, minlength=P)
    assert (rows["k"] == k).all() and (rows["n_t"] == k).all()
    s = w.sources[hits["event_id"]]
    d = np.stack([s["dx"], s["dy"], s["dz"]], 1).astype(float)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    c = np.stack([s["x"], s["y"], s["z"]], 1) + 0.5 * s["length_m"][:, None] * d
    m = w.doms[hits["dom_id"]]
    Rh = np.linalg.norm(np.stack([m["x"], m["y"], m["z"]], 1) - c, axis=1)
    tpm = float(np.float32(W.N_GROUP)) / 0.299792458
    delay = np.maximum(hits["time_ns"] - s["t0_ns"] - np.maximum(Rh - 5.0 - w.dom_radius_m, 0) * tpm, 0) + 0.01
    s1 = np.bincount(pair, weights=delay, minlength=P)
    s2 = np.bincount(pair, weights=np.log(delay), minlength=P)
    assert np.allclose(rows["s1"], s1, rtol=1e-4, atol=1e-2)
    assert np.allclose(rows["s2"], s2, rtol=1e-4, atol=1e-2)
    say("labels: hits", len(hits), "pairs with hits", int((k > 0).sum()))


def oracle_on_gpu_inputs(M, rows, theta, first, count):
    X = np.zeros((count, M.IN_PAD))
    X[:, :M.IN_REAL] = rows["features"][first:first + count]
    params = unflatten(M, theta)
    for p in params:
        p[0] = bf16_round(p[0])
    return X, params


def test_forward_and_gradients_match_oracle(mods, small_set):
    pp, surrogate, M = mods
    w, ctx, b, sur = small_set
    params0 = M.init_params(7)
    for _, bias in params0:
        bias[:] = np.random.default_rng(2).normal(0, 0.05, bias.shape)
    params0[-1][1][M.OUT_REAL:] = 0
    theta = flatten(M, params0)
    sur.set_params(theta)
    assert np.array_equal(sur.get_params(), theta)
    P = sur.training_size()
    rows = sur.training_rows(0, P)
    # inference path (features -> 5 GEMMs -> expected hits per pair)
    mu_gpu = sur.predict_pairs(b, 4).ravel()
    X, params = oracle_on_gpu_inputs(M, rows, theta, 0, P)
    Y, _ = M.forward(params, X)
    nph = np.repeat(w.sources["n_photons"].astype(float), len(w.doms))
    mu_ref = nph * rows["mu_base"] * np.exp(Y[:, 0])
    rel = np.abs(mu_gpu - mu_ref) / mu_ref
    say("forward: median rel", np.median(rel), "p99", np.quantile(rel, 0.99))
    assert np.median(rel) < FWD_MEDIAN and np.quantile(rel, 0.99) < FWD_P99
    # loss and gradients over 4096 rows
    first, count = 0, 4096
    loss, grad = sur.loss_grad(first, count)
    X, params = oracle_on_gpu_inputs(M, rows, theta, first, count)
    Y, cache = M.forward(params, X)
    sl = slice(first, first + count)
    loss_ref, dY = M.loss_and_grad_out(Y, rows["mu_base"][sl].astype(float), nph[sl], rows["k"][sl],
                                       rows["n_t"][sl], rows["s1"][sl], rows["s2"][sl])
    g_ref = flatten(M, M.backward(params, cache, dY)).astype(np.float64)
    say("loss gpu", loss, "oracle", loss_ref)
    assert abs(loss - loss_ref) <= LOSS_REL * abs(loss_ref) + 1e-6
    o = 0
    for li, (n_out, n_in) in enumerate(M.LAYER_SHAPES):
        for part, size in (("W", n_out * n_in), ("b", n_out)):
            a, r = grad[o:o + size].astype(np.float64), g_ref[o:o + size]
            o += size
            err = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-30)
            cos = a @ r / max(np.linalg.norm(a) * np.linalg.norm(r), 1e-30)
            say(f"grad layer {li} {part}: rel {err:.4f} cos {cos:.6f}")
            assert err < GRAD_REL and cos > GRAD_COS, (li, part, err, cos)


def test_gradients_on_ragged_unaligned_minibatches(mods, small_set):
    """Minibatches that start inside a 32-row block and end in a ragged tail
    give the oracle's loss and gradients too: 1001 rows from row 5037 (padded
    to 1024: 32 row blocks, 16 weight-gradient slices of two steps each), 37
    rows from row 19990 (one 64-row tile: two row blocks, the second all
    padding past row 32), a single row (one row block, one slice), the
    set's last three rows, and the benchmarked minibatch of 8192 rows (256
    row blocks, 16 slices of 16 steps: four full rounds of the load
    ring)."""
    pp, surrogate, M = mods
    w, ctx, b, sur = small_set
    theta = flatten(M, M.init_params(3))
    sur.set_params(theta)
    P = sur.training_size()
    rows = sur.training_rows(0, P)
    nph = np.repeat(w.sources["n_photons"].astype(float), len(w.doms))
    for first, count in ((5037, 1001), (19990, 37), (0, 1), (P - 3, 3), (100, 8192)):
        loss, grad = sur.loss_grad(first, count)
        X, params = oracle_on_gpu_inputs(M, rows, theta, first, count)
        Y, cache = M.forward(params, X)
        sl = slice(first, first + count)
        loss_ref, dY = M.loss_and_grad_out(Y, rows["mu_base"][sl].astype(float), nph[sl], rows["k"][sl],
                                           rows["n_t"][sl], rows["s1"][sl], rows["s2"][sl])
        g_ref = flatten(M, M.backward(params, cache, dY)).astype(np.float64)
        say(f"rows [{first}, {first + count}): loss gpu {loss} oracle {loss_ref}")
        assert abs(loss - loss_ref) <= LOSS_REL * abs(loss_ref) + 1e-6
        o = 0
        for li, (n_out, n_in) in enumerate(M.LAYER_SHAPES):
            for part, size in (("W", n_out * n_in), ("b", n_out)):
                a, r = grad[o:o + size].astype(np.float64), g_ref[o:o + size]
                o += size
                err = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-30)
                cos = a @ r / max(np.linalg.norm(a) * np.linalg.norm(r), 1e-30)
                assert err < GRAD_REL and cos > GRAD_COS, (first, count, li, part, err, cos)


def test_fused_expected_hits_equal_pair_sums(mods):
    """The fused inference kernel adds every pair's expectation to its
    module's sum: 37 sources x 5160 modules is 746 full tiles of 256 pairs
    and a ragged last one."""
    pp, surrogate, M = mods
    import torch
    w = W.full_detector(n_sources=37, photons_per_source=1000, seed=31)
    ctx = pp.Context(0, seed=0)
    ctx.load_workload(w)
    b = ctx.submit(w.sources)
    sur = surrogate.Surrogate(ctx, seed=6)
    per_pair = sur.predict_pairs(b, len(w.sources)).astype(np.float64)
    sums = sur.expected_hits(b).cpu().numpy()
    torch.cuda.synchronize()
    assert (37 * len(w.doms)) % 256 != 0
    ref = per_pair.sum(0)
    say("fused sums vs pair sums: max rel", np.max(np.abs(sums - ref) / np.maximum(ref, 1e-300)))
    assert np.allclose(sums, ref, rtol=1e-6, atol=1e-300)
    assert np.isfinite(per_pair).all() and (per_pair >= 0).all()


def test_training_calls_refuse_bad_row_ranges(mods, small_set):
    """Row ranges outside the training set, empty minibatches, batch sizes
    that are zero or not a multiple of 64 and invalid learning rates are
    refused with an error, and a refused call leaves the parameters as they
    were."""
    pp, surrogate, M = mods
    w, ctx, b, sur = small_set
    theta = flatten(M, M.init_params(4))
    sur.set_params(theta)
    P = sur.training_size()
    for first, count in ((0, 0), (P - 2, 5), (P, 1)):
        with pytest.raises(pp.PPError):
            sur.loss_grad(first, count)
        with pytest.raises(pp.PPError):
            sur.train_step(first, count, 1e-3)
    for kw in (dict(batch_size=0), dict(batch_size=100), dict(lr=-1e-3), dict(lr=float("nan"))):
        with pytest.raises(pp.PPError):
            sur.train(epochs=1, **kw)
    assert np.array_equal(sur.get_params(), theta)


def test_inference_at_full_size_on_sampled_pairs(mods):
    """The benchmarked inference workload, 1e5 full-detector segments x 5160
    modules (5.16e8 pairs, 4 031 250 workgroups in one launch, as the bench
    times it): the per-module sums equal the sums of the per-pair
    expectations, and 2048 sampled pairs (the first and the last among them)
    match the oracle's network on the oracle's own features within the
    forward bounds."""
    pp, surrogate, M = mods
    import torch
    w = W.full_detector(n_sources=100_000, photons_per_source=1, seed=303)
    ctx = pp.Context(0, seed=0)
    ctx.load_workload(w)
    b = ctx.submit(w.sources)
    sur = surrogate.Surrogate(ctx, seed=1)
    params0 = M.init_params(7)
    for _, bias in params0:
        bias[:] = np.random.default_rng(2).normal(0, 0.05, bias.shape)
    params0[-1][1][M.OUT_REAL:] = 0
    theta = flatten(M, params0)
    sur.set_params(theta)
    sums = sur.expected_hits(b).cpu().numpy()
    torch.cuda.synchronize()
    n_dom = len(w.doms)
    per_pair = sur.predict_pairs(b, len(w.sources))
    assert per_pair.shape == (100_000, n_dom) and np.isfinite(per_pair).all() and (per_pair >= 0).all()
    ref = per_pair.sum(0, dtype=np.float64)
    say("full size: fused sums vs pair sums, max rel", np.max(np.abs(sums - ref) / np.maximum(ref, 1e-300)))
    assert np.allclose(sums, ref, rtol=1e-6, atol=1e-300)
    n_pairs = per_pair.size
    idx = np.concatenate([[0, n_pairs - 1], np.random.default_rng(5).choice(n_pairs, 2046, replace=False)])
    src, dom = idx // n_dom, idx % n_dom
    X, mub, _ = M.pair_features(w, src, dom)
    params = unflatten(M, theta)
    for q in params:
        q[0] = bf16_round(q[0])
    Y, _ = M.forward(params, bf16_round(X))
    nph = w.sources["n_photons"][src].astype(float)
    mu_ref = nph * mub * np.exp(Y[:, 0])
    mu_gpu = per_pair.ravel()[idx].astype(np.float64)
    # expectations far below float32's normal range are compared as near 0
    big = mu_ref > 1e-30
    assert big.mean() > 0.9 and (mu_gpu[~big] <= 1e-29).all()
    rel = np.abs(mu_gpu[big] - mu_ref[big]) / mu_ref[big]
    say("full size, sampled pairs:", int(big.sum()), "median rel", np.median(rel), "p99", np.quantile(rel, 0.99),
        "max", rel.max())
    assert np.median(rel) < FWD_MEDIAN and np.quantile(rel, 0.99) < FWD_P99
    del per_pair
    sur.close()
    ctx.close()


def test_far_pair_sampling_follows_rule_and_oracle(mods):
    """Training-pair sampling on the device: the kept rows are exactly the
    pairs the rule keeps (module within 150 m of the segment centre, or
    (module + source) % 16 == 0), in source-major order, with weights 1 and
    16; their features and labels equal those of the same pairs in the full
    set; and the weighted loss and gradients match the oracle."""
    pp, surrogate, M = mods
    det = W.full_detector(n_sources=1, photons_per_source=1)
    ev = W.near_module_segments(det, 6, 300_000, seed=9, r_min=3.0, r_max=25.0)
    wl = det.with_sources(ev)
    ctx = pp.Context(0, seed=0)
    ctx.load_workload(det)
    b = ctx.submit(ev)
    ctx.propagate(b)
    n_dom = len(det.doms)
    full = surrogate.Surrogate(ctx, seed=1)
    full.set_training_set(b)
    P_all = full.training_size()
    assert P_all == 6 * n_dom
    pair_all, w_all = full.training_pairs(0, P_all)
    assert np.array_equal(pair_all, np.arange(P_all)) and (w_all == 1).all()
    rows_all = full.training_rows(0, P_all)
    full.close()
    sur = surrogate.Surrogate(ctx, seed=1)
    sur.set_sampling(150.0, 16)
    sur.set_training_set(b)
    P = sur.training_size()
    pair, wt = sur.training_pairs(0, P)
    pair = pair.astype(np.int64)
    src, dom = np.divmod(np.arange(P_all), n_dom)
    _, _, R = M.pair_features(wl, src, dom)
    keep_ref, w_ref = M.far_sample(R, src, dom, 150.0, 16)
    kept = np.zeros(P_all, bool)
    kept[pair] = True
    clear = np.abs(R - 150.0) > 1e-3  # pairs on the boundary may round either way
    say("sampled rows", P, "of", P_all, "near", int((wt == 1).sum()))
    assert (np.diff(pair) > 0).all()
    assert np.array_equal(kept[clear], keep_ref[clear])
    w_full = np.zeros(P_all)
    w_full[keep_ref] = w_ref
    assert np.array_equal(wt[clear[pair]], w_full[pair][clear[pair]].astype(np.float32))
    assert P < P_all / 8
    rows = sur.training_rows(0, P)
    assert np.array_equal(rows["features"], rows_all["features"][pair])
    assert np.array_equal(rows["mu_base"], rows_all["mu_base"][pair])
    assert np.array_equal(rows["k"], rows_all["k"][pair]) and np.array_equal(rows["n_t"], rows_all["n_t"][pair])
    assert np.allclose(rows["s1"], rows_all["s1"][pair], rtol=1e-5, atol=1e-3)
    assert np.allclose(rows["s2"], rows_all["s2"][pair], rtol=1e-5, atol=1e-3)
    # every hit on a near pair is a label
    near = R <= 150.0 - 1e-3
    assert rows["k"][wt == 1].sum() >= rows_all["k"][near].sum() > 0
    # weighted loss and gradients against the oracle
    params0 = M.init_params(8)
    theta = flatten(M, params0)
    sur.set_params(theta)
    count = min(P, 2048)
    loss, grad = sur.loss_grad(0, count)
    X, params = oracle_on_gpu_inputs(M, rows, theta, 0, count)
    Y, cache = M.forward(params, X)
    nph = ev["n_photons"][pair[:count] // n_dom].astype(float)
    loss_ref, dY = M.loss_and_grad_out(Y, rows["mu_base"][:count].astype(float), nph, rows["k"][:count],
                                       rows["n_t"][:count], rows["s1"][:count], rows["s2"][:count],
                                       weight=wt[:count].astype(float))
    g_ref = flatten(M, M.backward(params, cache, dY)).astype(np.float64)
    say("weighted loss gpu", loss, "oracle", loss_ref)
    assert abs(loss - loss_ref) <= LOSS_REL * abs(loss_ref) + 1e-6
    o = 0
    for li, (n_out, n_in) in enumerate(M.LAYER_SHAPES):
        for part, size in (("W", n_out * n_in), ("b", n_out)):
            a, r = grad[o:o + size].astype(np.float64), g_ref[o:o + size]
            o += size
            err = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-30)
            cos = a @ r / max(np.linalg.norm(a) * np.linalg.norm(r), 1e-30)
            say(f"weighted grad layer {li} {part}: rel {err:.4f} cos {cos:.6f}")
            assert err < GRAD_REL and cos > GRAD_COS, (li, part, err, cos)
    # a shuffled epoch with lr = 0 visits every weighted row once
    l_all, _ = sur.loss_grad(0, P)
    losses = sur.train(epochs=2, batch_size=512, lr=0.0)
    assert np.allclose(losses, l_all, rtol=2e-5, atol=1e-9)
    sur.close()


def test_sampling_edge_cases(mods, small_set):
    """near_m = inf keeps every pair with weight 1 (any stride); near_m = 0
    keeps exactly the strided pairs, each of weight stride; invalid
    arguments are refused and leave the setting unchanged."""
    pp, surrogate, M = mods
    w, ctx, b, sur0 = small_set
    n_dom = len(w.doms)
    sur = surrogate.Surrogate(ctx, seed=2)
    sur.set_sampling(float("inf"), 16)
    sur.set_training_set(b)
    P = sur.training_size()
    pair, wt = sur.training_pairs(0, P)
    assert P == 4 * n_dom and np.array_equal(pair, np.arange(P)) and (wt == 1).all()
    sur.set_sampling(0.0, 7)
    sur.set_training_set(b)
    P = sur.training_size()
    pair, wt = sur.training_pairs(0, P)
    src, dom = np.divmod(pair.astype(np.int64), n_dom)
    expect = np.nonzero((np.tile(np.arange(n_dom), 4) + np.repeat(np.arange(4), n_dom)) % 7 == 0)[0]
    assert np.array_equal(pair.astype(np.int64), expect) and (wt == 7).all()
    for bad in [(-1.0, 4), (float("nan"), 4), (10.0, 0)]:
        with pytest.raises(pp.PPError):
            sur.set_sampling(*bad)
    sur.set_training_set(b)
    assert sur.training_size() == P  # the valid setting still applies
    sur.close()


def test_inference_cut(mods):
    """With a 300 m cut, pairs farther apart expect exactly 0 hits, pairs
    inside are bit-identical to the uncut evaluation (whole tiles beyond
    the cut are skipped, the rest compute as before), and the module sums
    are the sums of the pairs; invalid cuts are refused."""
    pp, surrogate, M = mods
    import torch
    w = W.full_detector(n_sources=37, photons_per_source=1000, seed=31)
    ctx = pp.Context(0, seed=0)
    ctx.load_workload(w)
    b = ctx.submit(w.sources)
    sur = surrogate.Surrogate(ctx, seed=6)
    full = sur.predict_pairs(b, len(w.sources))
    sur.set_inference_cut(300.0)
    cut = sur.predict_pairs(b, len(w.sources))
    sums = sur.expected_hits(b).cpu().numpy()
    torch.cuda.synchronize()
    n_dom = len(w.doms)
    src, dom = np.divmod(np.arange(len(w.sources) * n_dom), n_dom)
    _, _, R = M.pair_features(w, src, dom)
    R = R.reshape(len(w.sources), n_dom)
    inside, outside = R < 300.0 - 1e-3, R > 300.0 + 1e-3
    say("cut: pairs inside", int(inside.sum()), "outside", int(outside.sum()))
    assert inside.sum() > 1000 and outside.sum() > 10 * inside.sum()
    assert (cut[outside] == 0).all() and np.array_equal(cut[inside], full[inside])
    assert (full[outside] > 0).any()
    assert np.allclose(sums, cut.astype(np.float64).sum(0), rtol=1e-6, atol=1e-300)
    for bad in (0.0, -5.0, float("nan")):
        with pytest.raises(pp.PPError):
            sur.set_inference_cut(bad)
    sur.set_inference_cut(float("inf"))
    assert np.array_equal(sur.predict_pairs(b, len(w.sources)), full)
    sur.close()


def test_adam_step_matches_definition(mods, small_set):
    pp, surrogate, M = mods
    w, ctx, b, sur = small_set
    theta0 = flatten(M, M.init_params(5))
    sur.set_params(theta0)
    _, g = sur.loss_grad(0, 2048)
    sur.set_params(theta0)  # clears Adam state
    sur.train_step(0, 2048, 1e-3)
    theta1 = sur.get_params().astype(np.float64)
    g = g.astype(np.float64)
    expect = theta0 - 1e-3 * g / (np.abs(g) + 1e-8)
    big = np.abs(g) > 1e-6
    assert np.allclose(theta1[big], expect[big], rtol=1e-5, atol=1e-7)
    assert np.allclose(theta1[~big], expect[~big], atol=1.1e-3)


def test_shuffled_epoch_visits_every_row_once(mods, small_set):
    """With lr = 0 the parameters stay put, so the mean loss of a shuffled
    epoch must equal the loss of the whole set in stored order: every row is
    visited exactly once, whatever the permutation."""
    pp, surrogate, M = mods
    w, ctx, b, sur = small_set
    theta = flatten(M, M.init_params(9))
    sur.set_params(theta)
    P = sur.training_size()
    full, _ = sur.loss_grad(0, P)
    losses = sur.train(epochs=3, batch_size=1024, lr=0.0)
    say("full-set loss", full, "shuffled epochs", losses)
    assert np.array_equal(sur.get_params(), theta)
    assert np.allclose(losses, full, rtol=2e-5, atol=1e-9)


def test_training_beats_the_untrained_baseline(mods):
    """Train on Monte Carlo of 64 segments placed near modules; on 32
    held-out segments the trained network's likelihood and per-module
    expected hits beat the network's starting point (the diffusion baseline,
    output 0)."""
    pp, surrogate, M = mods
    import torch
    det = W.full_detector(n_sources=1, photons_per_source=1)
    w_tr = det.with_sources(W.near_module_segments(det, 64, 400_000, seed=21))
    ctx, b_tr = propagated(pp, w_tr)
    sur = surrogate.Surrogate(ctx, seed=3)
    init = sur.get_params()
    zero = np.zeros_like(init)  # all-zero network: output 0, i.e. the baseline itself
    sur.set_training_set(b_tr)
    n_tr = sur.training_size() // 64 * 64
    sur.set_params(zero)
    l_tr0, _ = sur.loss_grad(0, n_tr)
    sur.set_params(init)
    losses = sur.train(epochs=12, batch_size=4096, lr=2e-3, lr_final=2e-5)
    say("epoch losses", losses)
    l_tr1, _ = sur.loss_grad(0, n_tr)
    say("training-set loss before", l_tr0, "after", l_tr1)
    assert l_tr1 < l_tr0
    trained = sur.get_params()
    w_te = det.with_sources(W.near_module_segments(det, 32, 4_000_000, seed=22))
    b_te = ctx.submit(w_te.sources)
    ctx.propagate(b_te)
    sur.set_training_set(b_te)
    n = sur.training_size() // 64 * 64
    l_trained, _ = sur.loss_grad(0, n)
    sur.set_params(zero)
    l_base, _ = sur.loss_grad(0, n)
    say("held-out loss trained", l_trained, "baseline", l_base)
    assert l_trained < l_base
    # per-module expected hits vs the Monte Carlo counts of the held-out set
    counts = ctx.dom_counts(b_te).cpu().numpy().astype(float)
    exp_base = sur.expected_hits(b_te).cpu().numpy()
    sur.set_params(trained)
    exp_tr = sur.expected_hits(b_te).cpu().numpy()
    torch.cuda.synchronize()
    bright = counts >= 40
    e_tr = np.abs(exp_tr[bright] - counts[bright]) / counts[bright]
    e_base = np.abs(exp_base[bright] - counts[bright]) / counts[bright]
    say("modules", int(bright.sum()), "median rel error trained", np.median(e_tr), "baseline", np.median(e_base))
    assert bright.sum() >= 5 and np.median(e_tr) < np.median(e_base)


def test_labels_training_and_sums_are_bit_reproducible(mods):
    """The same recipe gives the same network, bit for bit: labels built
    from two propagations whose hits arrive in different orders (different
    launch shapes) are identical, two training runs from the same start on
    them end in identical parameters and epoch losses, and so in identical
    per-pair predictions. Every sum on the way is formed in a fixed order or
    in exact fixed point."""
    pp, surrogate, M = mods
    det = W.full_detector(n_sources=1, photons_per_source=1)
    w = det.with_sources(W.near_module_segments(det, 24, 300_000, seed=5))
    runs = []
    for launch in ({}, {"block_size": 256, "chunk_size": 64, "refill_interval": 2}):
        ctx = pp.Context(0, seed=0)
        ctx.load_workload(w)
        ctx.set_launch_config(**launch)
        b = ctx.submit(w.sources)
        ctx.propagate(b)
        sur = surrogate.Surrogate(ctx, seed=3)
        sur.set_training_set(b)
        runs.append((ctx, b, sur))
    (ctx1, b1, s1), (ctx2, b2, s2) = runs
    P = s1.training_size()
    assert P == s2.training_size() == len(w.sources) * len(w.doms)
    r1, r2 = s1.training_rows(0, P), s2.training_rows(0, P)
    assert r1["k"].sum() > 500
    for key in r1:
        assert np.array_equal(r1[key].view(np.uint32), r2[key].view(np.uint32)), key
    l1 = s1.train(epochs=2, batch_size=4096, lr=1e-3)
    l2 = s2.train(epochs=2, batch_size=4096, lr=1e-3)
    say("epoch losses", l1, l2)
    assert np.array_equal(l1.view(np.uint32), l2.view(np.uint32))
    p1, p2 = s1.get_params(), s2.get_params()
    assert np.array_equal(p1.view(np.uint32), p2.view(np.uint32))
    # per-pair predictions of the two networks are identical; the per-module
    # sums add pairs with atomics, so only their last bits may differ
    assert np.array_equal(s1.predict_pairs(b1, len(w.sources)), s2.predict_pairs(b2, len(w.sources)))
    e1 = s1.expected_hits(b1).cpu().numpy()
    e3 = s2.expected_hits(b2).cpu().numpy()
    assert np.allclose(e1, e3, rtol=1e-12, atol=0)
    for ctx, b, sur in runs:
        sur.close()
        ctx.close()

"""FP64 CPU oracle of the learned surrogate (test infrastructure only).

The surrogate predicts, for a light source and an optical module, the
expected number of hits per emitted photon and gamma parameters of the hit
delay. It is a multilayer perceptron: five affine layers (29 features + 35 zero columns)
-> 256 -> 256 -> 256 -> 256 -> 64, three outputs used) with GELU between
them (GELU(z) = z Phi(z), Phi the standard normal CDF). Everything here is
the plain definition, in float64:

* features: geometry of the (source, module) pair up to a rotation about
  the vertical (the ice is layered in depth only) and the optical
  properties of the layers holding the source centre and the module, and
  of the layers 20 m above and below each;
* baseline: the diffusion estimate of the hit probability,
  mu_base = r^2 exp(-R/delta) / (4 D R), D = lambda_e/3,
  delta = sqrt(D lambda_a), with lambda_e and lambda_a averaged over the two
  layers; the network predicts log(mu / mu_base);
* loss per pair: Poisson negative log-likelihood of the hit count,
  mu_tot - k log mu_tot with mu_tot = N mu, plus the gamma negative
  log-likelihood of the hit delays from their sufficient statistics
  (n, sum delta, sum log delta): n (lgamma(kappa) + kappa log theta)
  - (kappa - 1) sum log delta + sum delta / theta, kappa = exp(y1),
  theta = tau0 exp(y2);
* gradients by the chain rule written out layer by layer;
* Adam (Kingma & Ba, 2015) with bias correction.

Only the test suite imports it. Nothing in the product path does.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

C_LIGHT = 0.299792458
IN_REAL, IN_PAD, HIDDEN, OUT_PAD, OUT_REAL = 29, 64, 256, 64, 3
TAN_CHERENKOV = math.tan(math.radians(41.0))
NEIGHBOUR_DZ_M = 20.0  # depth offset of the neighbouring optics features
LAYER_SHAPES = [(HIDDEN, IN_PAD), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN),
                (OUT_PAD, HIDDEN)]  # (out, in): weight matrices are out x in
TAU0_NS = 50.0
TIME_WEIGHT = 0.1


def gelu(z):
    return 0.5 * z * (1.0 + special.erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + special.erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


# ---------------------------------------------------------------- features --

def layer_index(z, z_lo, dz, n_layers):
    f = np.floor((np.asarray(z, np.float64) - z_lo) / dz)
    return np.clip(np.nan_to_num(f, nan=0.0), 0, n_layers - 1).astype(np.int64)


def pair_features(w, src_idx, dom_idx):
    """Features (P x 64, columns IN_REAL.. zero), baseline mu_base (P) per
    photon and centre distance R (P) for (source, module) pairs of workload w
    (Cherenkov sources)."""
    s = w.sources[np.asarray(src_idx)]
    d = w.doms[np.asarray(dom_idx)]
    L = w.layers
    a_all = 1.0 / L["abs_len_m"].astype(np.float64)
    g_all = L["g"].astype(np.float64)
    le_all = L["eff_scat_len_m"].astype(np.float64)
    dirv = np.stack([s["dx"], s["dy"], s["dz"]], 1).astype(np.float64)
    dirv /= np.linalg.norm(dirv, axis=1, keepdims=True)
    half = 0.5 * s["length_m"].astype(np.float64)
    c = np.stack([s["x"], s["y"], s["z"]], 1).astype(np.float64) + half[:, None] * dirv
    m = np.stack([d["x"], d["y"], d["z"]], 1).astype(np.float64)
    delta = m - c
    R = np.maximum(np.linalg.norm(delta, axis=1), 0.5)
    u = delta / R[:, None]
    cos_eta = (u * dirv).sum(1)
    n_layers = len(L)
    ls = layer_index(c[:, 2], w.z_lo_m, w.dz_m, n_layers)
    ld = layer_index(m[:, 2], w.z_lo_m, w.dz_m, n_layers)
    a_s, a_d = a_all[ls], a_all[ld]
    b_s = 1.0 / (le_all[ls] * (1.0 - g_all[ls]))
    b_d = 1.0 / (le_all[ld] * (1.0 - g_all[ld]))
    # Geometry up to a rotation about the vertical (the ice is layered in
    # depth only): vertical parts of the two unit vectors, horizontal and
    # vertical offsets, distance, the angle to the track and the relative
    # azimuth of the two horizontal projections.
    rho = np.hypot(delta[:, 0], delta[:, 1])
    h = dirv[:, 0] * u[:, 0] + dirv[:, 1] * u[:, 1]        # horizontal part of cos(eta)
    hh = np.sqrt((dirv[:, 0] ** 2 + dirv[:, 1] ** 2) * (u[:, 0] ** 2 + u[:, 1] ** 2))
    X = np.zeros((len(R), IN_PAD))
    X[:, 0] = u[:, 2]
    X[:, 1] = rho / 100.0
    X[:, 2] = delta[:, 2] / 100.0
    X[:, 3] = R / 100.0
    X[:, 4] = np.log(R / 10.0) / 3.0
    X[:, 5] = cos_eta
    X[:, 6] = cos_eta - math.cos(math.radians(41.0))
    X[:, 7] = dirv[:, 2]
    X[:, 8] = h
    X[:, 9] = np.where(hh > 1e-9, np.clip(h / np.maximum(hh, 1e-9), -1.0, 1.0), 0.0)  # cos(relative azimuth)
    X[:, 10] = c[:, 2] / 500.0
    X[:, 11] = m[:, 2] / 500.0
    X[:, 12] = 100.0 * a_s
    X[:, 13] = 10.0 * b_s
    X[:, 14] = 100.0 * a_d
    X[:, 15] = 10.0 * b_d
    # The segment's extent: impact parameter of the track line, along-track
    # offset of the closest approach from the centre, where on the segment
    # (in lengths, capped to [-1, 2]) direct Cherenkov light at 41 degrees
    # would leave for the module, and the distances to both ends.
    L = np.maximum(s["length_m"].astype(np.float64), 1e-3)
    p0 = np.stack([s["x"], s["y"], s["z"]], 1).astype(np.float64)
    v = m - p0
    along = (v * dirv).sum(1)
    b = np.linalg.norm(v - along[:, None] * dirv, axis=1)
    X[:, 16] = b / 100.0
    X[:, 17] = (along - 0.5 * L) / 100.0
    X[:, 18] = np.clip((along - b / TAN_CHERENKOV) / L, -1.0, 2.0)
    X[:, 19] = np.linalg.norm(v, axis=1) / 100.0
    X[:, 20] = np.linalg.norm(v - L[:, None] * dirv, axis=1) / 100.0
    # the optics NEIGHBOUR_DZ_M above and below the segment centre and the
    # module: where the depth profile changes within the range light
    # diffuses over (a dust layer), the two end layers alone do not say so
    for q, z in enumerate((c[:, 2] + NEIGHBOUR_DZ_M, c[:, 2] - NEIGHBOUR_DZ_M,
                           m[:, 2] + NEIGHBOUR_DZ_M, m[:, 2] - NEIGHBOUR_DZ_M)):
        li = layer_index(z, w.z_lo_m, w.dz_m, n_layers)
        X[:, 21 + 2 * q] = 100.0 * a_all[li]
        X[:, 22 + 2 * q] = 10.0 / (le_all[li] * (1.0 - g_all[li]))
    # diffusion baseline with the two layers' mean lengths
    lam_a = 0.5 * (1.0 / a_s + 1.0 / a_d)
    lam_e = 0.5 * (le_all[ls] + le_all[ld])
    D = lam_e / 3.0
    dl = np.sqrt(D * lam_a)
    r = float(w.dom_radius_m)
    mu_base = r * r * np.exp(-R / dl) / (4.0 * D * R)
    return X, mu_base, R


# ------------------------------------------------------------------- model --

def init_params(seed: int):
    """He-uniform init for each (out x in) weight; zero biases; the padded
    input columns and padded outputs are zero."""
    rng = np.random.default_rng(seed)
    params = []
    for li, (n_out, n_in) in enumerate(LAYER_SHAPES):
        fan_in = IN_REAL if li == 0 else n_in
        lim = math.sqrt(6.0 / fan_in)
        W = rng.uniform(-lim, lim, (n_out, n_in))
        if li == 0:
            W[:, IN_REAL:] = 0.0
        if li == len(LAYER_SHAPES) - 1:
            W *= 0.1
            W[OUT_REAL:, :] = 0.0
        params.append([W, np.zeros(n_out)])
    return params


def forward(params, X):
    """Returns the outputs Y (P x 64) and the cache of pre-activations and
    activations needed by backward."""
    acts = [X]
    pre = []
    h = X
    for li, (W, b) in enumerate(params):
        z = h @ W.T + b
        if li < len(params) - 1:
            pre.append(z)
            h = gelu(z)
            acts.append(h)
        else:
            h = z
    return h, (pre, acts)


def loss_and_grad_out(Y, mu_base, n_photons, k, n_t, s1, s2, weight=None):
    """Mean over rows of weight x (Poisson + 0.1 gamma NLL), and dLoss/dY.
    A row of integer weight w counts as w copies of its pair (weight None:
    every row 1)."""
    P = Y.shape[0]
    w = np.ones(P) if weight is None else np.asarray(weight, np.float64)
    mu = n_photons * mu_base * np.exp(Y[:, 0])
    kappa = np.exp(Y[:, 1])
    theta = TAU0_NS * np.exp(Y[:, 2])
    poisson = mu - k * np.log(mu)
    gam = n_t * (special.gammaln(kappa) + kappa * np.log(theta)) - (kappa - 1.0) * s2 + s1 / theta
    loss = (w * (poisson + TIME_WEIGHT * gam)).sum() / P
    dY = np.zeros_like(Y)
    dY[:, 0] = w * (mu - k) / P
    dY[:, 1] = w * TIME_WEIGHT * kappa * (n_t * (special.digamma(kappa) + np.log(theta)) - s2) / P
    dY[:, 2] = w * TIME_WEIGHT * (n_t * kappa - s1 / theta) / P
    return loss, dY


def far_sample(R, src_idx, dom_idx, near_m, far_stride):
    """Training-pair selection (a sampling rule of this implementation, not
    of the paper): keep a pair whose module centre lies within near_m of the
    segment centre (weight 1), else keep it if (module + source) mod
    far_stride == 0 (weight far_stride). Returns (keep mask, weights)."""
    near = np.asarray(R) <= near_m
    far_keep = (np.asarray(dom_idx) + np.asarray(src_idx)) % far_stride == 0
    keep = near | far_keep
    return keep, np.where(near, 1.0, float(far_stride))[keep]


def backward(params, cache, dY):
    """Gradients [(dW, db)] of the loss given dLoss/dY."""
    pre, acts = cache
    grads = [None] * len(params)
    g = dY
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        h_in = acts[li]
        grads[li] = (g.T @ h_in, g.sum(0))
        if li > 0:
            g = (g @ W) * gelu_grad(pre[li - 1])
    return grads


class Adam:
    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
        self.v = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for li in range(len(params)):
            for j in range(2):
                g = grads[li][j]
                self.m[li][j] = self.b1 * self.m[li][j] + (1 - self.b1) * g
                self.v[li][j] = self.b2 * self.v[li][j] + (1 - self.b2) * g * g
                mh = self.m[li][j] / c1
                vh = self.v[li][j] / c2
                params[li][j] = params[li][j] - self.lr * mh / (np.sqrt(vh) + self.eps)
        return params


def expected_hits_per_photon(params, X, mu_base):
    Y, _ = forward(params, X)
    return mu_base * np.exp(Y[:, 0])

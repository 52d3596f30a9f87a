"""Python binding of the surrogate C ABI (include/pp_surrogate.h):
argument marshalling only. Training, inference and the label and feature
computations run in libpp's kernels."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import pp

_vp, _u64, _u32 = C.c_void_p, C.c_uint64, C.c_uint32
_fp = C.POINTER(C.c_float)
SIGNATURES = {
    "pp_sur_create": (C.c_int, [_vp, _u64, C.POINTER(_vp)]),
    "pp_sur_destroy": (None, [_vp]),
    "pp_sur_param_count": (_u64, []),
    "pp_sur_get_params": (C.c_int, [_vp, _vp, _u64]),
    "pp_sur_set_params": (C.c_int, [_vp, _vp, _u64]),
    "pp_sur_set_sampling": (C.c_int, [_vp, C.c_float, _u32]),
    "pp_sur_set_inference_cut": (C.c_int, [_vp, C.c_float]),
    "pp_sur_set_training_set": (C.c_int, [_vp, _u64]),
    "pp_sur_get_training_pairs": (C.c_int, [_vp, _u64, _u64, _vp, _vp]),
    "pp_sur_training_size": (C.c_int, [_vp, C.POINTER(_u64)]),
    "pp_sur_get_training_rows": (C.c_int, [_vp, _u64, _u64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pp_sur_loss_grad": (C.c_int, [_vp, _u64, _u64, C.POINTER(C.c_double), _vp]),
    "pp_sur_train_step": (C.c_int, [_vp, _u64, _u64, C.c_float, C.POINTER(C.c_double)]),
    "pp_sur_feature_count": (C.c_uint32, []),
    "pp_sur_train": (C.c_int, [_vp, _u32, _u32, C.c_float, C.c_float, _vp, _vp]),
    "pp_sur_expected_hits": (C.c_int, [_vp, _u64, _vp, _vp]),
    "pp_sur_predict_pairs": (C.c_int, [_vp, _u64, _vp, _u64]),
}
for _name, (_res, _args) in SIGNATURES.items():
    _fn = getattr(pp._lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
_lib = pp._lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class Surrogate:
    """The learned surrogate bound to a context (its device, ice and
    geometry)."""

    _close_order = 1

    def __init__(self, ctx: "pp.Context", seed: int = 0):
        h = C.c_void_p()
        st = _lib.pp_sur_create(ctx._h, int(seed), C.byref(h))
        ctx._check(st)
        self._h = h
        self.ctx = ctx
        ctx._add_dependent(self)

    def close(self):
        if self._h:
            _lib.pp_sur_destroy(self._h)
            self._h = None
            self.ctx._release_dependent()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        self.ctx._check(st)

    @staticmethod
    def param_count() -> int:
        return int(_lib.pp_sur_param_count())

    def get_params(self) -> np.ndarray:
        out = np.empty(self.param_count(), np.float32)
        self._check(_lib.pp_sur_get_params(self._h, _p(out), out.size))
        return out

    def set_params(self, theta: np.ndarray):
        theta = np.ascontiguousarray(theta, np.float32)
        self._check(_lib.pp_sur_set_params(self._h, _p(theta), theta.size))

    def set_sampling(self, near_m: float = float("inf"), far_stride: int = 1):
        """Pairs kept by the next set_training_set: all (far_stride 1), or
        those within near_m plus a weighted 1-in-far_stride sample of the
        rest."""
        self._check(_lib.pp_sur_set_sampling(self._h, near_m, far_stride))

    def set_inference_cut(self, cut_m: float = float("inf")):
        """Pairs farther apart than cut_m expect 0 hits; tiles of pairs all
        beyond it skip the network."""
        self._check(_lib.pp_sur_set_inference_cut(self._h, cut_m))

    def set_training_set(self, batch: int):
        self._check(_lib.pp_sur_set_training_set(self._h, batch))

    def training_pairs(self, first: int, count: int):
        """(pair index, loss weight) of training rows [first, first + count)."""
        pair = np.empty(count, np.uint64)
        w = np.empty(count, np.float32)
        self._check(_lib.pp_sur_get_training_pairs(self._h, first, count, _p(pair), _p(w)))
        return pair, w

    def training_size(self) -> int:
        n = C.c_uint64()
        self._check(_lib.pp_sur_training_size(self._h, C.byref(n)))
        return n.value

    def training_rows(self, first: int, count: int) -> dict:
        out = {"features": np.empty((count, _lib.pp_sur_feature_count()), np.float32)}
        for k in ("mu_base", "k", "n_t", "s1", "s2"):
            out[k] = np.empty(count, np.float32)
        self._check(_lib.pp_sur_get_training_rows(
            self._h, first, count, _p(out["features"]), _p(out["mu_base"]), _p(out["k"]),
            _p(out["n_t"]), _p(out["s1"]), _p(out["s2"])))
        return out

    def loss_grad(self, first: int, count: int):
        loss = C.c_double()
        grad = np.empty(self.param_count(), np.float32)
        self._check(_lib.pp_sur_loss_grad(self._h, first, count, C.byref(loss), _p(grad)))
        return loss.value, grad

    def train_step(self, first: int, count: int, lr: float) -> float:
        loss = C.c_double()
        self._check(_lib.pp_sur_train_step(self._h, first, count, lr, C.byref(loss)))
        return loss.value

    def train(self, epochs: int, batch_size: int = 8192, lr: float = 1e-3, lr_final: float | None = None,
              stream=None) -> np.ndarray:
        """Shuffled minibatch Adam; the learning rate decays along a cosine
        from lr to lr_final (default: constant lr)."""
        losses = np.zeros(epochs, np.float32)
        self._check(_lib.pp_sur_train(self._h, epochs, batch_size, lr, lr if lr_final is None else lr_final,
                                      pp._stream_handle(stream), _p(losses)))
        return losses

    def expected_hits(self, batch: int, out=None, stream=None):
        """Per-module expected hits summed over the batch's sources (float64
        CUDA tensor)."""
        import torch
        if out is None:
            out = torch.empty(max(self.ctx.n_doms, 1), dtype=torch.float64,
                              device=f"cuda:{self.ctx.device}")
        self._check(_lib.pp_sur_expected_hits(self._h, batch, C.c_void_p(out.data_ptr()),
                                              pp._stream_handle(stream)))
        return out[: self.ctx.n_doms]

    def predict_pairs(self, batch: int, n_sources: int) -> np.ndarray:
        out = np.empty((n_sources, self.ctx.n_doms), np.float32)
        self._check(_lib.pp_sur_predict_pairs(self._h, batch, _p(out), out.size))
        return out

"""Python binding of liblmosem.so (include/lmosem.h): argument marshalling only.

Every function mirrors the C entry point of the same name; all computation
runs in the library's HIP kernels.  Device arrays are torch tensors on the
GPU (torch supplies memory and streams only).  There is no fallback: if the
library is not built, importing this module raises ImportError.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblmosem.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc for gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

ABI_VERSION = 2
OK, EINVAL, ERANGE, ENOMEM, EDEVICE, ESTATE, ENOTSUP = 0, -1, -2, -3, -4, -5, -6
_NAMES = {0: "OK", -1: "EINVAL", -2: "ERANGE", -3: "ENOMEM", -4: "EDEVICE", -5: "ESTATE",
          -6: "ENOTSUP"}


class LmosemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class lmosem_config(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("pixel_cm", ctypes.c_double), ("n_bins", ctypes.c_int32),
                ("bin_cm", ctypes.c_double), ("n_angles", ctypes.c_int32),
                ("angle0_rad", ctypes.c_double), ("e0_kev", ctypes.c_double),
                ("fwhm_e_kev", ctypes.c_double), ("fwhm_u_cm", ctypes.c_double),
                ("win_lo_kev", ctypes.c_double), ("win_hi_kev", ctypes.c_double),
                ("n_subsets", ctypes.c_int32), ("scatter_model", ctypes.c_int32),
                ("acq_time", ctypes.c_double)]


class lmosem_events(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("angle", ctypes.c_void_p), ("u_bin", ctypes.c_void_p),
                ("energy_kev", ctypes.c_void_p)]


class lmosem_batch(ctypes.Structure):
    _fields_ = [("n_real", ctypes.c_int32), ("offsets", ctypes.POINTER(ctypes.c_int64))]


class lmosem_stats(ctypes.Structure):
    _fields_ = [("n_support", ctypes.c_int64), ("skipped_events", ctypes.c_int64),
                ("inner_terms", ctypes.c_int64), ("useful_terms", ctypes.c_int64),
                ("table_ms", ctypes.c_double), ("table_bytes", ctypes.c_int64),
                ("event_tile", ctypes.c_int32), ("n_emission", ctypes.c_int32),
                ("forward_launches", ctypes.c_int64), ("forward_ms", ctypes.c_double),
                ("backproject_launches", ctypes.c_int64), ("backproject_ms", ctypes.c_double),
                ("update_launches", ctypes.c_int64), ("update_ms", ctypes.c_double),
                ("network_launches", ctypes.c_int64), ("network_ms", ctypes.c_double),
                ("network_pairs", ctypes.c_int64)]


_P = ctypes.c_void_p
_S = ctypes.c_int
_sigs = {
    "lmosem_abi_version": (ctypes.c_uint32, []),
    "lmosem_create": (_S, [ctypes.POINTER(lmosem_config), _P, _P, ctypes.POINTER(_P)]),
    "lmosem_create_emission": (_S, [ctypes.POINTER(lmosem_config), _P, _P, _P, ctypes.POINTER(_P)]),
    "lmosem_destroy": (None, [_P]),
    "lmosem_last_error": (ctypes.c_char_p, [_P]),
    "lmosem_sensitivity": (_S, [_P, ctypes.c_int32, _P]),
    "lmosem_forward": (_S, [_P, ctypes.POINTER(lmosem_events), _P, _P]),
    "lmosem_forward_noalloc": (_S, [_P, ctypes.POINTER(lmosem_events), _P, _P]),
    "lmosem_backproject": (_S, [_P, ctypes.POINTER(lmosem_events), _P, _P]),
    "lmosem_subset_update": (_S, [_P, ctypes.c_int32, ctypes.POINTER(lmosem_events), _P, _P]),
    "lmosem_reconstruct": (_S, [_P, ctypes.POINTER(lmosem_events), ctypes.POINTER(lmosem_batch),
                                ctypes.c_int32, _P, _P, ctypes.POINTER(ctypes.c_double)]),
    "lmosem_events_load": (_S, [_P, ctypes.POINTER(lmosem_events), ctypes.POINTER(lmosem_batch),
                                ctypes.POINTER(_P)]),
    "lmosem_events_free": (None, [_P]),
    "lmosem_iterate": (_S, [_P, _P, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_double)]),
    "lmosem_set_tuning": (_S, [_P, ctypes.c_int32]),
    "lmosem_set_pixel_tile": (_S, [_P, ctypes.c_int32]),
    "lmosem_get_stats": (_S, [_P, ctypes.POINTER(lmosem_stats)]),
    "lmosem_set_timing": (_S, [_P, ctypes.c_int32]),
    "lmosem_autotune": (_S, [_P, _P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                            ctypes.POINTER(ctypes.c_int32)]),
    "lmosem_set_graphs": (_S, [_P, ctypes.c_int32]),
    "lmosem_evset_plan": (_S, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "lmosem_set_memory_cap": (_S, [_P, ctypes.c_int64]),
    "lmosem_memory_held": (_S, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "lmosem_inject_failure": (_S, [_P]),
    "lmosem_cache_rows": (_S, [_P, _P, ctypes.c_int32]),
    "lmosem_bin_events": (_S, [_P, ctypes.POINTER(lmosem_events), ctypes.c_int32, _P, ctypes.c_int32, _P]),
    "lmosem_emission_mask": (_S, [_P, _P, ctypes.c_double, ctypes.c_int32, _P]),
    "lmosem_binned_rows": (_S, [_P, ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_int64, _P, _P]),
    "lmosem_binned_reconstruct": (_S, [_P, ctypes.c_int32, _P, ctypes.c_int32, _P, ctypes.c_int32, _P, _P]),
    "lmosem_net_create": (_S, [_P, _P, ctypes.POINTER(_P)]),
    "lmosem_net_destroy": (None, [_P]),
    "lmosem_net_get_params": (_S, [_P, _P]),
    "lmosem_net_forward": (_S, [_P, _P, ctypes.c_int64, _P]),
    "lmosem_net_gradient": (_S, [_P, _P, _P, ctypes.c_int32, _P]),
    "lmosem_net_forward_train": (_S, [_P, _P, ctypes.c_int32, _P]),
    "lmosem_net_train": (_S, [_P, _P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                              ctypes.c_float, ctypes.POINTER(ctypes.c_double)]),
    "lmosem_surrogate_samples": (_S, [_P, _P, _P, _P, _P, ctypes.c_int64, _P, _P, _P]),
    "lmosem_set_surrogate": (_S, [_P, _P]),
    "lmosem_measure_alu_rates": (_S, [_P, ctypes.POINTER(ctypes.c_double)]),
}
for _name, (_res, _args) in _sigs.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_sigs)


def _dev_ptr(t: torch.Tensor | None, dtype, what: str):
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"{what} must be a contiguous {dtype} tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _events(ev: dict) -> lmosem_events:
    a, u, e = ev["angle"], ev["u_bin"], ev["energy"]
    n = int(a.numel())
    if u.numel() != n or e.numel() != n:
        raise ValueError("event arrays differ in length")
    return lmosem_events(n, _dev_ptr(a, torch.int32, "angle"), _dev_ptr(u, torch.float32, "u_bin"),
                         _dev_ptr(e, torch.float32, "energy"))


def _batch(offsets):
    if offsets is None:
        return None, None
    arr = (ctypes.c_int64 * len(offsets))(*[int(x) for x in offsets])
    return lmosem_batch(len(offsets) - 1, arr), arr


def config(geom: dict) -> lmosem_config:
    return lmosem_config(ABI_VERSION, int(geom["nx"]), int(geom["ny"]), float(geom["pixel_cm"]),
                         int(geom["n_bins"]), float(geom["bin_cm"]), int(geom["n_angles"]),
                         float(geom.get("angle0_rad", 0.0)), float(geom["e0_kev"]),
                         float(geom["fwhm_e_kev"]), float(geom["fwhm_u_cm"]),
                         float(geom["win_lo_kev"]), float(geom["win_hi_kev"]),
                         int(geom["n_subsets"]), int(geom.get("scatter_model", 1)),
                         float(geom.get("acq_time", 1.0)))


def lmosem_abi_version() -> int:
    return int(_lib.lmosem_abi_version())


def _check(ctx, status: int):
    if status != OK:
        msg = _lib.lmosem_last_error(ctx).decode() if ctx else ""
        raise LmosemError(status, msg)


def lmosem_create(geom: dict, mu: torch.Tensor, stream: torch.cuda.Stream | None = None):
    """Context for one attenuation map; mu is [ny][nx] float32 on the GPU."""
    cfg = config(geom)
    st = (stream or torch.cuda.current_stream(mu.device)).cuda_stream
    out = ctypes.c_void_p()
    s = _lib.lmosem_create(ctypes.byref(cfg), _dev_ptr(mu, torch.float32, "mu"), ctypes.c_void_p(st),
                           ctypes.byref(out))
    if s != OK:
        raise LmosemError(s, "lmosem_create rejected the configuration or the map")
    return out


def lmosem_create_emission(geom: dict, mu: torch.Tensor, emission: torch.Tensor | None,
                           stream: torch.cuda.Stream | None = None):
    """Context whose estimated image is restricted to {mu > 0, emission > 0};
    emission is [ny][nx] float32 on the GPU, or None for the mu > 0 support."""
    cfg = config(geom)
    st = (stream or torch.cuda.current_stream(mu.device)).cuda_stream
    if emission is not None and emission.numel() != mu.numel():
        raise ValueError("emission and mu differ in size")
    em = _dev_ptr(emission, torch.float32, "emission")
    out = ctypes.c_void_p()
    s = _lib.lmosem_create_emission(ctypes.byref(cfg), _dev_ptr(mu, torch.float32, "mu"), em,
                                    ctypes.c_void_p(st), ctypes.byref(out))
    if s != OK:
        raise LmosemError(s, "lmosem_create_emission rejected the configuration, the map or the emission set")
    return out


def lmosem_destroy(ctx):
    _lib.lmosem_destroy(ctx)


def lmosem_last_error(ctx) -> str:
    return _lib.lmosem_last_error(ctx).decode()


def lmosem_sensitivity(ctx, subset: int, out: torch.Tensor):
    _check(ctx, _lib.lmosem_sensitivity(ctx, int(subset), _dev_ptr(out, torch.float32, "sens")))


def lmosem_forward(ctx, events: dict, image: torch.Tensor, mean_out: torch.Tensor):
    ev = _events(events)
    _check(ctx, _lib.lmosem_forward(ctx, ctypes.byref(ev), _dev_ptr(image, torch.float32, "image"),
                                    _dev_ptr(mean_out, torch.float32, "mean")))


def lmosem_forward_noalloc(ctx, events: dict, image: torch.Tensor, mean_out: torch.Tensor):
    ev = _events(events)
    _check(ctx, _lib.lmosem_forward_noalloc(ctx, ctypes.byref(ev), _dev_ptr(image, torch.float32, "image"),
                                            _dev_ptr(mean_out, torch.float32, "mean")))


def lmosem_backproject(ctx, events: dict, weights: torch.Tensor, image_out: torch.Tensor):
    ev = _events(events)
    _check(ctx, _lib.lmosem_backproject(ctx, ctypes.byref(ev),
                                        _dev_ptr(weights, torch.float32, "weights"),
                                        _dev_ptr(image_out, torch.float32, "image")))


def lmosem_subset_update(ctx, subset: int, events: dict, image: torch.Tensor,
                         mean_out: torch.Tensor | None = None):
    ev = _events(events)
    _check(ctx, _lib.lmosem_subset_update(ctx, int(subset), ctypes.byref(ev),
                                          _dev_ptr(image, torch.float32, "image"),
                                          _dev_ptr(mean_out, torch.float32, "mean")))


def lmosem_reconstruct(ctx, events: dict, n_iters: int, images_out: torch.Tensor,
                       init: torch.Tensor | None = None, batch_offsets=None, want_loglik=False):
    ev = _events(events)
    b, _keep = _batch(batch_offsets)
    n_real = 1 if batch_offsets is None else len(batch_offsets) - 1
    ll = (ctypes.c_double * (n_real * max(n_iters, 1)))() if want_loglik else None
    _check(ctx, _lib.lmosem_reconstruct(ctx, ctypes.byref(ev), ctypes.byref(b) if b else None,
                                        int(n_iters), _dev_ptr(init, torch.float32, "init"),
                                        _dev_ptr(images_out, torch.float32, "images"), ll))
    if want_loglik:
        return np.ctypeslib.as_array(ll).reshape(n_real, max(n_iters, 1))[:, :n_iters].copy()
    return None


def lmosem_events_load(ctx, events: dict, batch_offsets=None):
    ev = _events(events)
    b, _keep = _batch(batch_offsets)
    out = ctypes.c_void_p()
    _check(ctx, _lib.lmosem_events_load(ctx, ctypes.byref(ev), ctypes.byref(b) if b else None,
                                        ctypes.byref(out)))
    return out


def lmosem_events_free(evset):
    _lib.lmosem_events_free(evset)


def lmosem_iterate(ctx, evset, n_iters: int, images: torch.Tensor, n_real: int = 1,
                   want_loglik=False):
    ll = (ctypes.c_double * (n_real * max(n_iters, 1)))() if want_loglik else None
    _check(ctx, _lib.lmosem_iterate(ctx, evset, int(n_iters),
                                    _dev_ptr(images, torch.float32, "images"), ll))
    if want_loglik:
        return np.ctypeslib.as_array(ll).reshape(n_real, max(n_iters, 1))[:, :n_iters].copy()
    return None


def lmosem_set_tuning(ctx, event_tile: int):
    _check(ctx, _lib.lmosem_set_tuning(ctx, int(event_tile)))


def lmosem_set_pixel_tile(ctx, pixels: int):
    _check(ctx, _lib.lmosem_set_pixel_tile(ctx, int(pixels)))


def lmosem_get_stats(ctx) -> dict:
    s = lmosem_stats()
    _check(ctx, _lib.lmosem_get_stats(ctx, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in lmosem_stats._fields_}


def lmosem_set_timing(ctx, enable: bool):
    _check(ctx, _lib.lmosem_set_timing(ctx, 1 if enable else 0))


def lmosem_autotune(ctx, evset) -> tuple:
    """Returns (events per tile, rows per backprojection chunk, graphs 0/1)."""
    ev = ctypes.c_int32()
    ch = ctypes.c_int32()
    gr = ctypes.c_int32()
    _check(ctx, _lib.lmosem_autotune(ctx, evset, ctypes.byref(ev), ctypes.byref(ch), ctypes.byref(gr)))
    return ev.value, ch.value, gr.value


def lmosem_evset_plan(evset) -> dict:
    """The set's plan: events per tile, pixel tile in waves of 64, chunk rows, graphs."""
    out = (ctypes.c_int32 * 4)()
    _check_plain(_lib.lmosem_evset_plan(evset, out), "lmosem_evset_plan")
    return {"event_tile": out[0], "pixel_waves": out[1], "chunk_rows": out[2], "graphs": out[3]}


def lmosem_set_graphs(ctx, enable: bool):
    _check(ctx, _lib.lmosem_set_graphs(ctx, 1 if enable else 0))


def lmosem_set_memory_cap(ctx, nbytes: int):
    _check(ctx, _lib.lmosem_set_memory_cap(ctx, int(nbytes)))


def lmosem_memory_held(ctx) -> int:
    out = ctypes.c_int64()
    _check(ctx, _lib.lmosem_memory_held(ctx, ctypes.byref(out)))
    return out.value


def lmosem_inject_failure(ctx):
    _check(ctx, _lib.lmosem_inject_failure(ctx))


def lmosem_cache_rows(ctx, evset, enable: bool):
    _check(ctx, _lib.lmosem_cache_rows(ctx, evset, 1 if enable else 0))


def _edges(e_edges):
    return np.ascontiguousarray(e_edges, np.float64)


def lmosem_bin_events(ctx, events: dict, n_pos: int, e_edges, counts_out: torch.Tensor):
    ev = _events(events)
    ed = _edges(e_edges)
    _check(ctx, _lib.lmosem_bin_events(ctx, ctypes.byref(ev), int(n_pos), ed.ctypes.data, len(ed) - 1,
                                       _dev_ptr(counts_out, torch.float32, "counts")))


def lmosem_emission_mask(ctx, image: torch.Tensor, rel_threshold: float, margin_px: int, mask_out: torch.Tensor):
    """mask_out [ny][nx] = 1 on mu > 0 pixels within margin_px of a pixel with
    image >= rel_threshold * max(image), else 0."""
    if image.numel() != mask_out.numel():
        raise ValueError("image and mask differ in size")
    _check(ctx, _lib.lmosem_emission_mask(ctx, _dev_ptr(image, torch.float32, "image"), float(rel_threshold),
                                          int(margin_px), _dev_ptr(mask_out, torch.float32, "mask")))


def lmosem_binned_rows(ctx, n_pos: int, e_edges, bins: torch.Tensor, rows_out: torch.Tensor):
    ed = _edges(e_edges)
    _check(ctx, _lib.lmosem_binned_rows(ctx, int(n_pos), ed.ctypes.data, len(ed) - 1, int(bins.numel()),
                                        _dev_ptr(bins, torch.int32, "bins"),
                                        _dev_ptr(rows_out, torch.float32, "rows")))


def lmosem_binned_reconstruct(ctx, n_pos: int, e_edges, counts: torch.Tensor, n_iters: int,
                              image_out: torch.Tensor, init: torch.Tensor | None = None):
    ed = _edges(e_edges)
    _check(ctx, _lib.lmosem_binned_reconstruct(ctx, int(n_pos), ed.ctypes.data, len(ed) - 1,
                                               _dev_ptr(counts, torch.float32, "counts"), int(n_iters),
                                               _dev_ptr(init, torch.float32, "init"),
                                               _dev_ptr(image_out, torch.float32, "image")))


def lmosem_measure_alu_rates(stream: torch.cuda.Stream | None = None) -> dict:
    st = (stream or torch.cuda.current_stream()).cuda_stream
    out = (ctypes.c_double * 3)()
    s = _lib.lmosem_measure_alu_rates(ctypes.c_void_p(st), out)
    if s != OK:
        raise LmosemError(s, "ALU probe failed")
    return {"fma_per_s": out[0], "exp2_per_s": out[1], "term_per_s": out[2]}


N_NET_PARAMS = 34305
NET_KEYS = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")


def net_flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], np.float32).ravel() for k in NET_KEYS])


def net_unflatten(flat: np.ndarray) -> dict:
    shapes = {"W1": (8, 128), "b1": (128,), "W2": (128, 128), "b2": (128,), "W3": (128, 128),
              "b3": (128,), "W4": (128, 1), "b4": (1,)}
    out, o = {}, 0
    for k in NET_KEYS:
        n = int(np.prod(shapes[k]))
        out[k] = flat[o:o + n].reshape(shapes[k]).copy()
        o += n
    return out


def _check_plain(status: int, what: str):
    if status != OK:
        raise LmosemError(status, what)


def lmosem_net_create(params: dict, stream: torch.cuda.Stream | None = None):
    flat = np.ascontiguousarray(net_flatten(params))
    st = (stream or torch.cuda.current_stream()).cuda_stream
    out = ctypes.c_void_p()
    _check_plain(_lib.lmosem_net_create(flat.ctypes.data, ctypes.c_void_p(st), ctypes.byref(out)),
                 "lmosem_net_create")
    return out


def lmosem_net_destroy(net):
    _lib.lmosem_net_destroy(net)


def lmosem_net_get_params(net) -> dict:
    flat = np.empty(N_NET_PARAMS, np.float32)
    _check_plain(_lib.lmosem_net_get_params(net, flat.ctypes.data), "lmosem_net_get_params")
    return net_unflatten(flat)


def lmosem_net_forward(net, X: torch.Tensor, y_out: torch.Tensor):
    _check_plain(_lib.lmosem_net_forward(net, _dev_ptr(X, torch.float32, "X"), int(X.shape[0]),
                                         _dev_ptr(y_out, torch.float32, "y")), "lmosem_net_forward")


def lmosem_net_forward_train(net, X: torch.Tensor, y_out: torch.Tensor):
    _check_plain(_lib.lmosem_net_forward_train(net, _dev_ptr(X, torch.float32, "X"), int(X.shape[0]),
                                               _dev_ptr(y_out, torch.float32, "y")), "lmosem_net_forward_train")


def lmosem_net_gradient(net, X: torch.Tensor, dy: torch.Tensor) -> dict:
    g = np.empty(N_NET_PARAMS, np.float32)
    _check_plain(_lib.lmosem_net_gradient(net, _dev_ptr(X, torch.float32, "X"),
                                          _dev_ptr(dy, torch.float32, "dy"), int(X.shape[0]),
                                          g.ctypes.data), "lmosem_net_gradient")
    return net_unflatten(g)


def lmosem_net_train(net, X: torch.Tensor, t: torch.Tensor, batch: int, epochs: int, lr: float,
                     lr_decay: float = 1.0) -> np.ndarray:
    loss = (ctypes.c_double * max(epochs, 1))()
    _check_plain(_lib.lmosem_net_train(net, _dev_ptr(X, torch.float32, "X"), _dev_ptr(t, torch.float32, "t"),
                                       int(X.shape[0]), int(batch), int(epochs), float(lr), float(lr_decay),
                                       loss), "lmosem_net_train")
    return np.ctypeslib.as_array(loss)[:epochs].copy()


def lmosem_surrogate_samples(ctx, pixel: torch.Tensor, angle: torch.Tensor, u_bin: torch.Tensor,
                             energy: torch.Tensor, want_scatter=False):
    n = int(pixel.numel())
    dev = pixel.device
    X = torch.empty((n, 8), dtype=torch.float32, device=dev)
    t = torch.empty(n, dtype=torch.float32, device=dev)
    sc = torch.empty(n, dtype=torch.float32, device=dev) if want_scatter else None
    _check(ctx, _lib.lmosem_surrogate_samples(ctx, _dev_ptr(pixel, torch.int32, "pixel"),
                                              _dev_ptr(angle, torch.int32, "angle"),
                                              _dev_ptr(u_bin, torch.float32, "u_bin"),
                                              _dev_ptr(energy, torch.float32, "energy"), n,
                                              _dev_ptr(X, torch.float32, "X"), _dev_ptr(t, torch.float32, "t"),
                                              _dev_ptr(sc, torch.float32, "scatter")))
    return (X, t, sc) if want_scatter else (X, t)


def lmosem_set_surrogate(ctx, net):
    _check(ctx, _lib.lmosem_set_surrogate(ctx, net))


class Context:
    """Owning wrapper: a context plus convenience allocation of outputs."""

    def __init__(self, geom: dict, mu: torch.Tensor, stream: torch.cuda.Stream | None = None,
                 emission: torch.Tensor | None = None):
        self.geom = dict(geom)
        self.device = mu.device
        self.handle = lmosem_create_emission(geom, mu, emission, stream)

    def close(self):
        if self.handle:
            lmosem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _img(self, n=1):
        shape = (self.geom["ny"], self.geom["nx"]) if n == 1 else (n, self.geom["ny"], self.geom["nx"])
        return torch.zeros(shape, dtype=torch.float32, device=self.device)

    def sensitivity(self, subset: int = -1) -> torch.Tensor:
        out = self._img()
        lmosem_sensitivity(self.handle, subset, out)
        return out

    def forward(self, events: dict, image: torch.Tensor) -> torch.Tensor:
        out = torch.empty(events["angle"].numel(), dtype=torch.float32, device=self.device)
        lmosem_forward(self.handle, events, image, out)
        return out

    def backproject(self, events: dict, weights: torch.Tensor) -> torch.Tensor:
        out = self._img()
        lmosem_backproject(self.handle, events, weights, out)
        return out

    def subset_update(self, subset: int, events: dict, image: torch.Tensor) -> torch.Tensor:
        mean = torch.empty(events["angle"].numel(), dtype=torch.float32, device=self.device)
        lmosem_subset_update(self.handle, subset, events, image, mean)
        return mean

    def reconstruct(self, events: dict, n_iters: int, init=None, batch_offsets=None,
                    want_loglik=False):
        n_real = 1 if batch_offsets is None else len(batch_offsets) - 1
        out = self._img(n_real) if n_real > 1 else self._img()
        ll = lmosem_reconstruct(self.handle, events, n_iters, out, init, batch_offsets, want_loglik)
        return (out, ll) if want_loglik else out

    def set_tuning(self, event_tile: int, pixel_tile: int = 0):
        lmosem_set_tuning(self.handle, event_tile)
        lmosem_set_pixel_tile(self.handle, pixel_tile)

    def stats(self) -> dict:
        return lmosem_get_stats(self.handle)


def events_to_device(ev: dict, device="cuda") -> dict:
    """numpy event arrays -> GPU tensors of the dtypes the library takes."""
    return {"angle": torch.as_tensor(np.ascontiguousarray(ev["angle"], np.int32), device=device),
            "u_bin": torch.as_tensor(np.ascontiguousarray(ev["u_bin"], np.float32), device=device),
            "energy": torch.as_tensor(np.ascontiguousarray(ev["energy"], np.float32), device=device)}

"""FP64 CPU oracle for list-mode OS-EM with attenuation and scatter compensation.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may use this module.  It shares no code with the
GPU library (``paper_2002_12471_amd``) and neither imports the other.

Layers:
  * ``lmosem_oracle.c`` (plain C, double precision): line integrals, photon
    physics, detector response, system rows h(q; A_j) and sensitivities.
  * this file: ctypes access to it, and the EM algebra of Sec. 2 in NumPy:
    the per-event mean (denominator of Eq. 8), the backprojection
    (numerator of Eq. 7 summed over paths), the multiplicative update of
    Eq. 6/7 with subsets by detector angle, the iteration order of Eq. 9 and
    the list-mode log-likelihood of Eq. 3 up to constants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lmosem_oracle.c")
_LIB = os.path.join(_HERE, "liblmosem_oracle.so")
_lib = None

__all__ = ["build", "OracleModel", "os_lm_mlem", "subset_update", "log_likelihood",
           "surrogate_features", "surrogate_target", "line_extent", "binned_rows", "binned_os_mlem",
           "emission_mask",
           "compton_energy", "kn_shape", "kn_total", "rho", "psi_bar", "resp_K", "resp_D",
           "resp_G", "resp_W", "line_integral", "circle_mean", "default_threads"]


def build() -> str:
    """Compile the oracle with gcc (no fast-math: IEEE double throughout)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("dx", ctypes.c_double), ("n_bins", ctypes.c_int),
                ("bin_cm", ctypes.c_double), ("n_angles", ctypes.c_int),
                ("angle0", ctypes.c_double), ("e0", ctypes.c_double),
                ("fwhm_e", ctypes.c_double), ("fwhm_u", ctypes.c_double),
                ("win_lo", ctypes.c_double), ("win_hi", ctypes.c_double),
                ("n_subsets", ctypes.c_int), ("scatter", ctypes.c_int),
                ("acq_time", ctypes.c_double)]


_D = ctypes.c_double
_I = ctypes.c_int
_P = ctypes.c_void_p
_CB = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.c_double, ctypes.c_void_p)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        sig = {
            "orc_line_integral": (_D, [_P, _I, _D, _D, _D, _D, _D]),
            "orc_compton_energy": (_D, [_D, _D]),
            "orc_kn_shape": (_D, [_D, _D]),
            "orc_kn_total": (_D, [_D]),
            "orc_rho": (_D, [_D, _D]),
            "orc_circle_mean": (_D, [_CB, _P, _I]),
            "orc_psi_bar": (_D, [_D, _I]),
            "orc_K": (_D, [_D, _D]),
            "orc_D": (_D, [_D, _D, _D]),
            "orc_G": (_D, [_D, _D, _D]),
            "orc_W": (_D, [_D, _D, _D, _D]),
            "orc_model_create": (_I, [ctypes.POINTER(_Cfg), _P, _I, ctypes.POINTER(_P)]),
            "orc_model_free": (None, [_P]),
            "orc_n_support": (_I, [_P]),
            "orc_support": (None, [_P, _P]),
            "orc_psi_bar_of": (_D, [_P]),
            "orc_L": (_D, [_P, _I, _I]),
            "orc_B": (_D, [_P, _I, _I]),
            "orc_h": (_D, [_P, _I, _I, _D, _D]),
            "orc_sens_angle": (_D, [_P, _I, _I]),
            "orc_box_prob": (_D, [_P, _I, _I, _D, _D, _D, _D]),
            "orc_system_matrix": (_I, [_P, _P, _P, _P, ctypes.c_longlong, _P, _I, _P]),
            "orc_sensitivity": (_I, [_P, _I, _P, _I, _P]),
            "orc_box_sums": (_I, [_P, _P, _I, _D, _D, _D, _D, _P, _I, _P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# ---------------------------------------------------------------- physics
def compton_energy(e, c):
    return _load().orc_compton_energy(float(e), float(c))


def kn_shape(e, c):
    return _load().orc_kn_shape(float(e), float(c))


def kn_total(e):
    return _load().orc_kn_total(float(e))


def rho(e, e0):
    return _load().orc_rho(float(e), float(e0))


def psi_bar(e0, m=512):
    return _load().orc_psi_bar(float(e0), int(m))


def circle_mean(fn, m):
    """Periodic trapezoid mean of fn over [0, 2 pi) with m nodes."""
    cb = _CB(lambda phi, _arg: float(fn(phi)))
    return _load().orc_circle_mean(cb, None, int(m))


def resp_K(d, sigma):
    return _load().orc_K(float(d), float(sigma))


def resp_D(u_p, half, sigma):
    return _load().orc_D(float(u_p), float(half), float(sigma))


def resp_G(e, ep, sigma):
    return _load().orc_G(float(e), float(ep), float(sigma))


def resp_W(ep, lo, hi, sigma):
    return _load().orc_W(float(ep), float(lo), float(hi), float(sigma))


def line_integral(mu: np.ndarray, dx: float, p0, p1) -> float:
    m = np.ascontiguousarray(mu, dtype=np.float64)
    n = m.shape[0]
    assert m.shape == (n, n)
    return _load().orc_line_integral(m.ctypes.data, n, float(dx), float(p0[0]), float(p0[1]),
                                     float(p1[0]), float(p1[1]))


# ---------------------------------------------------------------- model
class OracleModel:
    """Geometry-dependent part of the system model for one attenuation map."""

    def __init__(self, geom: dict, mu: np.ndarray, scatter: int | None = None,
                 n_threads: int | None = None):
        lib = _load()
        self.geom = dict(geom)
        n = int(geom["nx"])
        if int(geom["ny"]) != n:
            raise ValueError("the oracle handles square grids")
        self.n = n
        self.mu = np.ascontiguousarray(mu, dtype=np.float64).reshape(n, n)
        sc = int(geom.get("scatter_model", 1) if scatter is None else scatter)
        self.cfg = _Cfg(n, float(geom["pixel_cm"]), int(geom["n_bins"]), float(geom["bin_cm"]),
                        int(geom["n_angles"]), float(geom.get("angle0_rad", 0.0)),
                        float(geom["e0_kev"]), float(geom["fwhm_e_kev"]),
                        float(geom["fwhm_u_cm"]), float(geom["win_lo_kev"]),
                        float(geom["win_hi_kev"]), int(geom["n_subsets"]), 1 if sc else 0,
                        float(geom.get("acq_time", 1.0)))
        self.n_threads = int(n_threads or default_threads())
        h = _P()
        rc = lib.orc_model_create(ctypes.byref(self.cfg), self.mu.ctypes.data, self.n_threads,
                                  ctypes.byref(h))
        if rc != 0:
            raise ValueError("oracle model rejected the configuration or map")
        self._h = h
        ns = lib.orc_n_support(h)
        sup = np.empty(ns, np.int32)
        if ns:
            lib.orc_support(h, sup.ctypes.data)
        self.support = sup

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_model_free(h)
            self._h = None

    @property
    def psi_bar(self) -> float:
        return _load().orc_psi_bar_of(self._h)

    def L(self, a: int, pix: int) -> float:
        return _load().orc_L(self._h, int(a), int(pix))

    def B(self, q: int, s: int) -> float:
        return _load().orc_B(self._h, int(q), int(s))

    def h(self, q: int, a: int, u_cm: float, e_kev: float) -> float:
        return _load().orc_h(self._h, int(q), int(a), float(u_cm), float(e_kev))

    def sens_angle(self, q: int, a: int) -> float:
        return _load().orc_sens_angle(self._h, int(q), int(a))

    def box_prob(self, q: int, a: int, ulo: float, uhi: float, elo: float, ehi: float) -> float:
        """Integral of h(q; a, u, E) over u in [ulo, uhi] (cm) and E in [elo, ehi] (keV)."""
        return _load().orc_box_prob(self._h, int(q), int(a), float(ulo), float(uhi), float(elo),
                                    float(ehi))

    def u_cm(self, u_bin):
        return (np.asarray(u_bin, np.float64) - 0.5 * self.geom["n_bins"]) * self.geom["bin_cm"]

    def system_matrix(self, events: dict, qlist=None) -> np.ndarray:
        """H[j, k] = h(qlist[k]; event j) in float64 (default qlist: the support)."""
        q = self.support if qlist is None else np.ascontiguousarray(qlist, np.int32)
        ang = np.ascontiguousarray(events["angle"], np.int32)
        ub = np.ascontiguousarray(events["u_bin"], np.float32)
        en = np.ascontiguousarray(events["energy"], np.float32)
        out = np.empty((len(ang), len(q)), np.float64)
        rc = _load().orc_system_matrix(self._h, ang.ctypes.data, ub.ctypes.data, en.ctypes.data,
                                       len(ang), q.ctypes.data, len(q), out.ctypes.data)
        if rc != 0:
            raise ValueError("event angle or pixel index out of range")
        return out

    def sensitivity(self, subset: int = -1, qlist=None) -> np.ndarray:
        """T * sum over the subset's angles of the path sensitivities, per listed pixel."""
        q = self.support if qlist is None else np.ascontiguousarray(qlist, np.int32)
        out = np.empty(len(q), np.float64)
        rc = _load().orc_sensitivity(self._h, int(subset), q.ctypes.data, len(q),
                                     out.ctypes.data)
        if rc != 0:
            raise ValueError("subset out of range")
        return out

    def box_sums(self, angles, ulo, uhi, elo, ehi, qlist=None) -> np.ndarray:
        """Per listed pixel: sum over the given angles of the box probability."""
        q = self.support if qlist is None else np.ascontiguousarray(qlist, np.int32)
        a = np.ascontiguousarray(angles, np.int32)
        out = np.empty(len(q), np.float64)
        rc = _load().orc_box_sums(self._h, a.ctypes.data, len(a), float(ulo), float(uhi),
                                  float(elo), float(ehi), q.ctypes.data, len(q), out.ctypes.data)
        if rc != 0:
            raise ValueError("angle out of range")
        return out

    def to_image(self, vec, qlist=None) -> np.ndarray:
        q = self.support if qlist is None else np.asarray(qlist)
        img = np.zeros(self.n * self.n, np.float64)
        img[q] = vec
        return img.reshape(self.n, self.n)


# ---------------------------------------------------------------- surrogate references
def line_extent(mu: np.ndarray, dx: float, foot, nvec) -> tuple:
    """Where the line foot + t nvec runs through pixels with mu > 0: the
    smallest and largest t of those stretches, or None when it meets none.
    Each stretch between consecutive crossings of the grid lines is assigned
    to the pixel holding its midpoint."""
    n = mu.shape[0]
    half = 0.5 * n * dx
    ts = []
    for k in range(2):
        if abs(nvec[k]) > 1e-15:
            for m in range(n + 1):
                ts.append(((m * dx - half) - foot[k]) / nvec[k])
    ts = np.unique(np.array(ts))
    t_in = t_out = None
    for t0, t1 in zip(ts[:-1], ts[1:]):
        if t1 - t0 < 1e-12:
            continue
        mid = foot + 0.5 * (t0 + t1) * np.asarray(nvec)
        i, j = int(np.floor(mid[0] / dx + 0.5 * n)), int(np.floor(mid[1] / dx + 0.5 * n))
        if 0 <= i < n and 0 <= j < n and mu[j, i] > 0:
            t_in = t0 if t_in is None else t_in
            t_out = t1
    return None if t_in is None else (float(t_in), float(t_out))


def surrogate_features(model: "OracleModel", pixel: int, a: int, u_cm: float, e_kev: float) -> np.ndarray:
    """Inputs of the scatter surrogate for (pixel, angle, position, energy),
    each with the fixed scale the network uses: the event's offset from the
    pixel's own detector position, the energy, where the event's detector
    line enters and leaves the body relative to the pixel's depth, the line's
    position-response-weighted attenuation sum_s mu(s) dx k(u - u_s) over all
    pixels s (k the unnormalised truncated Gaussian position response),
    the attenuation from the pixel toward and away from the detector, and mu
    at the pixel."""
    g = model.geom
    n, dx = model.n, float(g["pixel_cm"])
    th = float(g.get("angle0_rad", 0.0)) + 2 * np.pi * a / int(g["n_angles"])
    nvec = np.array([np.cos(th), np.sin(th)])
    tvec = np.array([-np.sin(th), np.cos(th)])
    idx = np.arange(n)
    cx, cy = (idx - (n - 1) / 2) * dx, (idx - (n - 1) / 2) * dx
    c = np.array([cx[pixel % n], cy[pixel // n]])
    far = 4.0 * n * dx
    uq, dq = float(c @ tvec), float(c @ nvec)
    to_det = line_integral(model.mu, dx, c, c + far * nvec)
    away = line_integral(model.mu, dx, c, c - far * nvec)
    ext = line_extent(model.mu, dx, u_cm * tvec, nvec)
    d_in, d_out = (0.0, 0.0) if ext is None else (ext[0] - dq, ext[1] - dq)
    sig_u = float(g["fwhm_u_cm"]) / (2 * np.sqrt(2 * np.log(2)))
    ck = 0.0
    for p in np.flatnonzero(model.mu.ravel() > 0):
        us = float(np.array([cx[p % n], cy[p // n]]) @ tvec)
        ck += model.mu.flat[p] * dx * max(np.exp(-(u_cm - us) ** 2 / (2 * sig_u ** 2)) - np.exp(-4.5), 0.0)
    return np.array([(u_cm - uq) / 2, (e_kev - 130) / 30, d_in / 10, d_out / 10, ck / 2, to_det, away,
                     10 * model.mu.flat[pixel]])


def surrogate_target(scatter_sum: float, geom: dict, floor: float = 1e-4) -> float:
    """Training target of the surrogate: ln(S / S0 + floor), S0 = 1 / (pixel_cm sigma_E)."""
    sig_e = float(geom["fwhm_e_kev"]) / (2 * np.sqrt(2 * np.log(2)))
    return float(np.log(scatter_sum * float(geom["pixel_cm"]) * sig_e + floor))


# ---------------------------------------------------------------- EM algebra
def subset_update(H_i: np.ndarray, f: np.ndarray, sens_i: np.ndarray, tiny: float = 1e-30):
    """One sub-iteration of Eq. 7 with the posterior of Eq. 8.

    H_i[j, q] = pr(A_j | P_q) s_eff(P_q) summed over the paths from q, for the
    events of this subset.  The mean of event j is sum_q f_q H_i[j, q] (the
    denominator of Eq. 8, with the normaliser of Eq. 4 cancelled); the
    expected number of event-j paths from q is f_q H_i[j, q] / mean_j; their
    sum over j divided by the subset sensitivity gives the new f_q.  Pixels
    with zero sensitivity keep their value; events whose mean is not above
    ``tiny`` are left out and counted."""
    mean = H_i @ f
    ok = mean > tiny
    inv = np.where(ok, 1.0 / np.where(ok, mean, 1.0), 0.0)
    b = H_i.T @ inv
    new = np.where(sens_i > 0, f * b / np.where(sens_i > 0, sens_i, 1.0), f)
    return new, mean, int((~ok).sum())


def log_likelihood(mean: np.ndarray, f: np.ndarray, sens_total: np.ndarray) -> float:
    """Eq. 3 without its f-independent terms: sum_j log mean_j - sum_q f_q sens_q
    (the expected count T sum_P f(P) s_eff(P))."""
    return float(np.sum(np.log(mean[mean > 0])) - np.dot(f, sens_total))


def binned_rows(model: "OracleModel", n_pos: int, e_edges, angles=None) -> np.ndarray:
    """System matrix of binned data (Sec. 2.2's binned alternative to list
    mode): for bin (a, b, k) — position bin b of n_pos equal bins over the
    detector, energy bin [e_edges[k], e_edges[k+1]) — the row over the support,
    H[(a, b, k), q] = integral of h(q; a, u, E) over the bin, from the
    closed-form box probability.  Rows in (a, b, k) order; angles default to
    all."""
    g = model.geom
    half = 0.5 * int(g["n_bins"]) * float(g["bin_cm"])
    width = 2 * half / n_pos
    angles = range(int(g["n_angles"])) if angles is None else angles
    rows = []
    for a in angles:
        for b in range(n_pos):
            for k in range(len(e_edges) - 1):
                rows.append(model.box_sums([a], -half + b * width, -half + (b + 1) * width,
                                           e_edges[k], e_edges[k + 1]))
    return np.array(rows)


def binned_os_mlem(H: np.ndarray, y: np.ndarray, row_angle: np.ndarray, n_subsets: int, n_iters: int,
                   f0: np.ndarray) -> np.ndarray:
    """Binned OS-MLEM (Eq. 7 with counts): subsets by detector angle as in
    list mode, each sub-iteration f <- f * H_i^T (y_i / H_i f) / H_i^T 1 over
    the subset's rows; bins with zero mean are left out."""
    f = np.asarray(f0, np.float64).copy()
    sub = np.asarray(row_angle) % n_subsets
    for _ in range(n_iters):
        for i in range(n_subsets):
            Hi, yi = H[sub == i], np.asarray(y, np.float64)[sub == i]
            mean = Hi @ f
            ok = mean > 1e-30
            ratio = np.where(ok, yi / np.where(ok, mean, 1.0), 0.0)
            sens = Hi.sum(axis=0)
            b = Hi.T @ ratio
            f = np.where(sens > 0, f * b / np.where(sens > 0, sens, 1.0), f)
    return f


def emission_mask(image: np.ndarray, mu: np.ndarray, rel_threshold: float, margin_px: int) -> np.ndarray:
    """Emission set from a crude image (Sec. 2.2: the estimate is confined to
    a rough object boundary from a binned OS-MLEM, since the work per
    iteration grows with the number of estimated pixels).  Reading: the
    boundary is {image >= rel_threshold * max(image)} grown by every pixel
    offset (di, dj) with di^2 + dj^2 <= margin_px^2, then intersected with
    mu > 0; the threshold comparison is in float64.  Returns a float32 0/1
    map."""
    img = np.asarray(image, np.float64)
    ny, nx = img.shape
    hot = img >= rel_threshold * img.max()
    m = int(margin_px)
    padded = np.zeros((ny + 2 * m, nx + 2 * m), bool)
    padded[m:m + ny, m:m + nx] = hot
    grown = np.zeros((ny, nx), bool)
    for dj in range(-m, m + 1):
        for di in range(-m, m + 1):
            if di * di + dj * dj <= m * m:
                grown |= padded[m + dj:m + dj + ny, m + di:m + di + nx]
    return (grown & (np.asarray(mu) > 0)).astype(np.float32)


def os_lm_mlem(H: np.ndarray, angle: np.ndarray, sens_subsets: np.ndarray, n_iters: int,
               f0: np.ndarray, n_subsets: int):
    """OS-LM-MLEM (Eq. 7-9): subsets by detector angle (subset i holds the
    angles a with a mod N_s == i), visited i = 0..N_s-1 within each global
    iteration; every sub-iteration starts from the latest estimate.

    Returns the final estimate and, per global iteration, the sum over
    sub-iterations of (sum_{j in S_i} log mean_j - sum_q f_q sens_q^(i)) at the
    estimate each sub-iteration started from (for one subset this is the
    log-likelihood of the estimate the iteration started from)."""
    f = np.asarray(f0, np.float64).copy()
    sub = np.asarray(angle) % n_subsets
    rows = [np.nonzero(sub == i)[0] for i in range(n_subsets)]
    ll = []
    for _t in range(n_iters):
        acc = 0.0
        for i in range(n_subsets):
            Hi = H[rows[i]]
            f_new, mean, _skipped = subset_update(Hi, f, sens_subsets[i])
            acc += log_likelihood(mean, f, sens_subsets[i])
            f = f_new
        ll.append(acc)
    return f, np.array(ll)

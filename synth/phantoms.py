"""Seeded synthetic workloads: geometry configurations and 2-D phantoms.

This module holds input generation only: image grids, detector geometry and
the activity / attenuation phantoms the reconstruction is run on.  It contains
none of the reconstruction's arithmetic.

The paper evaluates on the Zubal digital brain phantom with Monte-Carlo
list-mode data for a 2-D DaT-scan study (Sec. 3).  Neither is available here,
so these analytic phantoms stand in for them: a water disk with a hot ellipse
(tiny case) and a skull-ring head with caudate and putamen ellipses at 8:1
uptake (brain cases).  Pixels are rasterised by a pixel-centre test.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np


@dataclass
class Geometry:
    """Image grid, detector and energy settings of one workload."""
    nx: int
    ny: int
    pixel_cm: float
    n_bins: int
    bin_cm: float
    n_angles: int
    angle0_rad: float = 0.0
    e0_kev: float = 159.0           # I-123 photopeak (DaT tracer)
    fwhm_e_kev: float = 15.9        # 10 % energy resolution
    fwhm_u_cm: float | None = None  # defaults to the pixel pitch
    win_lo_kev: float = 100.0
    win_hi_kev: float = 175.0
    n_subsets: int = 1
    scatter_model: int = 1
    acq_time: float = 1.0

    def __post_init__(self):
        if self.fwhm_u_cm is None:
            self.fwhm_u_cm = self.pixel_cm

    def as_dict(self) -> dict:
        return asdict(self)


@dataclass
class Workload:
    name: str
    geom: Geometry
    n_events: int
    n_iters: int
    phantom: str
    n_real: int = 1
    extra: dict = field(default_factory=dict)


def pixel_centres(nx: int, ny: int, dx: float):
    """Centre coordinates (cm) of pixel (i, j), stored row-major [j][i]."""
    x = (np.arange(nx) - (nx - 1) / 2.0) * dx
    y = (np.arange(ny) - (ny - 1) / 2.0) * dx
    return np.meshgrid(x, y)  # X[j, i], Y[j, i]


def _ellipse(X, Y, cx, cy, ax, ay, rot_deg=0.0):
    t = math.radians(rot_deg)
    xr = (X - cx) * math.cos(t) + (Y - cy) * math.sin(t)
    yr = -(X - cx) * math.sin(t) + (Y - cy) * math.cos(t)
    return (xr / ax) ** 2 + (yr / ay) ** 2 <= 1.0


def disk_phantom(g: Geometry):
    """Water disk (mu 0.15/cm, radius 7 px) with an activity disk of radius
    6 px (value 1) and a hot ellipse of value 4."""
    X, Y = pixel_centres(g.nx, g.ny, g.pixel_cm)
    dx = g.pixel_cm
    mu = np.where(X ** 2 + Y ** 2 <= (7 * dx) ** 2, 0.15, 0.0)
    act = np.where(X ** 2 + Y ** 2 <= (6 * dx) ** 2, 1.0, 0.0)
    hot = _ellipse(X, Y, 2.0 * dx, 1.0 * dx, 2.5 * dx, 1.5 * dx)
    act = np.where(hot & (act > 0), 4.0, act)
    return act.astype(np.float32), mu.astype(np.float32)


def brain_phantom(g: Geometry):
    """Head: skull ring (mu 0.25/cm) around brain (mu 0.15/cm, activity 1),
    caudate and putamen ellipse pairs at activity 8 (8:1 striatal uptake).
    Sizes are in cm, so the same head rasterises at any pixel pitch."""
    X, Y = pixel_centres(g.nx, g.ny, g.pixel_cm)
    outer = _ellipse(X, Y, 0.0, 0.0, 7.6, 9.6)
    inner = _ellipse(X, Y, 0.0, 0.0, 6.8, 8.8)
    mu = np.where(outer, 0.25, 0.0)
    mu = np.where(inner, 0.15, mu)
    act = np.where(inner, 1.0, 0.0)
    striatum = (_ellipse(X, Y, -1.3, 1.0, 0.7, 1.1) | _ellipse(X, Y, 1.3, 1.0, 0.7, 1.1)
                | _ellipse(X, Y, -2.7, -0.4, 0.6, 1.5, rot_deg=-20.0)
                | _ellipse(X, Y, 2.7, -0.4, 0.6, 1.5, rot_deg=20.0))
    act = np.where(striatum & inner, 8.0, act)
    return act.astype(np.float32), mu.astype(np.float32)


def striatal_masks(g: Geometry):
    """Caudate and putamen masks of the brain phantom (task regions)."""
    X, Y = pixel_centres(g.nx, g.ny, g.pixel_cm)
    caud = _ellipse(X, Y, -1.3, 1.0, 0.7, 1.1) | _ellipse(X, Y, 1.3, 1.0, 0.7, 1.1)
    put = (_ellipse(X, Y, -2.7, -0.4, 0.6, 1.5, rot_deg=-20.0)
           | _ellipse(X, Y, 2.7, -0.4, 0.6, 1.5, rot_deg=20.0))
    return caud, put


def random_ellipse_map(g: Geometry, rng: np.random.Generator, shell_prob: float = 0.0,
                       body=(0.4, 0.9)):
    """Random elliptical attenuation map for surrogate training: a body
    ellipse (semi-axes a fraction `body` of the half field of view) plus 0-2
    inserts, each with its own mu in [0.1, 0.3]/cm.  With probability
    shell_prob the body gets a skull-like shell 0.4-1.2 cm thick with mu in
    [0.2, 0.3]/cm (no random numbers are drawn for it when shell_prob is 0)."""
    X, Y = pixel_centres(g.nx, g.ny, g.pixel_cm)
    half = 0.5 * g.nx * g.pixel_cm
    mu = np.zeros_like(X)
    body_a = rng.uniform(body[0], body[1], size=2) * half
    c = rng.uniform(-0.2, 0.2, size=2) * half
    rot = rng.uniform(0, 180)
    body_m = _ellipse(X, Y, c[0], c[1], body_a[0], body_a[1], rot)
    mu[body_m] = rng.uniform(0.1, 0.3)
    inside = body_m
    if shell_prob > 0 and rng.uniform() < shell_prob:
        t = rng.uniform(0.4, 1.2)
        inside = _ellipse(X, Y, c[0], c[1], body_a[0] - t, body_a[1] - t, rot)
        mu[body_m & ~inside] = rng.uniform(0.2, 0.3)
    for _ in range(rng.integers(0, 3)):
        ia = rng.uniform(0.1, 0.3, size=2) * half
        ic = c + rng.uniform(-0.3, 0.3, size=2) * half
        ins = _ellipse(X, Y, ic[0], ic[1], ia[0], ia[1], rng.uniform(0, 180)) & inside
        mu[ins] = rng.uniform(0.1, 0.3)
    return mu.astype(np.float32)


def workload(name: str) -> Workload:
    """The workloads: tiny disk, 64x64 brain, batched tiny realisations,
    surrogate training maps (tiny grid), 128x128 brain, surrogate training
    maps on the 128x128 grid."""
    if name == "tiny":
        g = Geometry(16, 16, 0.8, 16, 0.8, 16, win_lo_kev=100.0, win_hi_kev=175.0,
                     n_subsets=1)
        return Workload(name, g, 5000, 5, "disk")
    if name == "brain64":
        g = Geometry(64, 64, 0.4, 128, 0.2, 120, n_subsets=8)
        return Workload(name, g, 200_000, 10, "brain")
    if name == "batch_tiny":
        g = Geometry(16, 16, 0.8, 16, 0.8, 16, n_subsets=1)
        return Workload(name, g, 0, 5, "disk", n_real=64,
                        extra={"min_events": 50_000, "max_events": 500_000})
    if name == "surrogate_maps":
        g = Geometry(16, 16, 0.8, 16, 0.8, 16, n_subsets=1)
        return Workload(name, g, 0, 5, "random_maps", extra={"n_maps": 256,
                                                             "n_samples": 4_000_000})
    if name == "brain128":
        g = Geometry(128, 128, 0.2, 256, 0.1, 120, win_lo_kev=90.0, win_hi_kev=175.0,
                     n_subsets=16)
        return Workload(name, g, 2_000_000, 10, "brain", n_real=16)
    if name == "surrogate_maps_128":
        g = Geometry(128, 128, 0.2, 256, 0.1, 120, win_lo_kev=90.0, win_hi_kev=175.0,
                     n_subsets=16)
        return Workload(name, g, 0, 10, "random_maps", extra={"n_maps": 256, "n_samples": 4_000_000,
                                                              "shell_prob": 0.5, "body": (0.45, 0.8)})
    raise KeyError(name)


WORKLOAD_INDEX = {"tiny": 1, "brain64": 2, "batch_tiny": 3, "surrogate_maps": 4, "brain128": 5,
                  "surrogate_maps_128": 6}


def phantom(w: Workload):
    if w.phantom == "disk":
        return disk_phantom(w.geom)
    if w.phantom == "brain":
        return brain_phantom(w.geom)
    raise KeyError(w.phantom)


def seed_for(w: Workload, realisation: int = 0) -> int:
    return 20200403 + 1000 * WORKLOAD_INDEX[w.name] + realisation


def batch_event_counts(w: Workload) -> np.ndarray:
    """Log-uniform uneven realisation sizes for the batched workload."""
    rng = np.random.default_rng(seed_for(w, 999_999))
    lo, hi = w.extra["min_events"], w.extra["max_events"]
    return np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), size=w.n_real))).astype(np.int64)


# ---------------------------------------------------------------- surrogate
MLP_SIZES = (8, 128, 128, 128, 1)


def mlp_init_params(seed: int) -> dict:
    """Seeded initial weights of the 8-128-128-128-1 scatter surrogate
    (Glorot-uniform weights, zero biases); an input of training, shared by the
    GPU trainer and the FP64 reference."""
    rng = np.random.default_rng(seed)
    p = {}
    for i, (a, b) in enumerate(zip(MLP_SIZES[:-1], MLP_SIZES[1:]), start=1):
        lim = math.sqrt(6.0 / (a + b))
        p[f"W{i}"] = rng.uniform(-lim, lim, size=(a, b)).astype(np.float32)
        p[f"b{i}"] = np.zeros(b, np.float32)
    return p


def surrogate_sample_inputs(g: Geometry, mu: np.ndarray, n: int, rng: np.random.Generator) -> dict:
    """Seeded (pixel, angle, u_bin, energy) draws for surrogate training: the
    pixel uniform on the mu > 0 support, the angle uniform, the energy uniform
    over the acceptance window, and the position uniform over the support's
    projection widened by 3 sigma_u and a pixel (kept on the detector), outside
    the pixel's own position response |u - u_q| < 3 sigma_u (the near field,
    which the network does not model)."""
    support = np.flatnonzero(np.asarray(mu).ravel() > 0).astype(np.int32)
    k = rng.integers(0, support.size, size=n)
    pix = support[k]
    ang = rng.integers(0, g.n_angles, size=n).astype(np.int32)
    X, Y = pixel_centres(g.nx, g.ny, g.pixel_cm)
    xs, ys = X.ravel()[support], Y.ravel()[support]
    th = g.angle0_rad + 2 * np.pi * np.arange(g.n_angles) / g.n_angles
    u_all = -np.sin(th)[:, None] * xs[None, :] + np.cos(th)[:, None] * ys[None, :]
    sig_u = g.fwhm_u_cm / (2 * math.sqrt(2 * math.log(2)))
    pad = 3 * sig_u + g.pixel_cm
    half_det = 0.5 * g.n_bins * g.bin_cm
    lo = np.maximum((u_all.min(axis=1) - pad)[ang], -half_det)
    hi = np.minimum((u_all.max(axis=1) + pad)[ang], half_det * (1 - 1e-6))
    uq = u_all[ang, k]
    gap_lo = np.clip(uq - 3 * sig_u, lo, hi)
    gap_hi = np.clip(uq + 3 * sig_u, lo, hi)
    u = lo + (hi - lo - (gap_hi - gap_lo)) * rng.uniform(size=n)
    u = np.where(u >= gap_lo, u + (gap_hi - gap_lo), u)
    ub = np.clip(u / g.bin_cm + 0.5 * g.n_bins, 0.0, np.nextafter(np.float32(g.n_bins), 0))
    e = rng.uniform(g.win_lo_kev, g.win_hi_kev, size=n)
    return {"pixel": pix, "angle": ang, "u_bin": ub.astype(np.float32), "energy": e.astype(np.float32)}

"""Seeded synthetic inputs shared by the tests, the oracle checks and the bench.

Input generation only (phantoms, geometry, Monte-Carlo list-mode events); it
holds none of the reconstruction's arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .phantoms import (Geometry, Workload, workload, phantom, seed_for, mlp_init_params,  # noqa: F401,E501
                       surrogate_sample_inputs,
                       batch_event_counts, striatal_masks, random_ellipse_map,
                       disk_phantom, brain_phantom, pixel_centres)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mc_events.c")
_LIB = os.path.join(_HERE, "libmc_events.so")
_lib = None


def build() -> str:
    """Compile the event generator (plain C, gcc)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("dx", ctypes.c_double),
                ("n_bins", ctypes.c_int), ("bin_cm", ctypes.c_double),
                ("n_angles", ctypes.c_int), ("angle0", ctypes.c_double),
                ("e0", ctypes.c_double), ("fwhm_e", ctypes.c_double),
                ("fwhm_u", ctypes.c_double), ("win_lo", ctypes.c_double),
                ("win_hi", ctypes.c_double)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.mc_generate.restype = ctypes.c_longlong
        lib.mc_generate.argtypes = [ctypes.POINTER(_Geom), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_longlong, ctypes.c_uint64, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]
        _lib = lib
    return _lib


def default_threads() -> int:
    # a process may be given a share of 16 CPUs whatever os.cpu_count() says
    return max(1, min(16, os.cpu_count() or 1))


def generate_events(g: Geometry, activity: np.ndarray, mu: np.ndarray, n_events: int,
                    seed: int, n_threads: int | None = None) -> dict:
    """Draw exactly ``n_events`` detected photons from the Monte-Carlo acquisition.

    Returns SoA arrays: ``angle`` int32, ``u_bin`` float32 in [0, n_bins),
    ``energy`` float32 keV, ``kind`` uint8 (0 primary, 1 first-order scatter)
    and ``histories`` (candidate histories simulated)."""
    lib = _load()
    act = np.ascontiguousarray(activity, dtype=np.float32)
    m = np.ascontiguousarray(mu, dtype=np.float32)
    assert act.shape == (g.ny, g.nx) and m.shape == (g.ny, g.nx)
    out = {"angle": np.empty(n_events, np.int32), "u_bin": np.empty(n_events, np.float32),
           "energy": np.empty(n_events, np.float32), "kind": np.empty(n_events, np.uint8)}
    geo = _Geom(g.nx, g.ny, g.pixel_cm, g.n_bins, g.bin_cm, g.n_angles, g.angle0_rad,
                g.e0_kev, g.fwhm_e_kev, g.fwhm_u_cm, g.win_lo_kev, g.win_hi_kev)
    used = lib.mc_generate(ctypes.byref(geo), act.ctypes.data, m.ctypes.data, int(n_events),
                           int(seed) & 0xFFFFFFFFFFFFFFFF, int(n_threads or default_threads()),
                           out["angle"].ctypes.data, out["u_bin"].ctypes.data,
                           out["energy"].ctypes.data, out["kind"].ctypes.data)
    if used < 0:
        raise RuntimeError("event generation failed (empty activity or bad geometry)")
    out["histories"] = int(used)
    return out


def workload_events(w: Workload, realisation: int = 0, n_events: int | None = None,
                    n_threads: int | None = None) -> dict:
    act, mu = phantom(w)
    n = w.n_events if n_events is None else n_events
    return generate_events(w.geom, act, mu, n, seed_for(w, realisation), n_threads)


def random_weights(n: int, seed: int) -> np.ndarray:
    """Seeded positive weights in [0.5, 1.5) for linearity checks."""
    return np.random.default_rng(seed).uniform(0.5, 1.5, size=n).astype(np.float32)

"""Pins of the oracle's radiological paths (Siddon) and path factors against
closed forms, brute-force integration and invariants."""
import math

import numpy as np
import pytest

import oracle as O


def _clip_to_square(p0, p1, half):
    """Length of the segment inside [-half, half]^2 (Liang-Barsky clipping)."""
    x0, y0 = p0
    dx, dy = p1[0] - x0, p1[1] - y0
    t0, t1 = 0.0, 1.0
    for p, q in ((-dx, x0 + half), (dx, half - x0), (-dy, y0 + half), (dy, half - y0)):
        if p == 0:
            if q < 0:
                return 0.0
            continue
        r = q / p
        if p < 0:
            t0 = max(t0, r)
        else:
            t1 = min(t1, r)
    return max(0.0, t1 - t0) * math.hypot(dx, dy)


def _brute(mu, dx, p0, p1, steps=200_000):
    n = mu.shape[0]
    t = (np.arange(steps) + 0.5) / steps
    x = p0[0] + t * (p1[0] - p0[0])
    y = p0[1] + t * (p1[1] - p0[1])
    i = np.floor(x / dx + n / 2).astype(int)
    j = np.floor(y / dx + n / 2).astype(int)
    ok = (i >= 0) & (i < n) & (j >= 0) & (j < n)
    vals = np.zeros(steps)
    vals[ok] = mu[j[ok], i[ok]]
    return vals.sum() * math.hypot(p1[0] - p0[0], p1[1] - p0[1]) / steps


def test_empty_map_is_zero():
    mu = np.zeros((8, 8))
    assert O.line_integral(mu, 0.5, (-3, -2), (4, 1.5)) == 0.0


@pytest.mark.parametrize("seg", [((-5, 0.3), (5, 0.3)), ((-5, -5), (5, 5)), ((0.1, 0.2), (3, -7)),
                                 ((-1.3, 0.9), (1.7, -0.4)), ((-9, 2), (9, -1.1))])
def test_uniform_map_equals_mu_times_clipped_length(seg):
    n, dx, m = 10, 0.8, 0.2
    mu = np.full((n, n), m)
    ref = m * _clip_to_square(seg[0], seg[1], n * dx / 2)
    assert O.line_integral(mu, dx, *seg) == pytest.approx(ref, rel=1e-12, abs=1e-14)


def test_uniform_disk_chord_converges():
    # 2 mu sqrt(R^2 - d^2) for a chord at distance d from the centre
    R, m = 3.0, 0.15
    errs = []
    for n in (128, 512):
        dx = 8.0 / n
        c = (np.arange(n) - (n - 1) / 2) * dx
        X, Y = np.meshgrid(c, c)
        mu = np.where(X ** 2 + Y ** 2 <= R * R, m, 0.0)
        d = 1.1
        got = O.line_integral(mu, dx, (-4.5, d), (4.5, d * 0.97 + 0.0))
        # exact chord of the slightly tilted line through (-4.5, d) and (4.5, 0.97 d)
        p0, p1 = np.array([-4.5, d]), np.array([4.5, 0.97 * d])
        u = (p1 - p0) / np.linalg.norm(p1 - p0)
        foot = p0 - np.dot(p0, u) * u
        ref = 2 * m * math.sqrt(R * R - float(np.dot(foot, foot)))
        errs.append(abs(got - ref) / ref)
    assert errs[1] < 0.01
    assert errs[1] < errs[0]


def test_random_maps_match_brute_force():
    rng = np.random.default_rng(7)
    for trial in range(6):
        n, dx = 8, 0.5
        mu = rng.uniform(0.0, 0.3, size=(n, n)) * (rng.uniform(size=(n, n)) > 0.2)
        p0 = rng.uniform(-2.5, 2.5, size=2)
        p1 = rng.uniform(-2.5, 2.5, size=2)
        assert O.line_integral(mu, dx, p0, p1) == pytest.approx(_brute(mu, dx, p0, p1), rel=2e-4)


def test_symmetry_and_additivity():
    rng = np.random.default_rng(11)
    mu = rng.uniform(0.05, 0.3, size=(12, 12))
    dx = 0.4
    p0, p2 = np.array([-2.1, 1.3]), np.array([1.9, -1.7])
    p1 = p0 + 0.37 * (p2 - p0)
    a = O.line_integral(mu, dx, p0, p2)
    assert O.line_integral(mu, dx, p2, p0) == pytest.approx(a, rel=1e-13)
    assert O.line_integral(mu, dx, p0, p1) + O.line_integral(mu, dx, p1, p2) == pytest.approx(a, rel=1e-12)


def _geom(n, dx, n_angles=8, n_bins=None, **kw):
    g = dict(nx=n, ny=n, pixel_cm=dx, n_bins=n_bins or n, bin_cm=dx, n_angles=n_angles,
             angle0_rad=0.0, e0_kev=159.0, fwhm_e_kev=15.9, fwhm_u_cm=dx, win_lo_kev=100.0,
             win_hi_kev=175.0, n_subsets=1, scatter_model=1, acq_time=1.0)
    g.update(kw)
    return g


def test_detector_line_integral_of_model():
    # L_a(p): from the centre pixel of a centred uniform disk the path to the
    # detector is close to mu * R whatever the angle
    n, dx, R, m = 64, 0.25, 6.0, 0.15
    c = (np.arange(n) - (n - 1) / 2) * dx
    X, Y = np.meshgrid(c, c)
    mu = np.where(X ** 2 + Y ** 2 <= R * R, m, 0.0)
    mod = O.OracleModel(_geom(n, dx, n_angles=12), mu, scatter=0)
    p = (n // 2) * n + n // 2          # centre (0.125, 0.125) cm
    for a in range(12):
        assert mod.L(a, p) == pytest.approx(m * R, rel=0.06)   # staircase edge: O(dx/R)
    # along +x the exact value follows from the rasterised row
    row = mu[n // 2]
    assert mod.L(0, p) == pytest.approx(row[n // 2 + 1:].sum() * dx + row[n // 2] * dx / 2, rel=1e-12)


def test_scatter_point_factor_sums_to_interaction_probability():
    # sum_s B(q,s) over a uniform disk from its centre approaches the
    # probability that an emitted photon interacts before leaving the disk,
    # 1 - exp(-mu R), less the self-pixel share (about mu * 0.561 dx)
    n, dx, R, m = 96, 0.1, 4.0, 0.3
    c = (np.arange(n) - (n - 1) / 2) * dx
    X, Y = np.meshgrid(c, c)
    mu = np.where(X ** 2 + Y ** 2 <= R * R, m, 0.0)
    mod = O.OracleModel(_geom(n, dx), mu, scatter=0)       # B computed on the fly
    q = (n // 2) * n + n // 2
    total = sum(mod.B(q, s) for s in mod.support)
    expect = 1 - math.exp(-m * R) - m * 0.561 * dx
    assert total == pytest.approx(expect, rel=0.01)


def test_memoised_pair_paths_match_direct():
    rng = np.random.default_rng(3)
    n, dx = 10, 0.6
    mu = rng.uniform(0.05, 0.3, size=(n, n)) * (rng.uniform(size=(n, n)) > 0.3)
    g = _geom(n, dx)
    m1 = O.OracleModel(g, mu, scatter=1)
    m0 = O.OracleModel(g, mu, scatter=0)
    for q in m1.support[::7]:
        for s in m1.support[::5]:
            assert m1.B(q, s) == pytest.approx(m0.B(q, s), rel=1e-14)
            assert m1.B(q, s) == pytest.approx(m1.B(s, q) * mu.flat[s] / mu.flat[q], rel=1e-12) \
                if q != s else m1.B(q, s) == 0.0


def test_line_extent_axis_aligned_matches_mask():
    """A line along x through row j of a disk mask: the extent is the outer
    boundary of that row's first and last mu > 0 pixel."""
    n, dx = 16, 0.8
    idx = (np.arange(n) - (n - 1) / 2) * dx
    X, Y = np.meshgrid(idx, idx)
    mu = np.where(X ** 2 + Y ** 2 <= (7 * dx) ** 2, 0.15, 0.0)
    for j in (0, 1, 4, 8, 15):
        u = (j - n / 2 + 0.37) * dx           # a y inside row j
        ext = O.line_extent(mu, dx, np.array([0.0, u]), np.array([1.0, 0.0]))
        cols = np.flatnonzero(mu[j] > 0)
        if cols.size == 0:
            assert ext is None
            continue
        assert ext[0] == pytest.approx((cols[0] - n / 2) * dx, abs=1e-12)
        assert ext[1] == pytest.approx((cols[-1] + 1 - n / 2) * dx, abs=1e-12)


def test_line_extent_oblique_matches_dense_sampling():
    """Random map, oblique lines: the extent agrees with the first and last
    mu > 0 hit of a dense walk along the line (to the walk's step)."""
    rng = np.random.default_rng(9)
    n, dx = 12, 0.5
    mu = np.where(rng.uniform(size=(n, n)) < 0.4, 0.2, 0.0)
    step = 2e-4
    for _ in range(6):
        th = rng.uniform(0, 2 * np.pi)
        nvec, tvec = np.array([np.cos(th), np.sin(th)]), np.array([-np.sin(th), np.cos(th)])
        foot = rng.uniform(-2.5, 2.5) * tvec
        t = np.arange(-6.0, 6.0, step)
        pts = foot[None, :] + t[:, None] * nvec[None, :]
        i = np.floor(pts[:, 0] / dx + n / 2).astype(int)
        j = np.floor(pts[:, 1] / dx + n / 2).astype(int)
        ok = (i >= 0) & (i < n) & (j >= 0) & (j < n)
        hit = np.zeros(t.size, bool)
        hit[ok] = mu[j[ok], i[ok]] > 0
        ext = O.line_extent(mu, dx, foot, nvec)
        if not hit.any():
            assert ext is None
            continue
        assert ext[0] == pytest.approx(t[hit][0], abs=2 * step)
        assert ext[1] == pytest.approx(t[hit][-1], abs=2 * step)


@pytest.mark.parametrize("a", [0, 4])
def test_column_attenuation_feature_is_response_weighted_row_integrals(a):
    """The surrogate's response-weighted attenuation input (feature 4, ck / 2)
    at an axis-aligned angle: summing mu dx k(u - u_s) pixel by pixel is the
    same as summing, over the grid rows (or columns) that face the detector,
    the line integral of mu along that row's centre line times the row's
    position response k(u - u_row).  The line integrals come from the oracle's
    Siddon routine, pinned above; the equality fails for a wrong pixel
    weight, a wrong detector axis or response."""
    n, dx = 16, 0.8
    idx = (np.arange(n) - (n - 1) / 2) * dx
    X, Y = np.meshgrid(idx, idx)
    inside = X ** 2 + Y ** 2 <= (7 * dx) ** 2
    mu = np.where(inside, 0.15 + np.where(X > 2.0, 0.1, 0.0), 0.0)   # a disk, denser on one side
    g = _geom(n, dx, n_angles=16)
    m = O.OracleModel(g, mu)
    sig = dx / (2 * math.sqrt(2 * math.log(2)))

    def k(x):
        return max(math.exp(-x * x / (2 * sig * sig)) - math.exp(-4.5), 0.0)

    th = 2 * math.pi * a / 16
    nvec = np.array([math.cos(th), math.sin(th)])
    tvec = np.array([-math.sin(th), math.cos(th)])
    far = 4 * n * dx
    for u in (-3.31, -0.4, 0.05, 1.77, 4.9):
        ref = 0.0
        for r in idx:   # the row (a = 0) or column (a = 4) centre lines facing the detector
            foot = r * tvec
            ref += O.line_integral(mu, dx, foot - far * nvec, foot + far * nvec) * k(u - r)
        pix = int(m.support[0])
        got = 2.0 * O.surrogate_features(m, pix, a, u, 140.0)[4]
        assert got == pytest.approx(ref, rel=1e-12, abs=1e-15)
    assert inside.sum() == len(m.support)

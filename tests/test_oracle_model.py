"""Pins of the oracle's assembled system model: the per-event rows h and the
sensitivities must describe the same photons, the model must reduce to the
textbook list-mode EM of Parra and Barrett when nothing attenuates, and its
scatter must agree with an independent Monte-Carlo photon simulation."""
import math

import numpy as np
import pytest

import oracle as O
import synth


def _geom(n, dx, n_angles=4, n_bins=8, **kw):
    g = dict(nx=n, ny=n, pixel_cm=dx, n_bins=n_bins, bin_cm=dx, n_angles=n_angles,
             angle0_rad=0.0, e0_kev=159.0, fwhm_e_kev=15.9, fwhm_u_cm=dx, win_lo_kev=100.0,
             win_hi_kev=175.0, n_subsets=2, scatter_model=1, acq_time=1.0)
    g.update(kw)
    return g


def test_rows_integrate_to_sensitivity():
    # sum_{a in subset} int_detector int_window h(q; a, u, E) du dE = sens_q / T
    rng = np.random.default_rng(5)
    n, dx = 6, 0.8
    mu = rng.uniform(0.1, 0.3, size=(n, n)) * (rng.uniform(size=(n, n)) > 0.25)
    g = _geom(n, dx, acq_time=2.5)
    mod = O.OracleModel(g, mu)
    step = 1.0 / 128
    ub = np.arange(0, g["n_bins"] + step / 2, step)               # exact in float32
    wu = np.full(ub.size, step * g["bin_cm"])
    wu[0] *= 0.5
    wu[-1] *= 0.5
    xg, wg = np.polynomial.legendre.leggauss(40)
    lo, hi = g["win_lo_kev"], g["win_hi_kev"]
    parts = np.linspace(lo, hi, 4)
    E = np.concatenate([0.5 * (b - a) * xg + 0.5 * (a + b) for a, b in zip(parts[:-1], parts[1:])])
    wE = np.concatenate([0.5 * (b - a) * wg for a, b in zip(parts[:-1], parts[1:])])
    E32 = E.astype(np.float32)
    for subset in (0, 1):
        total = np.zeros(len(mod.support))
        for a in range(g["n_angles"]):
            if a % g["n_subsets"] != subset:
                continue
            U, EE = np.meshgrid(ub, E32)
            W = np.outer(wE, wu)
            ev = {"angle": np.full(U.size, a, np.int32), "u_bin": U.ravel().astype(np.float32),
                  "energy": EE.ravel()}
            H = mod.system_matrix(ev)
            total += W.ravel() @ H
        sens = mod.sensitivity(subset)
        assert total * g["acq_time"] == pytest.approx(sens, rel=2e-5)


def _textbook_lm_em(ang, u_cm, n, dx, n_angles, half, sigma, n_iters, f0):
    """Plain list-mode EM with a position-only detector kernel and no
    attenuation (Parra and Barrett, IEEE TMI 17(2), 1998)."""
    c = (np.arange(n) - (n - 1) / 2) * dx
    X, Y = np.meshgrid(c, c)
    X, Y = X.ravel(), Y.ravel()

    def kern(d):
        d = np.asarray(d)
        g = np.exp(-d * d / (2 * sigma * sigma)) - math.exp(-4.5)
        return np.where(np.abs(d) < 3 * sigma, g, 0.0)

    norm = np.trapezoid(kern(np.linspace(-3 * sigma, 3 * sigma, 200001)),
                        np.linspace(-3 * sigma, 3 * sigma, 200001))
    th = 2 * np.pi * np.arange(n_angles) / n_angles
    uq = -np.sin(th)[:, None] * X[None, :] + np.cos(th)[:, None] * Y[None, :]  # [a][q]
    A = kern(u_cm[:, None] - uq[ang]) / norm
    grid = np.linspace(-half, half, 40001)
    sens = np.array([[np.trapezoid(kern(grid - uq[a, q]) / norm, grid) for q in range(n * n)]
                     for a in range(n_angles)]).sum(axis=0)
    f = f0.copy()
    for _ in range(n_iters):
        f = f * (A.T @ (1.0 / (A @ f))) / sens
    return f


def test_no_attenuation_reduces_to_textbook_list_mode_em():
    n, dx, n_angles = 8, 0.5, 6
    g = _geom(n, dx, n_angles=n_angles, n_bins=10, n_subsets=1)
    mu = np.zeros((n, n))
    act = np.zeros((n, n), np.float32)
    act[2:6, 3:7] = 1.0
    act[4, 4] = 5.0
    gg = synth.Geometry(**{k: v for k, v in g.items()})
    ev = synth.generate_events(gg, act, mu.astype(np.float32), 600, seed=123)
    assert ev["kind"].sum() == 0          # nothing to scatter off
    mod = O.OracleModel(g, mu)
    allq = np.arange(n * n, dtype=np.int32)
    H = mod.system_matrix(ev, allq)
    sens = mod.sensitivity(0, allq)[None, :]
    f0 = np.ones(n * n)
    f_or, _ = O.os_lm_mlem(H, ev["angle"], sens, 4, f0, 1)
    sig = dx / (2 * math.sqrt(2 * math.log(2)))
    half = 0.5 * g["n_bins"] * g["bin_cm"]
    f_tb = _textbook_lm_em(ev["angle"], mod.u_cm(ev["u_bin"]), n, dx, n_angles, half, sig, 4, f0)
    # the energy factor G(E; E0) is common to every row and cancels in the
    # update; the window acceptance W(E0) of the sensitivity scales f by 1/W
    w = 0.5 * (math.erf((175 - 159) / (math.sqrt(2) * 6.752108312289752))
               - math.erf((100 - 159) / (math.sqrt(2) * 6.752108312289752)))
    np.testing.assert_allclose(f_or * w, f_tb, rtol=2e-6, atol=1e-12 * f_tb.max())


@pytest.fixture(scope="module")
def brain():
    w = synth.workload("brain64")
    act, mu = synth.phantom(w)
    g = w.geom.as_dict()
    mod = O.OracleModel(g, mu)
    ev = synth.workload_events(w, n_events=400_000)
    return w, g, act, mu, mod, ev


@pytest.mark.slow
def test_scatter_fraction_agrees_with_monte_carlo(brain):
    w, g, act, mu, mod, ev = brain
    f = act.ravel()[mod.support].astype(float)
    prim = O.OracleModel(g, mu, scatter=0)
    frac = 1 - (f @ prim.sensitivity(-1)) / (f @ mod.sensitivity(-1))
    mc = ev["kind"].mean()
    assert 0.3 < mc < 0.5
    assert frac == pytest.approx(mc, rel=0.05)


@pytest.mark.slow
def test_energy_spectrum_agrees_with_monte_carlo(brain):
    w, g, act, mu, mod, ev = brain
    f = act.ravel()[mod.support].astype(float)
    angles = np.arange(0, g["n_angles"], 8)
    half = 0.5 * g["n_bins"] * g["bin_cm"]
    edges = [100, 115, 130, 143, 160, 175]
    pred = np.array([f @ mod.box_sums(angles, -half, half, lo, hi)
                     for lo, hi in zip(edges[:-1], edges[1:])])
    pred /= pred.sum()
    sel = np.isin(ev["angle"], angles)
    hist = np.histogram(ev["energy"][sel], edges)[0].astype(float)
    hist /= hist.sum()
    np.testing.assert_allclose(pred, hist, rtol=0.08, atol=0.004)


def test_position_profile_agrees_with_monte_carlo():
    # the hot ellipse sits off-centre: per angle, the share of events on each
    # half of the detector pins the direction conventions
    w = synth.workload("tiny")
    act, mu = synth.phantom(w)
    g = w.geom.as_dict()
    mod = O.OracleModel(g, mu)
    ev = synth.workload_events(w, n_events=200_000)
    f = act.ravel()[mod.support].astype(float)
    half = 0.5 * g["n_bins"] * g["bin_cm"]
    u = mod.u_cm(ev["u_bin"])
    for a in range(0, 16, 2):
        lo = f @ mod.box_sums([a], -half, 0.0, 100.0, 175.0)
        hi = f @ mod.box_sums([a], 0.0, half, 100.0, 175.0)
        sel = ev["angle"] == a
        assert lo / (lo + hi) == pytest.approx((u[sel] < 0).mean(), abs=0.015)


# ---------------------------------------------------------------------------
# The scatter path weight against the continuous single-scatter integral.
#
# On a grid whose every pixel holds the same mu (the support is a square whose
# edges are pixel edges), the line integrals are exact chords, and the
# scatter part of the per-angle sensitivity of the centre pixel is a
# point-pixel (midpoint) sum of the continuous first-order in-plane scatter
# integral (Sec. 2.2) over the square:
#   I_a = int mu e^{-mu r} / (2 pi r) * Psi(c) / Psibar
#         * exp(-rho(E'(c)) mu l_exit(s, n_a)) * D(u_s) * W(E'(c)) d^2 s,
# r = |s - q|, c = cos(angle between s - q and n_a), l_exit the chord from s
# to the square's edge along n_a; with a detector far wider than the square,
# D = 1.  Everything below is computed here from its physical definition
# (Compton relation, Klein-Nishina shape integrated by quadrature for the
# total cross-sections and the circle mean, Gaussian window acceptance), in
# polar coordinates around q by adaptive quadrature.  The point-pixel sum
# carries an O(dx) error from the 1/r point kernel next to q (the self pixel
# is excluded) plus O(dx^2): a fit I + b dx + c dx^2 through three grids of
# odd size (the centre pixel sits at the origin in each) must land on I_a.

_ME = 510.99895
_SIG_E = 15.9 / (2 * math.sqrt(2 * math.log(2)))


def _psi(e, c):
    p = 1.0 / (1.0 + (e / _ME) * (1.0 - c))
    return p * p * (p + 1.0 / p - (1.0 - c * c))


def _sigma_kn(e):
    from scipy import integrate
    return integrate.quad(lambda c: _psi(e, c), -1.0, 1.0, epsabs=0, epsrel=1e-13)[0]


def _window(ep, lo, hi):
    s = math.sqrt(2.0) * _SIG_E
    return 0.5 * (math.erf((hi - ep) / s) - math.erf((lo - ep) / s))


def _exit(x, y, dx_, dy_, h):
    t = []
    for p, d in ((x, dx_), (y, dy_)):
        if d > 1e-15:
            t.append((h - p) / d)
        elif d < -1e-15:
            t.append((-h - p) / d)
    return min(t)


def _single_scatter_integral(theta, mu, side, e0=159.0, lo=100.0, hi=175.0):
    from scipy import integrate
    h = side / 2
    nx, ny = math.cos(theta), math.sin(theta)
    s_e0 = _sigma_kn(e0)
    psibar = integrate.quad(lambda p: _psi(e0, math.cos(p)), 0, 2 * math.pi, epsabs=0, epsrel=1e-13,
                            limit=200)[0] / (2 * math.pi)

    def along(phi):
        c = math.cos(phi - theta)
        ep = e0 / (1.0 + (e0 / _ME) * (1.0 - c))
        rho = _sigma_kn(ep) / s_e0
        ex, ey = math.cos(phi), math.sin(phi)

        def f(r):
            return mu * math.exp(-mu * r) / (2 * math.pi) * math.exp(-rho * mu * _exit(r * ex, r * ey, nx, ny, h))
        radial = integrate.quad(f, 0.0, _exit(0.0, 0.0, ex, ey, h), epsabs=0, epsrel=1e-11, limit=200)[0]
        return _psi(e0, c) / psibar * _window(ep, lo, hi) * radial

    kinks = sorted({k * math.pi / 4 for k in (1, 3, 5, 7)} | {theta % (2 * math.pi), (theta + math.pi) % (2 * math.pi)})
    return integrate.quad(along, 0, 2 * math.pi, points=kinks, epsabs=0, epsrel=1e-10, limit=400)[0]


@pytest.mark.parametrize("mu,a", [(0.15, 0), (0.15, 1), (0.15, 2), (0.25, 3)])
def test_scatter_weight_matches_continuous_single_scatter_integral(mu, a):
    side, n_angles = 8.4, 16
    theta = 2 * math.pi * a / n_angles
    ref = _single_scatter_integral(theta, mu, side)
    vals = []
    for n in (7, 21, 63):
        dx = side / n
        g = _geom(n, dx, n_angles=n_angles, n_bins=4 * n, n_subsets=1)
        m1 = O.OracleModel(g, np.full((n, n), mu))
        m0 = O.OracleModel(g, np.full((n, n), mu), scatter=0)
        q = (n // 2) * n + n // 2
        vals.append((dx, m1.sens_angle(q, a) - m0.sens_angle(q, a)))
    errs = [abs(v / ref - 1) for _, v in vals]
    assert errs[0] > errs[1] > errs[2], errs            # first order in dx: about 3x per level
    assert errs[2] < 0.03
    A = np.array([[1.0, d, d * d] for d, _ in vals])
    extrap = np.linalg.solve(A, [v for _, v in vals])[0]
    assert extrap == pytest.approx(ref, rel=3e-4)
